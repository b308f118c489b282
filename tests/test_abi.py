"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/lbm.h, and its velocity set is the oracle's D3Q19."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import lbm as olbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
LIB = os.path.join(ROOT, "paper_1601_01237_amd", "liblbm.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    from paper_1601_01237_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "lbm_step" in names and "lbm_adjoint_step" in names
    for name in names:
        assert hasattr(lib, name), name
    from paper_1601_01237_amd import _lib
    assert sorted(_lib.EXPORTED) == names


def test_velocity_set_matches_oracle(lib):
    from paper_1601_01237_amd import _lib
    c, w = _lib.velocity_set()
    np.testing.assert_array_equal(np.array(c), olbm.C)
    np.testing.assert_allclose(np.array(w), olbm.W, rtol=0, atol=0)


def test_status_strings(lib):
    lib.lbm_status_str.restype = ctypes.c_char_p
    assert lib.lbm_status_str(0) == b"ok"
    assert lib.lbm_status_str(-5) == b"not supported"


def test_null_arguments_are_rejected_without_a_gpu(lib):
    from paper_1601_01237_amd import _lib
    ctx = ctypes.c_void_p()
    p = _lib.Params()
    # null buffers -> invalid argument, checked before any HIP call
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), None, None, None, None, None) == -1
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_step_fields(None, None) == -1
    assert lib.lbm_adjoint_step_fields(None, None, None, None, None, None, 0, None, None) == -1
    assert lib.lbm_moments(None, None, None, None, None) == -1
    assert lib.lbm_destroy(None) == 0
    assert lib.lbm_time(None) == -1


def test_parameter_checks_without_a_gpu(lib):
    from paper_1601_01237_amd import _lib
    ctx = ctypes.c_void_p()
    p = _lib.Params()
    p.nx, p.ny, p.nz = 4, 4, 4
    p.tau[0], p.tau[1] = 1.0, 1.0
    dummy_a, dummy_b, dummy_r = ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(48)
    # G^{AA} != 0 is outside the model of the paper (Sec. 2): not supported
    p.G[0][0] = 0.5
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), dummy_a, dummy_b, None, dummy_r, None) == -5
    p.G[0][0] = 0.0
    # tau <= 1/2 is invalid (negative viscosity)
    p.tau[1] = 0.5
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), dummy_a, dummy_b, None, dummy_r, None) == -1
    p.tau[1] = 1.0
    p.storage = 7
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), dummy_a, dummy_b, None, dummy_r, None) == -1
    p.storage = 0
    p.nx = 0
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), dummy_a, dummy_b, None, dummy_r, None) == -1
    p.nx = 4
    # same buffer twice
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), dummy_a, dummy_a, None, dummy_r, None) == -1
    # population arrays beyond 32-bit offsets are refused
    p.nx, p.ny, p.nz = 2048, 1024, 1024
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), dummy_a, dummy_b, None, dummy_r, None) == -5


def _layout(nx, ny, es):
    """(rows per block B, population stride S, z-plane elements Z) of the
    row-blocked state layout: B = min(4, ny) rows for FP32 and ny for the
    16-bit forms; B*nx elements rounded up to 256 bytes, plus 256 bytes when
    that is a multiple of 64 KiB; 38 S per block, ceil(ny / B) blocks."""
    b = min(4, ny) if es == 4 else ny
    nbytes = b * nx * es
    padded = -(-nbytes // 256) * 256
    if padded % 65536 == 0:
        padded += 256
    s = padded // es
    rows = 38 if es == 4 else 40  # the 16-bit forms add the two rest-population residual rows
    return b, s, rows * s * -(-ny // b)


def test_plane_stride_and_state_size(lib):
    from paper_1601_01237_amd import _lib
    for nx, ny, st, es in [(128, 128, _lib.FP32, 4), (128, 128, _lib.FP16, 2), (96, 96, _lib.FP32, 4),
                           (70, 19, _lib.BF16, 2), (512, 512, _lib.FP32, 4), (1, 1, _lib.FP32, 4),
                           (32, 30, _lib.FP32, 4), (384, 192, _lib.FP32, 4), (256, 256, _lib.BF16, 2),
                           (130, 9, _lib.FP32, 4), (40, 2, _lib.FP32, 4), (4096, 4, _lib.FP32, 4)]:
        b, want, z = _layout(nx, ny, es)
        assert lib.lbm_row_block(nx, ny, st) == b, (nx, ny, st)
        got = lib.lbm_plane_stride(nx, ny, st)
        assert got == want, (nx, ny, st, got, want)
        assert got >= b * nx and (got * es) % 65536 != 0
        assert lib.lbm_state_elems(nx, ny, 7, st) == 7 * z
    assert lib.lbm_plane_stride(0, 4, _lib.FP32) == -1
    assert lib.lbm_plane_stride(4, 4, 3) == -1
    assert lib.lbm_row_block(4, 0, _lib.FP32) == -1
    assert lib.lbm_state_elems(4, 4, 0, _lib.FP32) == -1


def test_row_fold_query(lib):
    """16-bit rows of even length without walls are folded (h = nx/2); FP32
    rows, odd nx and contexts with walls are not."""
    from paper_1601_01237_amd import _lib
    for nx, st, walls, want in [(64, _lib.FP16, 0, 32), (70, _lib.BF16, 0, 35), (2, _lib.FP16, 0, 1),
                                (7, _lib.FP16, 0, 0), (64, _lib.FP32, 0, 0), (1, _lib.BF16, 0, 0),
                                (64, _lib.FP16, 1, 0), (70, _lib.BF16, 1, 0)]:
        assert lib.lbm_row_half(nx, st, walls) == want, (nx, st, walls)
    assert lib.lbm_row_half(0, _lib.FP16, 0) == -1
    assert lib.lbm_row_half(8, 3, 0) == -1


def _valid_params(_lib):
    p = _lib.Params()
    p.nx, p.ny, p.nz = 8, 8, 8
    p.storage = _lib.FP32
    p.tau[0], p.tau[1] = 1.0, 1.0
    p.G[0][1] = p.G[1][0] = -1.0
    p.collision = _lib.BGK
    return p


@pytest.mark.parametrize("field,value,status", [
    ("tau", (0.5, 1.0), -1),            # tau must exceed 1/2 (Eq. 2)
    ("tau", (1.0, float("nan")), -1),
    ("G", ((0.5, -1.0), (-1.0, 0.0)), -5),   # self-interaction G^{aa} != 0 (Sec. 2)
    ("storage", 3, -1),
    ("collision", 3, -1),
    ("nx", 0, -1),
    ("rho_wall", (float("inf"), 0.0), -1),
])
def test_invalid_parameters_are_rejected_before_any_device_call(lib, field, value, status):
    """lbm_init validates its parameters synchronously, before it allocates or
    launches anything; the dummy device pointers are never touched."""
    from paper_1601_01237_amd import _lib
    p = _valid_params(_lib)
    if field in ("tau", "rho_wall"):
        getattr(p, field)[0], getattr(p, field)[1] = value
    elif field == "G":
        for a in range(2):
            for b in range(2):
                p.G[a][b] = value[a][b]
    else:
        setattr(p, field, value)
    ctx = ctypes.c_void_p()
    dummy_a, dummy_b, dummy_rho = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), dummy_a, dummy_b, None, dummy_rho, None) == status
    assert ctx.value is None


# (nx, ny, nz, storage, supported): one z plane of the state below 2 GiB,
# N < 2^31 cells and N * element size < 4 GiB.
SIZE_CASES = [
    (4096, 3424, 4, 0, True),     # 856 row blocks of 38 * 65,792 B = 2.140e9 B per z plane
    (4096, 3440, 4, 0, False),    # 860 blocks: 2.150e9 >= 2^31
    (4096, 6552, 4, 1, True),     # 40 rows (38 + 2 residual) of 53.7 MB = 2.147e9 B
    (4096, 6560, 4, 2, False),
    (1024, 1024, 1023, 0, True),  # N * 4 just below 4 GiB
    (1024, 1024, 1024, 0, False),
    (1024, 1024, 2047, 1, True),  # N just below 2^31
    (1024, 1024, 2048, 1, False),
]


@pytest.mark.parametrize("nx,ny,nz,storage,ok", SIZE_CASES)
def test_size_limits_agree_with_init(lib, nx, ny, nz, storage, ok):
    """lbm_state_elems is -1 exactly where lbm_init answers LBM_ENOTSUP for
    the size; the check comes before any device call."""
    from paper_1601_01237_amd import _lib
    es = 4 if storage == _lib.FP32 else 2
    stride = lib.lbm_plane_stride(nx, ny, storage)
    elems = lib.lbm_state_elems(nx, ny, nz, storage)
    if ok:
        b, s, z = _layout(nx, ny, es)
        assert stride == s and z * es < 2 ** 31
        assert elems == nz * z
    else:
        assert elems == -1
    p = _valid_params(_lib)
    p.nx, p.ny, p.nz, p.storage = nx, ny, nz, storage
    ctx = ctypes.c_void_p()
    if not ok:
        # Only an unsupported size may reach the library here: a supported
        # one would go on to launch on the dummy pointers.
        rc = lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                          None, ctypes.c_void_p(0x3000), None)
        assert rc == -5 and ctx.value is None


def test_status_of_calls_on_a_null_context(lib):
    assert lib.lbm_set_tiling(None, -1, 0) == -1
    assert lib.lbm_set_placement(None, 0, -1) == -1
    assert lib.lbm_wall_classes(None) == -1
    assert lib.lbm_moments(None, None, None, None, None) == -1
    assert lib.lbm_adjoint_seed(None, None, None) == -1
    assert lib.lbm_destroy(None) == 0
