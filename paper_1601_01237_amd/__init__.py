"""MI355X-native two-component D3Q19 Shan-Chen lattice Boltzmann step.

The compute path is the HIP library ``liblbm.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/lbm.h``.  Python modules:

* :mod:`._lib`      ctypes binding of the C ABI (argument marshalling only);
* :mod:`.sim`       ``Sim``: device buffers in torch tensors, stepping, moments;
* :mod:`.autograd`  ``LBMFunction``: checkpointed adjoint behind autograd;
* :mod:`.inputs`    seeded synthetic initial fields (no lattice arithmetic);
* :mod:`.fits`      host-side least-squares fits of reduced diagnostics.

Submodules are imported lazily so that importing :mod:`.inputs` never loads
the shared library.
"""

__all__ = ["inputs", "fits"]
