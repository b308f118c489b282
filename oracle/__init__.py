"""FP64 CPU oracle for the two-component D3Q19 lattice Boltzmann step.

Test infrastructure only: ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
HIP library.  Modules:

* :mod:`oracle.lbm`          forward step, Sec. 2 of arXiv 1601.01237;
* :mod:`oracle.adjoint`      hand-written transpose of that step;
* :mod:`oracle.diagnostics`  global reductions (mass, momentum, Laplace
  pressure, droplet centre of mass).
"""

from . import adjoint, diagnostics, lbm  # noqa: F401
