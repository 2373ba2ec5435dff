"""Plain FP64 CPU reference of the DEC geometric-multigrid path (arXiv 2508.12501).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here.  The library under
``paper_2508_12501_amd/`` never does: it shares no code, table or helper with this package,
and this package never imports it.  Both take their seeded inputs from ``workloads``.

* ``dec``        meshes, face maps, d0/d1, subdivision map M(f), Hodge stars, Laplacian.
* ``multigrid``  hierarchy, Jacobi, V-cycle, stand-alone MG, MG-PCG, FCG(1), refinement.
* ``porous``     Darcy-Boussinesq step on the DEC and its discrete adjoint.

Parity status of each function against independent pins is listed in the test suite
(``tests/test_oracle_*.py``); functions without such a pin say "parity unpinned".
"""
from . import dec, multigrid  # noqa: F401
