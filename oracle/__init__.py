"""FP64 CPU reference ("oracle") of the discrete X-ray transform and its adjoint.

TEST INFRASTRUCTURE ONLY: tests/, __graft_entry__.smoke() and bench.py's CPU-baseline
leg are the only users.  Nothing here imports the HIP path, and the HIP path never
imports, links or executes anything in this package.

* geometry.py -- scan -> rays by the paper's transforms (Secs. 2.2, 3.2)
* xrt_oracle.c / core.py -- chord-partition forward, adjoint, hit lists (FP64, OpenMP)
* brute.py -- per-unit brute-force clipping for tiny grids
* solvers.py -- textbook CGLS in FP64
"""
from . import geometry, core, brute  # noqa: F401
