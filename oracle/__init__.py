"""Plain FP64 CPU oracle of the spatiotemporal two-level thermal method.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it; the GPU
library neither imports nor links anything from here, and this package uses
no code of the GPU library (the two share only the plain input records of
the `workloads` module).

Every function cites the passage of the paper (arXiv 2110.12932) it
follows.  Where the paper is silent or garbled, the reading adopted is
stated at the point of use:
  * material.py  -- Section 2 (thermal model, material model)
  * grid.py      -- Q1 hexahedral discretisation of the heat operator
  * laser.py     -- Section 5.2 (laser source, scan path)
  * level.py     -- one implicit step of one level (backward Euler)
  * twolevel.py  -- Sections 3-4 (two-level coupling, Algorithm 1)

Parity status: every function here is pinned by a CPU test against a
closed form, an invariant, a special case the paper states, or brute
force (see tests/test_oracle_*.py); none is "parity unpinned".
"""
from . import material, grid, laser, level, twolevel  # noqa: F401
from .twolevel import TwoLevel, run, single_level_run  # noqa: F401
