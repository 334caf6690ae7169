"""FP64 CPU oracle for the multi-level power-series H-matrix solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under this package: only the test suite, the smoke entry point
and the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library; the only common module is ``workloads`` (seeded input arrays).

It is a plain, slow, step-by-step FP64 rendering of the method of Negi,
Balakrishnan and Rao (arXiv 2307.03968):

  entries    synthetic stand-in for the MoM system [Z] x = b       (Sec. II, eq. 5)
  cluster    binary-tree division, admissibility, block partition  (Sec. III, eq. 6-7)
  aca        ACA with partial pivoting + recompression             (Sec. III)
  hmatrix    near/far H-matrix with symmetric half computation     (Sec. III-IV, eq. 6, 8)
  series     power series per level, exact solve, rho, refinement  (Sec. IV, eq. 9-22)

Every function is pinned by tests that do not re-type its formula (see the
pin tests under tests/).  Readings of points the paper leaves open are listed
in the repository's design notes.
"""
from . import entries, cluster, aca, hmatrix, series  # noqa: F401
