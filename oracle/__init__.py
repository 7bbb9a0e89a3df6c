"""CPU oracle for the structure-preserving Bethe-Salpeter eigensolver.

TEST INFRASTRUCTURE ONLY.  Plain, slow, unblocked FP64 NumPy code written
from the paper (Shao, da Jornada, Yang, Deslippe, Louie, "Structure preserving
parallel algorithms for solving the Bethe-Salpeter eigenvalue problem",
arXiv:1501.03830).  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it.  It shares no code with the GPU library
and the GPU library never calls it.
"""

from .bse_oracle import (  # noqa: F401
    OracleResult,
    symmetrize_lower,
    build_M,
    cholesky,
    form_W,
    skew_tridiagonalize,
    tridiag_T_s,
    sturm_count,
    bisect_positive,
    inverse_iteration,
    reorthogonalize_clusters,
    eigenvectors_T_s,
    householder_matrix,
    phi_LU,
    back_transform,
    canonical_phase,
    absorption_weights,
    solve,
)
from .real_bse import solve_real  # noqa: F401
from . import sbr  # noqa: F401
from . import spectra  # noqa: F401
from . import metrics  # noqa: F401
from . import mrrr  # noqa: F401
