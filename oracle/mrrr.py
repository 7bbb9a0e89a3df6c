"""Eigenvectors of T_s = tridiag(alpha, 0, alpha) by twisted factorisations.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.3 names MRRR (multiple relatively robust representations) as an
alternative to inverse iteration for the tridiagonal eigenvectors.  Its
per-vector step -- the twisted factorisation that gives an eigenvector in
O(N) without iterating -- is written here from its published definition
(Parlett and Dhillon, "Fernando's solution to Wilkinson's problem", 1997;
Dhillon and Parlett, "Multiple representations to compute orthogonal
eigenvectors of symmetric tridiagonal matrices", 2004), for T_s itself:

* top-down factorisation T_s - lam I = L+ D+ L+^T:
      d+_0 = -lam,   d+_{k+1} = -lam - alpha_k^2 / d+_k;
* bottom-up factorisation T_s - lam I = U- D- U-^T:
      d-_{N-1} = -lam,   d-_k = -lam - alpha_k^2 / d-_{k+1};
* twist gamma_k = d+_k + d-_k + lam (the diagonal entry -lam counted once),
  which equals 1 / [(T_s - lam I)^{-1}]_{kk};
* at r = argmin |gamma_k|, the vector with z_r = 1 and
      z_k = -(alpha_k / d+_k) z_{k+1}       (k < r),
      z_{k+1} = -(alpha_k / d-_{k+1}) z_k   (k >= r),
  solves (T_s - lam I) z = gamma_r e_r; it is then normalised.

Pivots smaller than pivmin in modulus are replaced by -pivmin, as in the
Sturm count of the bisection.  Where a recurrence meets z = 0, the row
equation of T_s - lam I two entries away gives the next entry (0 where that
row's coupling is exactly zero, a split of T_s).  The
representation tree of the full method (new shifted representations for
clusters of close eigenvalues) is not part of this step: a cluster's
vectors are orthogonalised by the same Gram-Schmidt as after inverse
iteration (eigenvectors_T_s_twisted).
"""

from __future__ import annotations

import numpy as np

from .bse_oracle import EPS, SAFMIN, gershgorin_bound, reorthogonalize_clusters


def _pivmin(alpha: np.ndarray) -> float:
    e2 = alpha * alpha
    return SAFMIN * max(1.0, float(np.max(e2)) if e2.size else 1.0)


def twist_factors(alpha: np.ndarray, lam: np.ndarray):
    """d+ and d- (N x m) of T_s - lam_j I for every shift lam_j, and the
    twists gamma (N x m)."""
    N = alpha.shape[0] + 1
    lam = np.asarray(lam, dtype=np.float64)
    m = lam.shape[0]
    pivmin = _pivmin(alpha)
    e2 = alpha * alpha
    fix = lambda q: np.where(np.abs(q) < pivmin, -pivmin, q)   # noqa: E731
    dp = np.zeros((N, m))
    dm = np.zeros((N, m))
    dp[0] = fix(-lam)
    for k in range(N - 1):
        dp[k + 1] = fix(-lam - e2[k] / dp[k])
    dm[N - 1] = fix(-lam)
    for k in range(N - 2, -1, -1):
        dm[k] = fix(-lam - e2[k] / dm[k + 1])
    gamma = dp + dm + lam[None, :]
    return dp, dm, gamma


def twisted_eigenvectors(alpha: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Unit eigenvectors (N x m) of T_s for the eigenvalue approximations lam,
    one twisted factorisation each."""
    N = alpha.shape[0] + 1
    m = np.asarray(lam).shape[0]
    dp, dm, gamma = twist_factors(alpha, lam)
    Z = np.zeros((N, m))
    for j in range(m):
        r = int(np.argmin(np.abs(gamma[:, j])))
        z = np.zeros(N)
        z[r] = 1.0
        for k in range(r - 1, -1, -1):
            if z[k + 1] != 0.0:
                z[k] = -(alpha[k] / dp[k, j]) * z[k + 1]
            else:   # row k+1: alpha_k z_k - lam z_{k+1} + alpha_{k+1} z_{k+2} = 0
                z[k] = -(alpha[k + 1] / alpha[k]) * z[k + 2] if alpha[k] != 0.0 else 0.0
        for k in range(r, N - 1):
            if z[k] != 0.0:
                z[k + 1] = -(alpha[k] / dm[k + 1, j]) * z[k]
            else:   # row k: alpha_{k-1} z_{k-1} - lam z_k + alpha_k z_{k+1} = 0
                z[k + 1] = -(alpha[k - 1] / alpha[k]) * z[k - 1] if alpha[k] != 0.0 else 0.0
        Z[:, j] = z / np.linalg.norm(z)
    return Z


def eigenvectors_T_s_twisted(alpha: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """V_+ (N x n): twisted factorisations, then the Gram-Schmidt of clusters
    closer than 1e-3 ||T_s|| (as after inverse iteration)."""
    Z = twisted_eigenvectors(alpha, lam)
    return reorthogonalize_clusters(Z, np.asarray(lam), 1e-3 * gershgorin_bound(alpha))


__all__ = ["twist_factors", "twisted_eigenvectors", "eigenvectors_T_s_twisted", "EPS"]
