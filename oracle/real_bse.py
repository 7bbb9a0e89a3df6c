"""Oracle of Algorithm 2 (real Bethe-Salpeter problem, Theorem 5).

TEST INFRASTRUCTURE ONLY.

For real symmetric A, B with A + B > 0 and A - B > 0 (eq. H-real and the
condition that follows it): A + B = L1 L1^T, A - B = L2 L2^T, and the SVD
L2^T L1 = U Lambda_+ V^T gives the positive eigenvalues Lambda_+ and
    X1 = (1/2)(L2 U + L1 V) Lambda_+^{-1/2},  X2 = (1/2)(L2 U - L1 V) Lambda_+^{-1/2}.
Reading: Algorithm 2 step 3 omits the factor 1/2 and Lambda_+^{-1/2} that
Theorem 5 carries; they are kept here, since they are what makes
X1^T X1 - X2^T X2 = I hold.  The SVD is LAPACK's (numpy), used as one step.
"""

from __future__ import annotations

import numpy as np

from .bse_oracle import cholesky, canonical_phase


def solve_real(A: np.ndarray, B: np.ndarray):
    """Returns (lam ascending, X = [X1; X2] (2n, n) real, info)."""
    a = np.tril(np.real(A)) + np.tril(np.real(A), -1).T
    b = np.tril(np.real(B)) + np.tril(np.real(B), -1).T
    n = a.shape[0]
    L1, info1 = cholesky(a + b)
    if info1:
        return np.zeros(0), np.zeros((2 * n, 0)), info1
    L2, info2 = cholesky(a - b)
    if info2:
        return np.zeros(0), np.zeros((2 * n, 0)), n + info2
    U, s, Vt = np.linalg.svd(L2.T @ L1)
    order = np.argsort(s)
    s = s[order]
    U = U[:, order]
    V = Vt.T[:, order]
    scale = 1.0 / np.sqrt(s)
    X1 = 0.5 * (L2 @ U + L1 @ V) * scale[None, :]
    X2 = 0.5 * (L2 @ U - L1 @ V) * scale[None, :]
    X = np.vstack([X1, X2])
    return s, np.real(canonical_phase(X.astype(np.complex128))), 0
