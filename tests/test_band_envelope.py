"""The property the GPU's banded reorthogonalisation rests on: a symmetric
positive definite matrix G whose entry (i, j) is zero whenever the sorted
eigenvalues differ by more than a tolerance (|lambda_i - lambda_j| > tol)
has a Cholesky factor with exactly the same zeros (no fill outside that
envelope).  So tiles outside the band can be skipped in the Gram product,
the Cholesky updates and the triangular solve without changing the
result."""

import numpy as np
import pytest


@pytest.mark.parametrize("n,tol", [(50, 0.05), (200, 0.02), (400, 0.01)])
def test_cholesky_keeps_the_eigenvalue_band(n, tol):
    rng = np.random.default_rng(n)
    lam = np.sort(rng.uniform(0.0, 1.0, n))
    far = np.abs(lam[:, None] - lam[None, :]) > tol
    E = rng.standard_normal((n, n)) * 1e-3
    G = np.eye(n) + (E + E.T)
    G[far] = 0.0
    L = np.linalg.cholesky(G)
    lower_far = np.tril(far, -1)
    assert np.all(L[lower_far] == 0.0)
    # and the factor is that of G
    assert np.max(np.abs(L @ L.T - G)) <= 1e-14
    # the band is what the GPU keeps: rows reach back to the first column
    # within tol, a contiguous envelope
    first = np.argmax(~far, axis=1)
    for i in range(n):
        assert np.all(~far[i, first[i]:i + 1])
