"""Real Bethe-Salpeter problems (bse_solve_real, Algorithm 2) against the
oracle of Algorithm 2 (oracle/real_bse.py: two Cholesky factorisations and a
LAPACK SVD of L2^T L1, an independent route) and against the complex path
on the same inputs, through the C ABI.

Tolerances as the complex parity tests: eigenvalues 1e-13 lambda_max,
eigenvectors basis-invariant 1e-9, X1^T X1 - X2^T X2 = I and H X = X Lambda
to 1e-12.  On the same matrices the real path builds the same M as the
complex path, so its eigenvalues are bit for bit the complex path's.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import metrics
from bse_inputs import gen_real, gen_real_closed_form

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def tt(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def npc(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    from paper_1501_03830_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def check_real_result(p, lam, X, tag):
    n = p.A.shape[0]
    a = np.real(p.A)
    b = np.real(p.B)
    a = np.tril(a) + np.tril(a, -1).T
    b = np.tril(b) + np.tril(b, -1).T
    H = np.block([[a, b], [-b, -a]])
    lmax = float(lam.max())
    res = float(np.max(np.abs(H @ X - X * lam[None, :]))) / lmax
    G = X[:n].T @ X[:n] - X[n:].T @ X[n:]
    nerr = float(np.max(np.abs(G - np.eye(n))))
    say(f"  {tag}: residual {res:.2e} normalisation {nerr:.2e}")
    assert res <= 1e-12 and nerr <= 1e-12


@pytest.mark.parametrize("n", [1, 2, 17, 64, 129, 300])
def test_real_matches_algorithm2_oracle(ctx, n):
    p = gen_real(n, seed=700 + n)
    say(f"[real] n={n}")
    r = ctx.solve_real(tt(p.A.real), tt(p.B.real), d_r=tt(p.d))
    assert r["info"] == 0
    lam, X, w = npc(r["lam"]), npc(r["X"]), npc(r["w"])
    assert X.dtype == np.float64
    lo, Xo, info = oracle.solve_real(p.A, p.B)
    assert info == 0
    normH = float(lo.max())
    el = float(np.max(np.abs(lam - lo))) / normH
    ev = metrics.compare_eigvecs(Xo.astype(np.complex128), X.astype(np.complex128), lo, 1e-6 * normH)
    wo = oracle.absorption_weights(Xo.astype(np.complex128), p.d, p.d)
    we = metrics.compare_weights(wo, w, lo, 1e-6 * normH)
    say(f"  eig {el:.2e} vec {ev:.2e} w {we:.2e}")
    assert el <= 1e-13 and ev <= 1e-9 and we <= 1e-10
    check_real_result(p, lam, X, "real path")
    # the complex path on the same (real) matrices
    c = ctx.solve(tt(p.A), tt(p.B))
    assert torch.equal(c["lam"], r["lam"])
    Xc = npc(c["X"])
    assert float(np.max(np.abs(Xc.imag))) <= 1e-12
    assert metrics.compare_eigvecs(Xc, X.astype(np.complex128), lam, 1e-6 * normH) <= 1e-9


@pytest.mark.parametrize("n", [40, 200])
def test_real_degenerate_eigenvalues_give_real_basis(ctx, n):
    """Exactly repeated eigenvalues (a double and a triple) in the real
    closed form: the returned basis of each eigenspace is real, satisfies
    H X = X Lambda and X1^T X1 - X2^T X2 = I, and the eigenvalues are exact."""
    p = gen_real_closed_form(n, seed=41, planted=[(3, 0.0), (10, 0.0), (11, 0.0)])
    r = ctx.solve_real(tt(p.A.real), tt(p.B.real), d_r=tt(p.d))
    assert r["info"] == 0
    lam, X = npc(r["lam"]), npc(r["X"])
    exact = np.asarray(p.exact_lambda)
    el = float(np.max(np.abs(lam - exact))) / float(exact.max())
    say(f"[real degenerate] n={n}: eig {el:.2e}")
    assert el <= 1e-13
    check_real_result(p, lam, X, "degenerate")


def test_real_not_definite_minor(ctx):
    """b_k = +2 u_k makes A - B fail at minor k + 1 (info n + k + 1), b_k = -2 u_k
    makes A + B fail there (info k + 1)."""
    n = 30
    u = np.random.default_rng(2).uniform(2.0, 5.0, size=n)
    for k, sign, want in ((7, 1.0, n + 8), (19, -1.0, 20)):
        b = np.zeros(n)
        b[k] = sign * 2.0 * u[k]
        r = ctx.solve_real(tt(np.diag(u)), tt(np.diag(b)), vectors=False)
        assert r["info"] == want
