"""The CPU oracle against what the paper and the mathematics fix.

Nothing here calls the GPU library.  Sizes are small so the suite runs in
seconds; the closed-form and library special cases pin every step of the
oracle independently of its own code.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import bse_oracle as bo
from oracle import metrics
from bse_inputs import (gen_bse, gen_closed_form, gen_b_zero, gen_real,
                        gen_not_definite, omega_is_positive_definite)

from pins import run_all, failures, check_factors, check_spectrum, check_vectors

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (3, 3), (8, 4), (17, 5), (32, 6), (64, 1)])
def test_all_pins_generic(n, seed):
    p = gen_bse(n, seed=seed)
    bad = failures(run_all(p.A, p.B, p.d))
    assert not bad, bad


@pytest.mark.parametrize("n,s_a", [(48, 0.3), (96, 0.1)])
def test_all_pins_denser_kernel(n, s_a):
    p = gen_bse(n, s_a=s_a, s_b=0.05, seed=11)
    bad = failures(run_all(p.A, p.B, p.d))
    assert not bad, bad


@pytest.mark.parametrize("n", [1, 5, 16, 64, 150])
def test_closed_form_eigenvalues(n):
    p = gen_closed_form(n, seed=30 + n)
    r = oracle.solve(p.A, p.B, p.d)
    assert r.info == 0
    normH = np.linalg.norm(metrics.H_matrix(p.A, p.B), 2)
    err = np.max(np.abs(r.lam - p.exact_lambda)) / normH
    assert err <= 1e-13, err


def test_closed_form_eigenvectors():
    # For the closed-form generator the eigenvector of lambda_k is
    # [U0 e_k p_k; conj(U0) e_k q_k] with (p_k, q_k) the +lambda eigenvector of
    # the 2x2 block; check that the oracle's vectors span the same lines.
    n = 12
    p = gen_closed_form(n, seed=3)
    r = oracle.solve(p.A, p.B, p.d)
    H = metrics.H_matrix(p.A, p.B)
    for j in range(n):
        v = r.X[:, j]
        res = np.linalg.norm(H @ v - r.lam[j] * v) / np.linalg.norm(v)
        assert res <= 1e-13 * np.linalg.norm(H)


def test_kron_closed_form_generator():
    # The large-n closed-form path (Kronecker unitary) produces the same
    # decoupled structure; check its eigenvalues against the oracle at n=64.
    p = gen_closed_form(64, seed=9, kron_above=16)
    r = oracle.solve(p.A, p.B, p.d)
    assert np.max(np.abs(r.lam - p.exact_lambda)) <= 1e-12


@pytest.mark.parametrize("n", [4, 33, 64])
def test_b_zero_gives_eig_of_A(n):
    p = gen_b_zero(n, seed=n)
    r = oracle.solve(p.A, p.B, p.d)
    ea = np.linalg.eigvalsh(p.A)
    assert np.max(np.abs(r.lam - ea)) <= 1e-13 * np.max(np.abs(ea))


@pytest.mark.parametrize("n", [3, 20, 64])
def test_real_case_matches_algorithm2(n):
    # Theorem 5 / Algorithm 2 (SVD of L2^T L1) solves the real case by a
    # different route; the complex oracle must agree with it.
    p = gen_real(n, seed=n)
    r = oracle.solve(p.A, p.B, p.d)
    lr, Xr, info = oracle.solve_real(p.A, p.B)
    assert info == 0
    assert np.max(np.abs(r.lam - lr)) <= 1e-13 * lr.max()
    assert metrics.compare_eigvecs(r.X, Xr.astype(complex), r.lam, 1e-8) <= 1e-10
    # Algorithm 2's own guarantees
    H = metrics.H_matrix(p.A, p.B).real
    assert np.max(np.abs(H @ Xr - Xr * lr[None, :])) <= 1e-12
    X1, X2 = Xr[:n], Xr[n:]
    assert np.max(np.abs(X1.T @ X1 - X2.T @ X2 - np.eye(n))) <= 1e-12


@pytest.mark.parametrize("n,k", [(6, 0), (6, 3), (10, 9), (9, 4)])
def test_not_definite_info(n, k):
    # Omega is indefinite exactly through index k.  M's first n pivots are
    # u_j + Re b_j; the Schur complement at column n+k is
    # (u_k^2 - |b_k|^2)/(u_k + Re b_k) (derived from the 2x2 block of M).
    p = gen_not_definite(n, k, seed=k)
    assert not omega_is_positive_definite(p.A, p.B)
    u = np.diag(p.A).real
    b = np.diag(p.B)
    expect = k + 1 if u[k] + b[k].real <= 0 else n + k + 1
    _, info = bo.cholesky(bo.build_M(p.A, p.B))
    assert info == expect
    assert oracle.solve(p.A, p.B).info == expect


def test_sturm_count_brute_force():
    rng = np.random.default_rng(3)
    for N in [2, 3, 7, 20]:
        alpha = rng.standard_normal(N - 1)
        ev = np.linalg.eigvalsh(bo.tridiag_T_s(alpha))
        xs = np.concatenate([ev + 1e-7, ev - 1e-7, rng.uniform(-4, 4, 10)])
        cnt = bo.sturm_count(alpha, xs)
        want = np.array([np.sum(ev < x) for x in xs])
        assert np.array_equal(cnt, want)


def test_bisection_matches_library():
    rng = np.random.default_rng(5)
    for N in [2, 4, 10, 64, 200]:
        alpha = rng.uniform(0.1, 3.0, N - 1) * rng.choice([-1, 1], N - 1)
        lam = bo.bisect_positive(alpha)
        ev = np.linalg.eigvalsh(bo.tridiag_T_s(alpha))[N // 2:]
        # both are backward stable: |error| <= p(N) eps ||T_s||
        assert np.max(np.abs(lam - ev)) <= 2 * N * EPS * bo.gershgorin_bound(alpha)


def test_bisection_clement_closed_form():
    """The Clement matrix (zero diagonal, off-diagonals sqrt(k (N - k))) has
    the eigenvalues N - 1, N - 3, ..., -(N - 1): the positive half from
    bisection, and the inverse-iteration vectors of this equally spaced,
    chained spectrum, against the closed form."""
    for N in [2, 8, 64, 256]:
        k = np.arange(1, N, dtype=np.float64)
        alpha = np.sqrt(k * (N - k))
        lam = bo.bisect_positive(alpha)
        exact = np.arange(1, N, 2, dtype=np.float64)
        assert np.max(np.abs(lam - exact)) <= 4 * EPS * N
    V = bo.inverse_iteration(alpha, lam)
    Ts = bo.tridiag_T_s(alpha)
    assert np.max(np.abs(Ts @ V - V * lam[None, :])) <= 1e-12 * N


def test_inverse_iteration_far_pairs_orthogonal():
    """Inverse iteration alone (no reorthogonalisation) leaves eigenvectors
    whose eigenvalues are farther apart than 0.01 ||T_s||_1 orthogonal to
    far below 1e-13: the measured basis for leaving such pairs out of the
    GPU's cluster reorthogonalisation (inner products scale like
    eps ||T_s|| / |lambda_i - lambda_j|)."""
    cases = []
    p = gen_bse(384, s_a=0.3, s_b=0.05, seed=3)
    Lo, _ = bo.cholesky(bo.build_M(p.A, p.B))
    ao, _, _ = bo.skew_tridiagonalize(bo.form_W(Lo))
    cases.append(ao)
    N = 1024
    k = np.arange(1, N, dtype=np.float64)
    cases.append(np.sqrt(k * (N - k)))
    for alpha in cases:
        lam = bo.bisect_positive(alpha)
        tn = bo.gershgorin_bound(alpha)
        V = bo.inverse_iteration(alpha, lam)
        G = np.abs(V.T @ V - np.eye(lam.shape[0]))
        far = np.abs(lam[:, None] - lam[None, :]) > 0.01 * tn
        assert np.max(G[far]) <= 2e-14


def test_inverse_iteration_split_degenerate():
    # alpha with zeros splits T_s into identical blocks: eigenvalues are exactly
    # repeated and the reorthogonalised vectors must still be an orthonormal
    # eigenbasis.
    blk = np.array([1.0, 0.7, 2.0])
    alpha = np.concatenate([blk, [0.0], blk, [0.0], blk[:3]])[:11]
    N = alpha.shape[0] + 1
    lam = bo.bisect_positive(alpha)
    V = bo.eigenvectors_T_s(alpha, lam)
    Ts = bo.tridiag_T_s(alpha)
    assert np.max(np.abs(Ts @ V - V * lam[None, :])) <= 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(N // 2))) <= 1e-13


def test_inverse_iteration_residual_and_orthogonality():
    p = gen_bse(64, seed=1)
    r = oracle.solve(p.A, p.B, keep=True)
    Ts = bo.tridiag_T_s(r.alpha)
    V = r.V
    assert np.max(np.abs(Ts @ V - V * r.lam[None, :])) <= 1e-13 * np.max(np.abs(r.alpha))
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) <= 1e-13


def test_reorthogonalization_is_gram_schmidt():
    rng = np.random.default_rng(0)
    V = rng.standard_normal((10, 4))
    lam = np.array([1.0, 1.0 + 1e-9, 2.0, 2.0 + 1e-9])
    out = bo.reorthogonalize_clusters(V, lam, 1e-6)
    Q1, _ = np.linalg.qr(V[:, :2])
    Q2, _ = np.linalg.qr(V[:, 2:])
    ref = np.hstack([Q1, Q2])
    ref *= np.sign(np.sum(ref * V, axis=0))[None, :]
    assert np.max(np.abs(out - ref)) <= 1e-13


def test_residual_certificate_bounds_distance():
    p = gen_bse(24, seed=2)
    r = oracle.solve(p.A, p.B)
    M = bo.build_M(p.A, p.B)
    rng = np.random.default_rng(1)
    for j in [0, 7, 23]:
        c = metrics.residual_certificate(p.A, p.B, r.lam[j], r.X[:, j], M)
        assert c <= 1e-13
        # perturbed pair: the certificate must still bound the true distance
        x = r.X[:, j] + 1e-3 * (rng.standard_normal(48) + 1j * rng.standard_normal(48))
        lt = r.lam[j] + 2e-4
        c = metrics.residual_certificate(p.A, p.B, lt, x, M)
        assert c >= np.min(np.abs(r.lam - lt)) * (1 - 1e-9)


def test_canonical_phase():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((6, 3)) + 1j * rng.standard_normal((6, 3))
    Y = bo.canonical_phase(X)
    for j in range(3):
        i = np.argmax(np.abs(Y[:, j]))
        assert abs(Y[i, j].imag) <= 1e-15 and Y[i, j].real > 0
        assert np.allclose(np.abs(Y[:, j]), np.abs(X[:, j]))


def test_weights_sum_rule_complex_dipoles():
    p = gen_bse(16, seed=4)
    r = oracle.solve(p.A, p.B)
    rng = np.random.default_rng(2)
    dr = rng.standard_normal(32) + 1j * rng.standard_normal(32)
    dl = rng.standard_normal(32) + 1j * rng.standard_normal(32)
    wa = metrics.weights_all_pairs(r.X, dr, dl)
    assert abs(np.sum(wa) - np.vdot(dr, dl)) <= 1e-12 * np.linalg.norm(dr) * np.linalg.norm(dl)


def test_eigvec_comparison_is_basis_invariant():
    p = gen_bse(10, seed=3)
    r = oracle.solve(p.A, p.B)
    rng = np.random.default_rng(0)
    ph = np.exp(1j * rng.uniform(0, 6.28, 10))
    assert metrics.compare_eigvecs(r.X, r.X * ph[None, :], r.lam, 1e-9) <= 1e-14
    Xs = r.X.copy()
    Xs[:, 3] = r.X[:, 4]
    assert metrics.compare_eigvecs(r.X, Xs, r.lam, 1e-9) > 0.5


def test_closed_form_planted_pairs():
    # near-degenerate pairs of relative gap 1e-9, 1e-8, 1e-7 and an exact one:
    # the oracle resolves every eigenvalue to the exact closed form
    n = 40
    p = gen_closed_form(n, seed=8, planted=[(3, 1e-9), (10, 1e-8), (20, 1e-7), (30, 0.0)])
    r = oracle.solve(p.A, p.B, p.d)
    assert r.info == 0
    err = np.max(np.abs(r.lam - p.exact_lambda)) / np.max(p.exact_lambda)
    assert err <= 1e-13, err
    d = np.diff(np.sort(p.exact_lambda))
    assert np.min(d) == 0.0 or np.min(d) <= 1e-15 * np.max(p.exact_lambda)


def test_weight_comparison_rejects_wrong_weights():
    """compare_weights does not see the basis chosen inside a cluster, but
    it does see a changed cluster sum.  An exactly degenerate pair (closed
    form, planted gap 0) rotated by a unitary inside its eigenspace keeps
    Y^H X = I and every cluster sum: it passes while its per-vector weights
    change.  A 1e-6 relative change of one weight, and weight moved between
    two different clusters, fail."""
    n = 10
    p = gen_closed_form(n, seed=5, planted=[(2, 0.0)])
    r = oracle.solve(p.A, p.B, p.d)
    lam = r.lam
    j = int(np.argmin(np.diff(lam)))
    assert lam[j + 1] - lam[j] <= 1e-12 * lam[-1]
    gap = 1e-9 * lam[-1]
    assert metrics.compare_weights(r.w, r.w, lam, gap) == 0.0
    th, ph = 0.7, 1.1
    U = np.array([[math.cos(th), -np.exp(1j * ph) * math.sin(th)],
                  [np.exp(-1j * ph) * math.sin(th), math.cos(th)]])
    Xr = r.X.copy()
    Xr[:, j:j + 2] = r.X[:, j:j + 2] @ U
    assert metrics.normalization_error(Xr) <= 1e-12
    wr = metrics.weights_all_pairs(Xr, p.d, p.d)[:n]
    assert np.max(np.abs(wr - r.w)) > 1e-3 * np.max(np.abs(r.w))
    assert metrics.compare_weights(r.w, wr, lam, gap) <= 1e-13
    # moving weight inside the cluster is invisible, across clusters it is not
    w_in = r.w.copy()
    w_in[j] += 0.1
    w_in[j + 1] -= 0.1
    assert metrics.compare_weights(r.w, w_in, lam, gap) <= 1e-15
    k = 0 if j > 1 else n - 2
    w_out = r.w.copy()
    w_out[k] += 0.1 * abs(r.w[k])
    w_out[k + 1] -= 0.1 * abs(r.w[k])
    assert metrics.compare_weights(r.w, w_out, lam, gap) > 1e-4 * abs(r.w[k])
    # a 1e-6 relative change of a single weight fails a 1e-10 tolerance
    big = int(np.argmax(np.abs(r.w)))
    w_one = r.w.copy()
    w_one[big] *= 1.0 + 1e-6
    assert metrics.compare_weights(r.w, w_one, lam, gap) > 1e-10
