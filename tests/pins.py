"""Checks that pin the oracle to facts the paper and the mathematics fix.

Each check returns (name, ok, value).  The same suite runs on the real oracle
(where every check must pass) and on oracles with a planted mistake (where at
least one must fail), so the suite is known to be sensitive to the kind of
error it guards against.
"""

from __future__ import annotations

import math

import numpy as np

from oracle import bse_oracle as bo
from oracle import metrics

EPS = np.finfo(np.float64).eps


def _Q(n):
    return metrics.Q_matrix(n)


def check_embedding(A, B):
    """Theorem 2: Q^H Omega Q = M and Q^H H Q = -i J M."""
    n = A.shape[0]
    M = bo.build_M(A, B)
    Q = _Q(n)
    om = metrics.omega_matrix(A, B)
    H = metrics.H_matrix(A, B)
    J = bo.J_matrix(n)
    e1 = np.max(np.abs(Q.conj().T @ om @ Q - M))
    e2 = np.max(np.abs(Q.conj().T @ H @ Q - (-1j) * J @ M))
    scale = np.max(np.abs(M))
    return [("embedding QOQ=M", e1 <= 50 * EPS * scale, e1),
            ("embedding QHQ=-iJM", e2 <= 50 * EPS * scale, e2)]


def check_factors(A, B):
    """Cholesky reconstructs M; W is skew with W22 = 0 (derived from the block
    form of L^T J L); W = U T U^T with U orthogonal."""
    n = A.shape[0]
    N = 2 * n
    M = bo.build_M(A, B)
    L, info = bo.cholesky(M)
    out = [("cholesky info", info == 0, info)]
    e = np.linalg.norm(L @ L.T - M) / np.linalg.norm(M)
    out.append(("cholesky LL^T=M", e <= 10 * N * EPS, e))
    out.append(("cholesky lower", np.all(np.triu(L, 1) == 0), 0))
    W = bo.form_W(L)
    ws = np.max(np.abs(W + W.T))
    out.append(("W skew", ws <= 10 * EPS * np.max(np.abs(W)), ws))
    out.append(("W22 zero", np.all(W[n:, n:] == 0), float(np.max(np.abs(W[n:, n:])))))
    alpha, vs, taus = bo.skew_tridiagonalize(W)
    U = bo.householder_matrix(vs, taus, N)
    T = bo.tridiag_T(alpha)
    e = np.linalg.norm(W - U @ T @ U.T) / max(np.linalg.norm(W), 1e-300)
    out.append(("W=UTU^T", e <= 20 * N * EPS, e))
    e = np.max(np.abs(U.T @ U - np.eye(N)))
    out.append(("U orthogonal", e <= 20 * N * EPS, e))
    # -i D^H T D = tridiag(alpha, 0, alpha) with D = diag(i^k)
    D = np.diag([1j ** (k % 4) for k in range(N)])
    e = np.max(np.abs(-1j * D.conj().T @ T @ D - bo.tridiag_T_s(alpha)))
    out.append(("D similarity", e <= 4 * EPS * np.max(np.abs(alpha)), e))
    # T_s (zero diagonal) is a perfect shuffle of [[0, G^T], [G, 0]] with G
    # upper bidiagonal, diagonal alpha[0], alpha[2], ..., superdiagonal
    # alpha[1], alpha[3], ...: its positive eigenvalues are G's singular values.
    G = np.diag(np.abs(alpha[0::2])) + np.diag(np.abs(alpha[1::2]), 1)
    sv = np.sort(np.linalg.svd(G, compute_uv=False))
    lam = bo.bisect_positive(alpha)
    e = np.max(np.abs(lam - sv)) / np.max(sv)
    out.append(("T_s eig = bidiag SVD", e <= 20 * EPS * N, e))
    return out


def check_spectrum(A, B, lam, brute=True):
    """Eigenvalues: brute force (the paper's ZGEEV comparison), +/- pairs and
    real spectrum (Theorem 1, eq. GMG), bounds lambda_min(M) <= lam <=
    lambda_max(M), the Tamm-Dancoff overestimate (Theorem 4)."""
    n = A.shape[0]
    out = []
    H = metrics.H_matrix(A, B)
    M = bo.build_M(A, B)
    normH = np.linalg.norm(H, 2)
    out.append(("ascending", bool(np.all(np.diff(lam) >= 0)), 0))
    out.append(("positive", bool(np.all(lam > 0)), float(lam.min())))
    if brute:
        ev = np.linalg.eig(H)[0]
        evr = np.sort(ev.real)
        e_pos = np.max(np.abs(evr[n:] - lam)) / normH
        e_neg = np.max(np.abs(evr[:n][::-1] + lam)) / normH
        out.append(("eig brute force", e_pos <= 1e-11, e_pos))
        out.append(("+- pairs", e_neg <= 1e-11, e_neg))
        out.append(("real spectrum", float(np.max(np.abs(ev.imag))) <= 1e-8 * normH, float(np.max(np.abs(ev.imag)))))
    em = np.linalg.eigvalsh(M)
    out.append(("lam within eig(M)", bool(lam.min() >= em[0] * (1 - 1e-12) and lam.max() <= em[-1] * (1 + 1e-12)), 0))
    a_full, _ = bo.symmetrize_lower(A, B)
    ea = np.sort(np.linalg.eigvalsh(a_full))[::-1]
    lh = np.sort(lam)[::-1]
    viol = float(np.max(lh - ea))
    out.append(("TDA overestimates", viol <= 1e-12 * normH, viol))
    return out


def check_vectors(A, B, lam, X, d=None):
    """Eigenvectors: H X = X Lambda, eq. normalization, Table 1 metrics,
    left eigenvectors Y = S X (Theorem 3), weight sum rule and phase
    invariance (eq. absp)."""
    n = A.shape[0]
    out = []
    H = metrics.H_matrix(A, B)
    r = metrics.eig_residual(A, B, lam, X)
    out.append(("HX=XL", r <= 1e-14 * max(1, n) ** 0.5 * 10, r))
    e = metrics.normalization_error(X)
    out.append(("X1^HX1-X2^HX2=I", e <= 1e-12, e))
    r1, r2 = metrics.table1_metrics(A, B, lam, X)
    out.append(("table1 YHX-L", r1 <= 1e-13, r1))
    out.append(("table1 YX-I", r2 <= 1e-13, r2))
    Y = X.copy()
    Y[n:] *= -1
    e = np.max(np.abs(Y.conj().T @ H - lam[:, None] * Y.conj().T)) / np.linalg.norm(H)
    out.append(("left eigvecs", e <= 1e-13, e))
    if d is not None:
        w = bo.absorption_weights(X, d, d)
        wa = metrics.weights_all_pairs(X, d, d)
        e = abs(np.sum(wa) - np.vdot(d, d))
        out.append(("weights sum rule", e <= 1e-12, e))
        e = np.max(np.abs(wa[:n] - w))
        out.append(("weights = first half", e <= 1e-14, e))
        rng = np.random.default_rng(7)
        ph = np.exp(1j * rng.uniform(0, 2 * math.pi, n))
        w2 = bo.absorption_weights(X * ph[None, :], d, d)
        e = np.max(np.abs(w2 - w))
        out.append(("weights phase invariant", e <= 1e-14, e))
    return out


def run_all(A, B, d, brute=True):
    """Every check for one problem; returns the list of (name, ok, value)."""
    res = bo.solve(A, B, d)
    out = []
    if res.info != 0:
        return [("solve info", False, res.info)]
    out += check_embedding(A, B)
    out += check_factors(A, B)
    out += check_spectrum(A, B, res.lam, brute=brute)
    out += check_vectors(A, B, res.lam, res.X, d)
    return out


def failures(checks):
    return [(name, val) for name, ok, val in checks if not ok]
