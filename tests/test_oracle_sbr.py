"""Pins of the two-stage reduction oracle (oracle/sbr.py):

* stage 1 leaves a skew matrix of bandwidth b that is orthogonally similar
  to W (B = Q1^T W Q1 with the returned reflectors);
* stage 2 leaves a tridiagonal skew matrix similar to B;
* U e_1 = e_1 and W = U T U^T with U orthogonal;
* |alpha| equals the one-stage reduction's (implicit-Q argument) and the
  positive eigenvalues of T_s equal the brute-force eigenvalues of -iW;
* planted mistakes (a reflector built from the wrong column, a chase that
  skips the last block, the skew rank-2 update's sign) fail one of these.
"""

import numpy as np
import pytest

from oracle import bse_oracle as bo
from oracle import sbr


def skew(N, seed):
    g = np.random.default_rng(seed).standard_normal((N, N))
    return g - g.T


def bandwidth(A, tol):
    N = A.shape[0]
    bw = 0
    for i in range(N):
        nz = np.nonzero(np.abs(A[i, :i]) > tol)[0]
        if nz.size:
            bw = max(bw, i - int(nz.min()))
    return bw


def check_two_stage(W, b, band_fn=sbr.band_reduce, tri_fn=sbr.band_to_tridiag):
    N = W.shape[0]
    tol = 1e-12 * np.abs(W).max() * N
    out = []
    B, r1 = band_fn(W, b)
    out.append(("stage 1 bandwidth", bandwidth(B, tol) <= b, bandwidth(B, tol)))
    out.append(("stage 1 skew", np.max(np.abs(B + B.T)) <= tol, np.max(np.abs(B + B.T))))
    T, alpha, r2 = tri_fn(B, b)
    out.append(("stage 2 tridiagonal", bandwidth(T, tol) <= 1, bandwidth(T, tol)))
    U = np.eye(N)
    for r0, v, tau in r1 + r2:
        sl = slice(r0, r0 + v.shape[0])
        U[:, sl] -= tau * np.outer(U[:, sl] @ v, v)
    out.append(("U orthogonal", np.max(np.abs(U.T @ U - np.eye(N))) <= 1e-12, 0))
    out.append(("U e1 = e1", np.max(np.abs(U[:, 0] - np.eye(N)[:, 0])) == 0.0, 0))
    rec = np.max(np.abs(U @ T @ U.T - W))
    out.append(("W = U T U^T", rec <= tol, rec))
    a1 = bo.skew_tridiagonalize(W)[0]
    da = np.max(np.abs(np.abs(a1) - np.abs(alpha)))
    out.append(("|alpha| as one stage", da <= tol, da))
    lam = np.sort(np.abs(np.linalg.eigvals(W).imag))[N % 2:][::2]
    lt = np.sort(np.abs(np.linalg.eigvals(T).imag))[N % 2:][::2]
    out.append(("eigenvalues", np.max(np.abs(lam - lt)) <= tol, np.max(np.abs(lam - lt))))
    return out


@pytest.mark.parametrize("N,b", [(8, 2), (40, 4), (65, 8), (96, 16), (50, 3), (33, 32)])
def test_two_stage_pins(N, b):
    for name, ok, val in check_two_stage(skew(N, N + b), b):
        assert ok, (name, val)


def test_two_stage_on_a_bse_W():
    from bse_inputs import gen_bse
    p = gen_bse(24, s_a=0.3, s_b=0.05, seed=8)
    L = bo.cholesky(bo.build_M(p.A, p.B))[0]
    W = bo.form_W(L)
    for name, ok, val in check_two_stage(W, 8):
        assert ok, (name, val)


def _band_wrong_column(W, b):
    A = np.array(W, dtype=np.float64)
    N = A.shape[0]
    refl = []
    for k0 in range(0, N, b):
        r0 = k0 + b
        if r0 >= N - 1:
            break
        for j in range(b):
            if r0 + j >= N - 1:
                break
            _beta, tau, v = bo._larfg(A[r0 + j:, k0 + j - 1 if j else k0].copy())
            sbr._apply_two_sided(A, r0 + j, v, tau)
            refl.append((r0 + j, v, tau))
    return A, refl


def _tri_short_chase(B, b):
    A = np.array(B, dtype=np.float64)
    N = A.shape[0]
    refl = []
    for s in range(N - 2):
        col, r0 = s, s + 1
        while r0 < N - 1 - b:
            r1 = min(r0 + b - 1, N - 1)
            _beta, tau, v = bo._larfg(A[r0:r1 + 1, col].copy())
            sbr._apply_two_sided(A, r0, v, tau)
            refl.append((r0, v, tau))
            col, r0 = r0, r1 + 1
    return A, np.array([A[k + 1, k] for k in range(N - 1)]), refl


def _tri_one_sided(B, b):
    A = np.array(B, dtype=np.float64)
    N = A.shape[0]
    refl = []
    for s in range(N - 2):
        col, r0 = s, s + 1
        while r0 < N - 1:
            r1 = min(r0 + b - 1, N - 1)
            _beta, tau, v = bo._larfg(A[r0:r1 + 1, col].copy())
            sl = slice(r0, r1 + 1)
            A[sl, :] -= tau * np.outer(v, v @ A[sl, :])   # left side only
            refl.append((r0, v, tau))
            col, r0 = r0, r1 + 1
    return A, np.array([A[k + 1, k] for k in range(N - 1)]), refl


@pytest.mark.parametrize("mut", ["band", "chase", "onesided"])
def test_two_stage_mutants_fail(mut):
    W = skew(40, 7)
    kw = {"band": {"band_fn": _band_wrong_column}, "chase": {"tri_fn": _tri_short_chase},
          "onesided": {"tri_fn": _tri_one_sided}}[mut]
    assert not all(ok for _, ok, _ in check_two_stage(W, 4, **kw))
