"""Planted mistakes in the oracle must be caught by the pins.

Each case swaps one oracle function for a copy with a plausible slip (a sign,
a transposed operand, a dropped term, a wrong index) -- on the CPU, in this
process only -- and checks that the pin suite reports at least one failure.
"""

import math

import numpy as np
import pytest

from oracle import bse_oracle as bo
from bse_inputs import gen_bse

from pins import run_all, failures


def _bad_M_sign(A, B):
    a, b = bo.symmetrize_lower(A, B)
    return np.block([[(a + b).real, (a - b).imag],
                     [(a + b).imag, (a - b).real]])          # lost minus


def _bad_M_swap(A, B):
    a, b = bo.symmetrize_lower(A, B)
    return np.block([[(a + b).real, (a + b).imag],
                     [-(a - b).imag, (a - b).real]])         # swapped Im terms


def _bad_W_transpose(L):
    n = L.shape[0] // 2
    return L @ bo.J_matrix(n) @ L.T                          # L J L^T


def _bad_tridiag_no_update(W):
    # forgets the -p v^T half of the skew update
    Wk = np.array(W, dtype=np.float64, copy=True)
    N = Wk.shape[0]
    alpha = np.zeros(N - 1)
    vs, taus = [], []
    for k in range(N - 1):
        x = Wk[k + 1:, k].copy()
        if k == N - 2:
            beta, tau, v = x[0], 0.0, np.ones(1)
        else:
            beta, tau, v = bo._larfg(x)
        alpha[k] = -beta
        vs.append(v)
        taus.append(tau)
        if k == N - 2:
            break
        Wk[k + 1:, k] = 0.0
        Wk[k + 1, k] = beta
        Wk[k, k + 1:] = 0.0
        Wk[k, k + 1] = -beta
        if tau != 0.0:
            S = Wk[k + 1:, k + 1:]
            p = tau * (S @ v)
            S += np.outer(v, p)
    return alpha, vs, np.array(taus)


def _bad_back_transform_no_scale(Phi, V, lam):
    return _orig["back_transform"](Phi, V, lam) * np.sqrt(lam)[None, :]


def _bad_back_transform_D(Phi, V, lam):
    # D = diag((-i)^k) instead of diag(i^k).  (diag(i^{k+1}) would only be a
    # global phase, which is why the range of D's index does not matter.)
    N = Phi.shape[0]
    n = N // 2
    Phi1, Phi2 = Phi[:n], Phi[n:]
    Qphi = np.vstack([Phi1 - 1j * Phi2, Phi1 + 1j * Phi2]) / math.sqrt(2.0)
    dk = np.array([(-1j) ** (k % 4) for k in range(N)])
    Y = (Qphi * dk[None, :]) @ V
    Y[n:] = -Y[n:]
    return Y / np.sqrt(lam)[None, :]


def _bad_back_transform_no_S(Phi, V, lam):
    X = _orig["back_transform"](Phi, V, lam)
    X[len(X) // 2:] *= -1
    return X


def _bad_phi_order(L, vs, taus):
    Phi = np.array(L, dtype=np.float64, copy=True)
    for k in range(len(vs) - 1, -1, -1):                    # reversed order
        if taus[k] == 0.0:
            continue
        v = vs[k]
        blk = Phi[:, k + 1:]
        blk -= taus[k] * np.outer(blk @ v, v)
    return Phi


def _bad_bisect_off_by_one(alpha, max_iter=200):
    lam = _orig["bisect_positive"](alpha, max_iter)
    out = lam.copy()
    out[:-1] = lam[1:]
    return out


def _bad_inverse_iteration_no_solve(alpha, lam, seed=12345, iters=3):
    N = alpha.shape[0] + 1
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1.0, 1.0, size=(N, lam.shape[0]))
    return b / np.linalg.norm(b, axis=0, keepdims=True)


def _bad_weights_no_S(X, d_r, d_l):
    num = (d_r.conj() @ X) * (X.conj().T @ d_l)
    den = np.einsum("ij,ij->j", X.conj(), X)
    return num / den


def _bad_cholesky_sign(M):
    L, info = _orig["cholesky"](M)
    L = L.copy()
    L[1:, 0] *= -1
    return L, info


_orig = {name: getattr(bo, name) for name in
         ["build_M", "form_W", "skew_tridiagonalize", "back_transform", "phi_LU",
          "bisect_positive", "inverse_iteration", "absorption_weights", "cholesky"]}

MUTATIONS = [
    ("build_M", _bad_M_sign),
    ("build_M", _bad_M_swap),
    ("form_W", _bad_W_transpose),
    ("skew_tridiagonalize", _bad_tridiag_no_update),
    ("back_transform", _bad_back_transform_no_scale),
    ("back_transform", _bad_back_transform_D),
    ("back_transform", _bad_back_transform_no_S),
    ("phi_LU", _bad_phi_order),
    ("bisect_positive", _bad_bisect_off_by_one),
    ("inverse_iteration", _bad_inverse_iteration_no_solve),
    ("absorption_weights", _bad_weights_no_S),
    ("cholesky", _bad_cholesky_sign),
]


@pytest.mark.parametrize("target,bad", MUTATIONS, ids=[f"{t}-{f.__name__}" for t, f in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, target, bad):
    p = gen_bse(12, seed=8)
    monkeypatch.setattr(bo, target, bad)
    try:
        checks = run_all(p.A, p.B, p.d)
        caught = bool(failures(checks))
    except Exception:
        caught = True        # a crash is also a detection
    assert caught, f"mutation {bad.__name__} of {target} passed every pin"
