"""Pins of the twisted-factorisation eigenvector oracle (oracle/mrrr.py).

* The twist gamma_k of T_s - x I equals 1 / [(T_s - x I)^{-1}]_{kk}, from a
  dense inverse (a closed form of twisted factorisations).
* The vectors equal numpy.linalg.eigh's eigenvectors of the dense T_s up to
  sign, for spectra without close eigenvalues.
* Golub-Kahan structure (derived): with C the upper bidiagonal matrix with
  diagonal alpha_0, alpha_2, ... and superdiagonal alpha_1, alpha_3, ..., the
  eigenvector of T_s for +sigma_k interleaves the right and left singular
  vectors of C, [v_k(0), u_k(0), v_k(1), u_k(1), ...] / sqrt(2)
  (numpy.linalg.svd).
* Residuals ||T_s z - lam z|| within a few N eps ||T_s||.
* Planted mistakes (the bottom-up pivots used on both sides, a lost sign in
  the upward recurrence, the twist without its diagonal term, an index slip
  in the downward recurrence) each fail one of these.
"""

import numpy as np
import pytest

from oracle import bse_oracle as bo
from oracle import mrrr


def well_separated(N, seed, rel=1e-2):
    """alpha whose T_s has every gap above rel ||T_s|| (rel relaxed for
    larger N, where random spectra are denser)."""
    rng = np.random.default_rng(seed)
    for _ in range(500):
        a = rng.uniform(0.5, 2.0, N - 1)
        w = np.linalg.eigvalsh(bo.tridiag_T_s(a))
        if np.min(np.diff(w)) > rel * np.max(np.abs(w)):
            return a
    raise RuntimeError("no well-separated spectrum found")


def gk_vectors(alpha):
    """Eigenvectors of T_s for its positive eigenvalues (ascending) from the
    SVD of the Golub-Kahan bidiagonal C (N even)."""
    N = alpha.shape[0] + 1
    n = N // 2
    C = np.diag(alpha[0::2]) + np.diag(alpha[1::2], 1)
    U, s, Vt = np.linalg.svd(C)
    order = np.argsort(s)
    Z = np.zeros((N, n))
    Z[0::2] = Vt.T[:, order]
    Z[1::2] = U[:, order]
    return s[order], Z / np.sqrt(2.0)


def check(alpha, tf=mrrr.twist_factors, te=mrrr.twisted_eigenvectors):
    """(name, ok, value) for each pin."""
    out = []
    N = alpha.shape[0] + 1
    T = bo.tridiag_T_s(alpha)
    w, V = np.linalg.eigh(T)
    # twist identity at shifts between and beside eigenvalues (off the
    # midpoints: the one between +-sigma pairs is 0, where the inverse of the
    # zero-diagonal T_s has a zero diagonal)
    xs = np.concatenate([(0.3 * w[:-1] + 0.7 * w[1:])[::max(1, N // 6)], [w[-1] + 0.1]])
    _, _, g = tf(alpha, xs)
    worst = 0.0
    for i, x in enumerate(xs):
        inv_diag = np.diag(np.linalg.inv(T - x * np.eye(N)))
        worst = max(worst, float(np.max(np.abs(g[:, i] * inv_diag - 1.0))))
    out.append(("gamma = 1/inv diag", worst <= 1e-9, worst))
    # against the dense eigenvectors, all eigenvalues (N arbitrary)
    Z = te(alpha, w)
    dv = float(np.max(np.abs(np.abs(np.sum(Z * V, axis=0)) - 1.0)))
    out.append(("eigh vectors", dv <= 1e-11, dv))
    res = float(np.max(np.linalg.norm(T @ Z - Z * w[None, :], axis=0)))
    out.append(("residual", res <= 4 * N * bo.EPS * np.max(np.abs(w)), res))
    if N % 2 == 0:
        s, Zg = gk_vectors(alpha)
        Zp = te(alpha, s)
        dg = float(np.max(np.abs(np.abs(np.sum(Zp * Zg, axis=0)) - 1.0)))
        out.append(("Golub-Kahan vectors", dg <= 1e-11, dg))
    return out


@pytest.mark.parametrize("N,seed,rel", [(2, 1, 1e-2), (3, 2, 1e-2), (4, 3, 1e-2), (17, 4, 1e-2), (40, 5, 1e-2),
                                        (64, 6, 1e-3), (101, 7, 1e-3)])
def test_twisted_pins(N, seed, rel):
    a = well_separated(N, seed, rel)
    for name, ok, val in check(a):
        assert ok, (name, val)


def test_twisted_on_a_bse_spectrum():
    """T_s of a BSE problem (n = 60) with the bisection eigenvalues, then the
    cluster Gram-Schmidt: orthonormal and matching the dense eigenvectors
    where the eigenvalues are isolated."""
    from bse_inputs import gen_bse
    p = gen_bse(60, s_a=0.3, seed=11)
    L, info = bo.cholesky(bo.build_M(p.A, p.B))
    assert info == 0
    W = bo.form_W(L)
    alpha = bo.skew_tridiagonalize(W)[0]
    lam = bo.bisect_positive(alpha)
    V = mrrr.eigenvectors_T_s_twisted(alpha, lam)
    T = bo.tridiag_T_s(alpha)
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) <= 1e-12
    assert np.max(np.linalg.norm(T @ V - V * lam[None, :], axis=0)) <= 1e-12 * np.max(lam)
    w, Vd = np.linalg.eigh(T)
    gaps = np.minimum(np.diff(np.concatenate([[-np.inf], lam])), np.diff(np.concatenate([lam, [np.inf]])))
    iso = gaps > 1e-3 * np.max(lam)
    d = np.abs(np.abs(np.sum(V * Vd[:, V.shape[0] // 2:], axis=0)) - 1.0)
    assert np.max(d[iso]) <= 1e-10


# ------------------------------------------------------------- planted mistakes

def _tf_dplus_both(alpha, lam):
    dp, dm, g = mrrr.twist_factors(alpha, lam)
    return dp, dp, dp + dp + np.asarray(lam)[None, :]


def _tf_no_diag(alpha, lam):
    dp, dm, _ = mrrr.twist_factors(alpha, lam)
    return dp, dm, dp + dm


def _te_from(tf, up_sign=-1.0, down_shift=0):
    def te(alpha, lam):
        N = alpha.shape[0] + 1
        dp, dm, gamma = tf(alpha, lam)
        Z = np.zeros((N, len(lam)))
        for j in range(len(lam)):
            r = int(np.argmin(np.abs(gamma[:, j])))
            z = np.zeros(N)
            z[r] = 1.0
            for k in range(r - 1, -1, -1):
                z[k] = up_sign * (alpha[k] / dp[k, j]) * z[k + 1]
            for k in range(r, N - 1):
                kk = min(k + down_shift, N - 2)
                z[k + 1] = -(alpha[kk] / dm[k + 1, j]) * z[k]
            Z[:, j] = z / np.linalg.norm(z)
        return Z
    return te


@pytest.mark.parametrize("mut", ["dplus_both", "up_sign", "no_diag", "down_index"])
def test_twisted_mutants_fail(mut):
    a = well_separated(40, 5)
    kw = {
        "dplus_both": {"tf": _tf_dplus_both, "te": _te_from(_tf_dplus_both)},
        "up_sign": {"te": _te_from(mrrr.twist_factors, up_sign=1.0)},
        "no_diag": {"tf": _tf_no_diag},
        "down_index": {"te": _te_from(mrrr.twist_factors, down_shift=1)},
    }[mut]
    assert not all(ok for _, ok, _ in check(a, **kw))
