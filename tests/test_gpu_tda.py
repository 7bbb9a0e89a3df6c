"""Tamm-Dancoff solve (bse_solve_tda) and the broadened spectra
(bse_spectra) on the GPU against the oracle (oracle/spectra.py), through the
C ABI.

Tolerances: TDA eigenvalues 1e-13 lambda_max (the chain is the FP64
structure-preserving one, whose eigenvalue error is ~1e-15 ||H||),
eigenvectors basis-invariant 1e-9 and weights 1e-10 as in the full-problem
parity tests; the zero block of x_j = [v_j; 0] to rounding (1e-13); spectra
relative to their maximum, 1e-12 (sums of the same Gaussians in another
order) plus the effect of the grid's rounding on a narrow Gaussian,
10 |omega| eps / sigma.
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import metrics, spectra
from bse_inputs import gen_bse

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


@pytest.mark.parametrize("n", [1, 2, 17, 64, 129, 300])
def test_tda_matches_oracle(ctx, n):
    p = gen_bse(n, s_a=0.3, s_b=0.05, seed=300 + n)
    say(f"[tda] n={n}")
    res = ctx.solve_tda(tt(p.A), d_r=tt(p.d))
    assert res["info"] == 0
    lam, X, w = npc(res["lam"]), npc(res["X"]), npc(res["w"])
    lo, Xo, wo = spectra.tda_solve(p.A, p.d)
    normH = float(lo.max())
    el = float(np.max(np.abs(lam - lo))) / normH
    ev = metrics.compare_eigvecs(Xo, X, lo, 1e-6 * normH)
    we = metrics.compare_weights(wo, w, lo, 1e-6 * normH)
    z = float(np.max(np.abs(X[n:])))
    say(f"  eig {el:.2e} vec {ev:.2e} w {we:.2e} zero block {z:.2e}")
    assert el <= 1e-13 and ev <= 1e-9 and we <= 1e-10 and z <= 1e-13


@pytest.mark.parametrize("n", [40, 300])
def test_tda_two_stage_with_vectors(ctx, n):
    """bse_solve_tda through the two-stage reduction and both stages'
    back-transformations: the same bar as the one-stage TDA path."""
    from paper_1501_03830_amd import _lib
    p = gen_bse(n, s_a=0.3, s_b=0.05, seed=320 + n)
    res = ctx.solve_tda(tt(p.A), d_r=tt(p.d), extra_flags=_lib.BSE_TWO_STAGE)
    assert res["info"] == 0
    lam, X, w = npc(res["lam"]), npc(res["X"]), npc(res["w"])
    lo, Xo, wo = spectra.tda_solve(p.A, p.d)
    normH = float(lo.max())
    el = float(np.max(np.abs(lam - lo))) / normH
    ev = metrics.compare_eigvecs(Xo, X, lo, 1e-6 * normH)
    we = metrics.compare_weights(wo, w, lo, 1e-6 * normH)
    z = float(np.max(np.abs(X[n:])))
    say(f"[tda two-stage] n={n}: eig {el:.2e} vec {ev:.2e} w {we:.2e} zero block {z:.2e}")
    assert el <= 1e-13 and ev <= 1e-9 and we <= 1e-10 and z <= 1e-13


@pytest.mark.parametrize("n,s_a", [(200, 0.3), (2048, 0.3), (1000, 0.1)])
def test_tda_overestimates_on_gpu(ctx, n, s_a):
    """Theorem 4 on the GPU results: the TDA eigenvalues bound the full
    problem's from above, pair by pair in sorted order."""
    p = gen_bse(n, s_a=s_a, s_b=0.05, seed=400 + n, check_definite=False)
    full = ctx.solve(tt(p.A), tt(p.B), vectors=False)
    tda = ctx.solve_tda(tt(p.A), vectors=False)
    assert full["info"] == 0 and tda["info"] == 0
    lf, lt = npc(full["lam"]), npc(tda["lam"])
    shift = (lt - lf) / lf
    say(f"[tda vs full] n={n} s_a={s_a}: relative shift min {shift.min():.2e} max {shift.max():.2e}")
    assert np.all(lf <= lt + 1e-13 * lt.max())
    assert shift.max() > 1e-6


def test_tda_not_definite_reports_minor(ctx):
    """A with a negative eigenvalue: its real embedding [Re A, Im A;
    -Im A, Re A] first fails at the leading minor of that diagonal entry."""
    u = np.random.default_rng(9).uniform(1.0, 10.0, size=40)
    u[12] = -1.0
    A = np.diag(u).astype(np.complex128)
    res = ctx.solve_tda(tt(A), vectors=False)
    assert res["info"] == 13


@pytest.mark.parametrize("n,npts,sigma", [(1, 1, 0.1), (64, 1000, 0.05), (300, 4097, 5e-4)])
def test_spectra_match_oracle(ctx, n, npts, sigma):
    p = gen_bse(n, s_a=0.3, s_b=0.05, seed=500 + n)
    r = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d))
    lam, w = r["lam"], r["w"]
    lo_, hi_ = float(lam.min()) - 8 * sigma, float(lam.max()) + 8 * sigma
    dom = (hi_ - lo_) / max(npts - 1, 1)
    d, e = ctx.spectra(lam, w, lo_, dom, npts, sigma)
    om = lo_ + dom * np.arange(npts)
    do = spectra.dos(npc(lam), om, sigma)
    eo = spectra.absorption(npc(lam), npc(w), om, sigma)
    ed = float(np.max(np.abs(npc(d) - do))) / max(float(do.max()), 1e-300)
    ee = float(np.max(np.abs(npc(e) - eo))) / max(float(np.abs(eo).max()), 1e-300)
    # omega_k carries a rounding of about |omega| eps, which moves a Gaussian
    # of width sigma by |t| |omega| eps / sigma^2 relative (|t| <= ~6 sigma
    # where it matters): 1e-12 plus 10 |omega|_max eps / sigma
    tol = 1e-12 + 10.0 * max(abs(lo_), abs(hi_)) * np.finfo(np.float64).eps / sigma
    say(f"[spectra] n={n} npts={npts} sigma={sigma}: dos {ed:.2e} eps {ee:.2e} (tol {tol:.1e})")
    assert ed <= tol and ee <= tol


def test_spectra_dos_only_and_argument_errors(ctx):
    from paper_1501_03830_amd import _lib
    lam = torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64, device=ctx.device)
    d, e = ctx.spectra(lam, None, -4.0, 0.01, 801, 0.1)
    assert e is None
    om = -4.0 + 0.01 * np.arange(801)
    assert np.max(np.abs(npc(d) - spectra.dos(npc(lam), om, 0.1))) <= 1e-12 * float(npc(d).max())
    lib = ctx.lib
    assert lib.bse_spectra(ctx.h, 3, lam.data_ptr(), None, 0, 0.0, 0.1, 0.1, lam.data_ptr(), None) == -5
    assert lib.bse_spectra(ctx.h, 3, lam.data_ptr(), None, 10, 0.0, 0.1, 0.0, lam.data_ptr(), None) == -8
    assert lib.bse_spectra(ctx.h, 3, lam.data_ptr(), None, 10, 0.0, 0.1, 0.1, None, lam.data_ptr()) == -4
