"""Eigenvectors by twisted factorisations (BSE_EIGVEC_TWISTED, the
per-vector step of MRRR) through the C ABI, against the oracle of the same
method (oracle/mrrr.py) and end to end against the Algorithm 1 oracle.

* Stage: bse_tridiag_eig_flags on the oracle's alpha; eigenvalues bit for
  bit the bisection's; vectors equal the oracle's twisted vectors (up to
  sign; inside clusters the same span) to 1e-9, residuals and orthogonality
  to 1e-13 as for inverse iteration.
* A split, exactly degenerate T_s (three equal blocks): the degenerate
  eigenvalues go to inverse iteration, the rest stay twisted; orthonormal.
* End to end (n from 1 to 200, s_a = 0.3 at n = 160, the 256-problem batch's
  first members, the mixed policy): the same tolerances as the parity tests,
  and X against the default path's X (basis-invariant).
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import bse_oracle as bo
from oracle import metrics, mrrr
from bse_inputs import gen_bse, batched_sizes

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1501_03830_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def npc(t):
    return t.detach().cpu().numpy()


def tt(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def TW():
    from paper_1501_03830_amd import _lib
    return _lib.BSE_EIGVEC_TWISTED


@pytest.mark.parametrize("n", [1, 2, 3, 8, 17, 64, 65, 100, 200])
def test_twisted_stage_matches_oracle(ctx, n):
    say(f"[twisted stage] n={n}")
    p = gen_bse(n, s_a=0.3 if n >= 64 else 0.1, seed=60 + n)
    Lo, _ = bo.cholesky(bo.build_M(p.A, p.B))
    ao, _, _ = bo.skew_tridiagonalize(bo.form_W(Lo))
    lam_o = bo.bisect_positive(ao)
    lam, V = ctx.tridiag_eig(tt(ao), flags=TW())
    lam, V = npc(lam), npc(V)
    assert np.array_equal(lam, lam_o)
    Ts = bo.tridiag_T_s(ao)
    tn = bo.gershgorin_bound(ao)
    res = float(np.max(np.abs(Ts @ V - V * lam[None, :])))
    orth = float(np.max(np.abs(V.T @ V - np.eye(n))))
    Vo = mrrr.eigenvectors_T_s_twisted(ao, lam_o)
    worst = 0.0
    for s_, e_ in metrics.clusters(lam, 1e-6 * tn):
        P, Q = Vo[:, s_:e_], V[:, s_:e_]
        worst = max(worst, float(np.linalg.norm(Q - P @ (P.T @ Q))))
    say(f"  residual {res:.2e}, orthogonality {orth:.2e}, vs oracle {worst:.2e}")
    assert res <= 1e-13 * tn * max(1.0, math.sqrt(n) / 8)
    assert orth <= 1e-13 * max(1.0, math.sqrt(n) / 8)
    assert worst <= 1e-9


def test_twisted_split_degenerate(ctx):
    say("[twisted stage] split degenerate")
    blk = [1.0, 0.7, 2.0, 0.3, 1.1]
    alpha = np.array(blk + [0.0] + blk + [0.0] + blk)   # N = 18, three equal blocks
    N = alpha.shape[0] + 1
    lam, V = ctx.tridiag_eig(tt(alpha), flags=TW())
    lam, V = npc(lam), npc(V)
    Ts = bo.tridiag_T_s(alpha)
    assert np.max(np.abs(Ts @ V - V * lam[None, :])) <= 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(N // 2))) <= 1e-13


def _check(A, B, d, res, ro, tag, vec_tol=1e-9):
    n = A.shape[0]
    lam, X, w = npc(res["lam"]), npc(res["X"]), npc(res["w"])
    H = metrics.H_matrix(*bo.symmetrize_lower(A, B))
    normH = np.linalg.norm(H, 2)
    el = np.max(np.abs(lam - ro.lam)) / normH
    gap = 1e-6 * normH
    ev = metrics.compare_eigvecs(ro.X, X, ro.lam, gap)
    we = metrics.compare_weights(ro.w, w, ro.lam, gap)
    r1, r2 = metrics.table1_metrics(*bo.symmetrize_lower(A, B), lam, X)
    say(f"  {tag}: eig {el:.2e}, eigvec {ev:.2e}, weights {we:.2e}, table1 {r1:.1e} {r2:.1e}")
    assert el <= 1e-13 and ev <= vec_tol and we <= 1e-10 and r1 <= 1e-12 and r2 <= 1e-12
    assert metrics.normalization_error(X) <= 1e-12


@pytest.mark.parametrize("n,s_a", [(1, 0.1), (2, 0.1), (3, 0.1), (17, 0.1), (64, 0.1), (65, 0.1), (129, 0.1),
                                   (200, 0.1), (160, 0.3)])
def test_twisted_solve_matches_oracle(ctx, n, s_a):
    say(f"[twisted solve] n={n} s_a={s_a}")
    p = gen_bse(n, s_a=s_a, seed=70 + n)
    ro = oracle.solve(p.A, p.B, p.d)
    res = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), extra_flags=TW())
    assert res["info"] == 0
    _check(p.A, p.B, p.d, res, ro, f"n={n}")
    # the same X as the default path (basis-invariant inside clusters)
    r0 = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d))
    H = metrics.H_matrix(*bo.symmetrize_lower(p.A, p.B))
    assert torch.equal(res["lam"], r0["lam"])
    ev = metrics.compare_eigvecs(npc(r0["X"]), npc(res["X"]), npc(r0["lam"]), 1e-6 * np.linalg.norm(H, 2))
    assert ev <= 1e-9


def test_twisted_batched_members_equal_solo(ctx):
    """Batch members with the flag equal their solo solves with the flag bit
    for bit (the first 40 sizes of the batched workload)."""
    say("[twisted batched]")
    ns = [int(k) for k in batched_sizes(256, 64, 1024, seed=4)][:40:4]
    ps = [gen_bse(k, s_a=0.1, seed=1000 + i) for i, k in enumerate(ns)]
    out, _ = ctx.solve_batched([tt(p.A) for p in ps], [tt(p.B) for p in ps], ds=[tt(p.d) for p in ps],
                               extra_flags=TW())
    for p, o in zip(ps, out):
        assert o["info"] == 0
        solo = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), extra_flags=TW())
        assert torch.equal(o["lam"], solo["lam"]) and torch.equal(o["X"], solo["X"]) and torch.equal(o["w"], solo["w"])


def test_twisted_mixed_policy(ctx):
    from paper_1501_03830_amd import _lib
    say("[twisted mixed] n=150 s_a=0.3")
    p = gen_bse(150, s_a=0.3, seed=91)
    ro = oracle.solve(p.A, p.B, p.d)
    res = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), prec=_lib.BSE_PREC_FP32_REFINE, extra_flags=TW(), report=True)
    assert res["info"] == 0
    H = metrics.H_matrix(*bo.symmetrize_lower(p.A, p.B))
    normH = np.linalg.norm(H, 2)
    el = np.max(np.abs(npc(res["lam"]) - ro.lam)) / normH
    ev = metrics.compare_eigvecs(ro.X, npc(res["X"]), ro.lam, 1e-6 * normH)
    say(f"  eig {el:.2e}, eigvec {ev:.2e}, sweeps {res['report']['refine_sweeps']}")
    assert el <= 1e-10 and ev <= 1e-6
