"""Batched solves through bse_solve_batched.

A problem's arithmetic does not depend on the batch it is solved in (the
launch shapes that fix a summation order are chosen per problem), so every
member of a batch must equal, bit for bit, the same problem solved alone
with bse_solve.  Members are also checked against the CPU oracle to the
tolerances of the single-solve tests (eigenvalues <= 1e-10 ||H||_2,
eigenvectors and weights by the cluster-invariant comparison).
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import bse_oracle as bo
from oracle import metrics
from bse_inputs import gen_bse, gen_not_definite, batched_sizes

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


def _same(a, b):
    return (a is None and b is None) or torch.equal(a, b)


# ragged sizes: several tiles, tails of 1 and 63, duplicates, the minimum n
RAGGED = [65, 1, 130, 2, 33, 64, 5, 100, 257, 64, 17, 3]


def test_batched_equals_single_bitwise(ctx):
    say(f"[batched] sizes {RAGGED}")
    probs = [gen_bse(n, seed=700 + i) for i, n in enumerate(RAGGED)]
    out, rep = ctx.solve_batched([tt(p.A) for p in probs], [tt(p.B) for p in probs],
                                 ds=[tt(p.d) for p in probs], report=True)
    say(f"  batch report total {rep['total_ms']:.2f} ms")
    for i, p in enumerate(probs):
        single = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d))
        assert out[i]["info"] == 0 and single["info"] == 0
        assert torch.equal(out[i]["lam"], single["lam"]), i
        assert torch.equal(out[i]["X"], single["X"]), i
        assert torch.equal(out[i]["w"], single["w"]), i


@pytest.mark.parametrize("idx", [0, 2, 8])
def test_batched_members_match_oracle(ctx, idx):
    n = RAGGED[idx]
    say(f"[batched] member {idx} n={n} vs oracle")
    probs = [gen_bse(k, seed=700 + i) for i, k in enumerate(RAGGED)]
    out, _ = ctx.solve_batched([tt(p.A) for p in probs], [tt(p.B) for p in probs],
                               ds=[tt(p.d) for p in probs])
    p = probs[idx]
    ro = oracle.solve(p.A, p.B, p.d)
    H = metrics.H_matrix(*bo.symmetrize_lower(p.A, p.B))
    normH = np.linalg.norm(H, 2)
    lam = npc(out[idx]["lam"])
    el = np.max(np.abs(lam - ro.lam)) / normH
    say(f"  eig err {el:.2e}")
    assert el <= 1e-10
    gap = 1e-6 * normH
    X = npc(out[idx]["X"])
    ev = metrics.compare_eigvecs(ro.X, X, ro.lam, gap)
    assert ev <= 1e-9, ev
    r1, r2 = metrics.table1_metrics(*bo.symmetrize_lower(p.A, p.B), lam, X)
    assert r1 <= 1e-12 and r2 <= 1e-12
    we = metrics.compare_weights(ro.w, npc(out[idx]["w"]), ro.lam, gap)
    assert we <= 1e-10, we


def test_batched_not_definite_member(ctx):
    """A member whose M is not definite reports its leading minor (the same
    as bse_solve and the oracle) and leaves the others untouched."""
    say("[batched] one member not definite")
    good = [gen_bse(n, seed=900 + n) for n in (40, 70)]
    bad = gen_not_definite(50, 17, seed=3)
    As = [tt(good[0].A), tt(bad.A), tt(good[1].A)]
    Bs = [tt(good[0].B), tt(bad.B), tt(good[1].B)]
    out, _ = ctx.solve_batched(As, Bs)
    _, info_o = bo.cholesky(bo.build_M(bad.A, bad.B))
    single_bad = ctx.solve(tt(bad.A), tt(bad.B))
    assert out[1]["info"] == info_o == single_bad["info"] > 0
    for k, i in ((0, 0), (1, 2)):
        s = ctx.solve(tt(good[k].A), tt(good[k].B))
        assert out[i]["info"] == 0
        assert torch.equal(out[i]["lam"], s["lam"])
        assert torch.equal(out[i]["X"], s["X"])


def test_batched_eigenvalues_only(ctx):
    say("[batched] eigenvalues only")
    probs = [gen_bse(n, seed=40 + n) for n in (90, 7, 200)]
    out, _ = ctx.solve_batched([tt(p.A) for p in probs], [tt(p.B) for p in probs], vectors=False)
    for i, p in enumerate(probs):
        s = ctx.solve(tt(p.A), tt(p.B), vectors=False)
        assert out[i]["X"] is None
        assert torch.equal(out[i]["lam"], s["lam"])


def test_batched_empty(ctx):
    out, _ = ctx.solve_batched([], [])
    assert out == []


def test_batched_config_sizes_sample(ctx):
    """The log-uniform size mix of the 256-problem workload (first 24
    members, seeds 1000+i): batch vs single, bit for bit."""
    ns = [int(k) for k in batched_sizes(256, 64, 1024, seed=4)[:24]]
    say(f"[batched] workload sizes {ns}")
    probs = [gen_bse(n, seed=1000 + i, check_definite=False) for i, n in enumerate(ns)]
    out, rep = ctx.solve_batched([tt(p.A) for p in probs], [tt(p.B) for p in probs], report=True)
    say(f"  batch total {rep['total_ms']:.1f} ms")
    for i in (0, 5, 11, 23):
        p = probs[i]
        s = ctx.solve(tt(p.A), tt(p.B))
        assert out[i]["info"] == 0
        assert torch.equal(out[i]["lam"], s["lam"]), i
        assert torch.equal(out[i]["X"], s["X"]), i


# ---------------------------------------------------------------------------
# The full 256-problem workload in one call (sizes log-uniform in [64, 1024],
# size seed 4, problem i from seed 1000 + i), as the benchmark runs it.  A
# batch this large takes the paths a small one never reaches: the matvec and
# update launches locate their problem by ballots over 64 prefixes at a time
# (several rounds past 64 active problems), and the per-panel planning kernel
# gives each thread several problems.  Every member's eigenvalues, and the
# eigenvectors and weights of members spread over the sorted order (the
# launches' problem index) including positions past 64 and past 128, must
# equal bse_solve on the member alone, bit for bit.

@pytest.fixture(scope="module")
def config4():
    ns = [int(k) for k in batched_sizes(256, 64, 1024, seed=4)]
    probs = [gen_bse(n, s_a=0.1, s_b=0.05, seed=1000 + i, check_definite=False) for i, n in enumerate(ns)]
    # descriptor order inside the library: decreasing n, stable
    order = sorted(range(len(ns)), key=lambda i: -ns[i])
    return ns, probs, order


@pytest.mark.parametrize("prec_name", ["fp64", "fp32_refine"])
def test_batched_full_workload_equals_single(ctx, config4, prec_name):
    from paper_1501_03830_amd import _lib
    prec = _lib.BSE_PREC_FP64 if prec_name == "fp64" else _lib.BSE_PREC_FP32_REFINE
    ns, probs, order = config4
    say(f"[batched] full workload, 256 problems, {prec_name}")
    out, rep = ctx.solve_batched([tt(p.A) for p in probs], [tt(p.B) for p in probs],
                                 ds=[tt(p.d) for p in probs], report=True, prec=prec)
    say(f"  batch total {rep['total_ms']:.1f} ms")
    assert all(o["info"] == 0 for o in out)
    ranks = [0, 1, 31, 63, 64, 65, 100, 127, 128, 129, 160, 191, 192, 224, 254, 255]
    full = {order[r] for r in ranks}
    for i, p in enumerate(probs):
        s = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), prec=prec)
        assert s["info"] == 0
        assert torch.equal(out[i]["lam"], s["lam"]), (i, ns[i])
        if i in full:
            assert torch.equal(out[i]["X"], s["X"]), (i, ns[i])
            assert torch.equal(out[i]["w"], s["w"]), (i, ns[i])
    say(f"  all 256 eigenvalue sets and {len(full)} vector sets equal")
