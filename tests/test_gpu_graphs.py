"""Graph replay of the chain after the Cholesky (bse_ctx_set_graphs): the
results of captured and replayed graphs equal plain stream launches bit for
bit, on every replay, with other work and synchronisations between the
replays (graphs on this device have given wrong results on replays after the
first when they held memset nodes; the chain records none, and this test
checks every replay)."""

import sys

import numpy as np
import pytest
import torch

from bse_inputs import gen_bse, gen_not_definite

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def tt(a):
    return torch.from_numpy(np.ascontiguousarray(a))


@pytest.fixture(scope="module")
def ctx():
    from paper_1501_03830_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def batch(ctx, probs, graphs, report=True):
    ctx.set_graphs(graphs)
    out, rep = ctx.solve_batched([tt(p.A) for p in probs], [tt(p.B) for p in probs],
                                 ds=[tt(p.d) for p in probs], report=report)
    torch.cuda.synchronize()
    return out, rep


def same(a, b):
    for x, y in zip(a, b):
        assert x["info"] == y["info"]
        if x["info"] != 0:
            continue
        assert torch.equal(x["lam"], y["lam"])
        assert torch.equal(x["X"], y["X"])
        assert torch.equal(x["w"], y["w"])


def test_batched_replays_equal_plain_launches(ctx):
    ns = [70, 33, 129, 64, 200, 17, 90, 150]
    probs = [gen_bse(n, s_a=0.3, s_b=0.05, seed=900 + i) for i, n in enumerate(ns)]
    plain, rp = batch(ctx, probs, False)
    assert rp["graph"] == 0
    other = gen_bse(45, seed=5)
    for it in range(4):
        out, rep = batch(ctx, probs, True)
        say(f"[graph] replay {it}: graph {rep['graph']}, {rep['total_ms']:.1f} ms")
        assert rep["graph"] == 1
        same(out, plain)
        # eager work and synchronisations between replays
        ctx.set_graphs(False)
        ctx.solve(tt(other.A), tt(other.B))
        torch.cuda.synchronize()
        _ = (torch.ones(1 << 20, device=ctx.device) * 3.0).sum().item()


def test_graph_shapes_and_dropped_member(ctx):
    """A batch whose member is not definite runs a smaller live batch (a
    shape of its own); the result still equals plain launches."""
    ns = [40, 80, 60]
    probs = [gen_bse(n, seed=950 + i) for i, n in enumerate(ns)]
    probs[1] = gen_not_definite(80, k=11, seed=3)
    plain, _ = batch(ctx, probs, False)
    assert plain[1]["info"] > 0
    for _ in range(2):
        out, rep = batch(ctx, probs, True)
        same(out, plain)


def test_single_solve_replay(ctx):
    p = gen_bse(300, s_a=0.3, seed=77)
    ctx.set_graphs(False)
    a = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), report=True)
    assert a["report"]["graph"] == 0
    ctx.set_graphs(True)
    for _ in range(3):
        b = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), report=True)
        assert b["report"]["graph"] == 1
        assert torch.equal(a["lam"], b["lam"]) and torch.equal(a["X"], b["X"]) and torch.equal(a["w"], b["w"])
    ctx.set_graphs(True)
