"""Request serving (bse_submit / bse_poll / bse_release): continuous batching.

Each result must be bit for bit the one bse_solve gives for the same request
alone: batching and concurrent slots change neither the arithmetic nor its
order.  The server must also overlap work (more than one batch and more than
one request in flight), respect its memory pool, report failures per
request, and free resident workspaces on release.
"""

import sys
import time

import numpy as np
import pytest
import torch

from bse_inputs import gen_bse, gen_not_definite, serving_stream

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def tt(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def _ctx(pool=4 * GiB, slots=3, max_batch=16):
    from paper_1501_03830_amd.api import Context
    c = Context(0)
    c.serve_config(pool, slots, max_batch)
    return c


def _wait(ctx, tickets, timeout=120.0):
    from paper_1501_03830_amd import _lib
    t0 = time.time()
    pending = set(tickets)
    states = {}
    while pending:
        for t in list(pending):
            st, info = ctx.poll(t)
            if st in (_lib.BSE_DONE, _lib.BSE_FAILED):
                states[t] = (st, info)
                pending.discard(t)
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(pending)} requests not finished")
        time.sleep(0.002)
    return states


def test_serving_results_equal_alone():
    """A stream of mixed sizes submitted in waves while earlier ones run:
    every result equals bse_solve on the request alone."""
    from paper_1501_03830_amd import _lib
    _, ns = serving_stream(count=30, qps=1.0, lo=16, hi=300, big=600, big_frac=0.1, seed=11)
    ns = [int(k) for k in ns]
    say(f"[serving] sizes {ns}")
    probs = [gen_bse(n, seed=100000 + i, check_definite=False) for i, n in enumerate(ns)]
    ctx = _ctx()
    try:
        tickets, outs = [], []
        for i, p in enumerate(probs):
            t, o = ctx.submit(tt(p.A), tt(p.B), d_r=tt(p.d))
            tickets.append(t)
            outs.append(o)
            if i % 10 == 9:
                time.sleep(0.05)   # later waves arrive while earlier batches run
        states = _wait(ctx, tickets)
        stats = ctx.serve_stats()
        say(f"  stats {stats}")
        for i, p in enumerate(probs):
            st, info = states[tickets[i]]
            assert st == _lib.BSE_DONE and info == 0, (i, st, info)
            alone = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d))
            assert torch.equal(outs[i]["lam"], alone["lam"]), i
            assert torch.equal(outs[i]["X"], alone["X"]), i
            assert torch.equal(outs[i]["w"], alone["w"]), i
        assert stats["solved"] == len(probs)
        assert stats["batches"] >= 2
        assert stats["max_inflight"] >= 2
        ts = [ctx.ticket_times(t) for t in tickets]
        assert all(0 <= a <= b <= c for a, b, c in ts)
        for t in tickets:
            assert ctx.release(t) == 0
        assert ctx.serve_stats()["used_bytes"] == 0
        with pytest.raises(RuntimeError):
            ctx.poll(tickets[0])
    finally:
        ctx.close()


def test_serving_failure_is_per_request():
    from paper_1501_03830_amd import _lib
    from oracle import bse_oracle as bo
    good = [gen_bse(n, seed=n) for n in (30, 45)]
    bad = gen_not_definite(40, 9, seed=4)
    _, info_o = bo.cholesky(bo.build_M(bad.A, bad.B))
    ctx = _ctx()
    try:
        t0, o0 = ctx.submit(tt(good[0].A), tt(good[0].B))
        tb, _ = ctx.submit(tt(bad.A), tt(bad.B))
        t1, o1 = ctx.submit(tt(good[1].A), tt(good[1].B))
        states = _wait(ctx, [t0, tb, t1])
        assert states[tb] == (_lib.BSE_FAILED, info_o)
        assert states[t0] == (_lib.BSE_DONE, 0) and states[t1] == (_lib.BSE_DONE, 0)
        a0 = ctx.solve(tt(good[0].A), tt(good[0].B))
        assert torch.equal(o0["lam"], a0["lam"]) and torch.equal(o0["X"], a0["X"])
    finally:
        ctx.close()


def test_serving_admission_by_footprint():
    """A pool that holds only two of the requests at a time: all complete,
    the pool is never exceeded, and results still equal bse_solve alone."""
    from paper_1501_03830_amd import _lib
    from paper_1501_03830_amd.api import footprint_bytes
    n = 200
    fp = footprint_bytes(n)
    pool = 2 * fp + 2 * 1024 * 1024
    probs = [gen_bse(n, seed=300 + i) for i in range(5)]
    ctx = _ctx(pool=pool, slots=2, max_batch=8)
    try:
        tickets, outs = [], []
        for p in probs:
            t, o = ctx.submit(tt(p.A), tt(p.B), vectors=False)
            tickets.append(t)
            outs.append(o)
        lams = {}
        t0 = time.time()
        while len(lams) < len(tickets):   # release results as they finish
            for t, o in zip(tickets, outs):
                if t in lams:
                    continue
                st, info = ctx.poll(t)
                if st == _lib.BSE_DONE:
                    lams[t] = o["lam"].clone()
                    assert ctx.release(t) == 0
            assert time.time() - t0 < 120
            time.sleep(0.002)
        stats = ctx.serve_stats()
        say(f"  stats {stats}")
        assert stats["peak_used_bytes"] <= pool
        assert stats["solved"] == len(probs)
        for p, t in zip(probs, tickets):
            a = ctx.solve(tt(p.A), tt(p.B), vectors=False)
            assert torch.equal(lams[t], a["lam"])
    finally:
        ctx.close()


def test_serving_rejects_oversized_and_bad_requests():
    from paper_1501_03830_amd import _lib
    from paper_1501_03830_amd.api import footprint_bytes
    ctx = _ctx(pool=footprint_bytes(64) + 2 * 1024 * 1024, slots=1)
    try:
        p = gen_bse(200, seed=1)
        with pytest.raises(_lib.BseError) as e:
            ctx.submit(tt(p.A), tt(p.B))
        assert e.value.code == _lib.BSE_ENOMEM
        q = gen_bse(64, seed=2)
        t, o = ctx.submit(tt(q.A), tt(q.B))
        st = _wait(ctx, [t])
        assert st[t][0] == _lib.BSE_DONE
        assert ctx.release(t) == 0
        with pytest.raises(_lib.BseError) as e:
            ctx.release(t)
        assert e.value.code == _lib.BSE_ENOTICKET
    finally:
        ctx.close()


def test_serving_batch_past_64_requests():
    """One batch of more than 64 requests (max_batch 128, one slot): a large
    request keeps the slot busy while 100 small ones of similar order queue
    up, so they run together as one batch, the way the server's default
    batch limit (64) and beyond are reached under load.  Results equal
    bse_solve alone, bit for bit, across the batch's whole sorted order."""
    from paper_1501_03830_amd import _lib
    rng = np.random.default_rng(12)
    ns = [int(k) for k in rng.integers(40, 71, size=100)]
    say(f"[serving] 100 requests n in [40, 70] behind one n=1200 request, max_batch 128")
    from paper_1501_03830_amd.api import to_colmajor, from_colmajor
    big = gen_bse(1200, seed=5)
    probs = [gen_bse(n, seed=200000 + i, check_definite=False) for i, n in enumerate(ns)]
    ctx = _ctx(pool=8 * GiB, slots=1, max_batch=128)
    dev = ctx.device
    try:
        # inputs and outputs staged on the device first, so that the small
        # requests are all queued while the large one runs
        staged = []
        for p in probs:
            n = p.A.shape[0]
            staged.append((n, to_colmajor(tt(p.A), dev), to_colmajor(tt(p.B), dev),
                           torch.empty(n, dtype=torch.float64, device=dev),
                           torch.empty((n, 2 * n), dtype=torch.complex128, device=dev),
                           tt(p.d).to(dev), torch.empty(n, dtype=torch.complex128, device=dev)))
        torch.cuda.synchronize()
        tb, _ = ctx.submit(tt(big.A), tt(big.B))
        tickets = [ctx.submit_raw(n, Ac, Bc, lam, X, d, None, w) for (n, Ac, Bc, lam, X, d, w) in staged]
        outs = [{"lam": lam, "X": from_colmajor(X), "w": w} for (n, Ac, Bc, lam, X, d, w) in staged]
        states = _wait(ctx, [tb] + tickets)
        stats = ctx.serve_stats()
        say(f"  stats {stats}")
        assert all(states[t] == (_lib.BSE_DONE, 0) for t in tickets)
        assert stats["max_inflight"] > 64
        order = sorted(range(len(ns)), key=lambda i: -ns[i])
        for r in (0, 1, 30, 63, 64, 65, 80, 99):
            i = order[r]
            p = probs[i]
            alone = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d))
            assert torch.equal(outs[i]["lam"], alone["lam"]), i
            assert torch.equal(outs[i]["X"], alone["X"]), i
            assert torch.equal(outs[i]["w"], alone["w"]), i
        for t in [tb] + tickets:
            assert ctx.release(t) == 0
    finally:
        ctx.close()
