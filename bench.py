"""Benchmark of the full structure-preserving Bethe-Salpeter eigensolve.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192] [--s_a 0.3]

One step is one complete solve through the C ABI (Algorithm 1 as organised by
Algorithm 3: embedding, Cholesky, W = L^T J L, skew tridiagonalisation,
bisection + inverse iteration, back-transformation to x_j, and the absorption
weights) of one synthetic problem whose matrices are already resident in HBM.
The default workload is n = 8192 (real 16384 x 16384 Hamiltonian form) with
the generator of the mixed-precision configuration (kernel scale 0.3 so that
eigenvalues cluster), solved in FP64.

Printed: one JSON line with the metric (seconds per solve), the roofline of
the dominant kernel (the tiled skew matrix-vector product, HBM-bound) measured
live with hipEvents around each of its launches, per-stage times and
roofline fractions, and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6           # MI355X dense FP64 (matrix and vector), TFLOP/s
FP32_PEAK_TFS = 157.3          # MI355X dense FP32 matrix, TFLOP/s


def stage_work(n: int, mixed: bool = False, sweeps: int = 0):
    """Algorithmic work per stage: (bound, amount, peak).  Flop counts are
    the method's own (triangular structure used), bytes the data a stage
    must move once.  Bisection and inverse iteration are chains of
    dependent scalar operations (bound "latency", no fraction)."""
    N = 2 * n
    wbytes = 4.0 if mixed else 8.0
    tri_bytes = sum(wbytes * m * (m - 1) / 2 for m in range(1, N))    # symv reads
    work = {
        "build_M": ("hbm", 2 * 16.0 * n * (n + 1) / 2 + 8.0 * N * (N + 1) / 2, HBM_PEAK_GBS),
        "potrf": ("mfma", N ** 3 / 3.0, FP64_PEAK_TFS),
        "form_W": ("mfma", 5.0 / 3.0 * n ** 3, FP64_PEAK_TFS),
        "sktrd": ("hbm", tri_bytes, HBM_PEAK_GBS),
        "bisect": ("latency", 0.0, None),
        "invit": ("latency", 0.0, None),
        "apply_U": ("mfma", 16.0 * n ** 3, FP32_PEAK_TFS if mixed else FP64_PEAK_TFS),
        "apply_L": ("mfma", 8.0 * n ** 3, FP64_PEAK_TFS),
    }
    if mixed:
        # per sweep 8 n^3 (Y = L Ub, L triangular) + 8 (C = Y_top^T Y_bot)
        # + 8 (G, lower) in FP64 and 16 n^3 (the FP32 update), each part
        # against its own peak (the final eigenvalues come from the product
        # with L of the output, O(n^2))
        work["refine"] = ("mfma_split", (24.0 * sweeps * n ** 3, 16.0 * sweeps * n ** 3),
                          (FP64_PEAK_TFS, FP32_PEAK_TFS))
    else:
        # one Cholesky QR pass: Gram matrix, its Cholesky, forward substitution
        work["reorth"] = ("mfma", 2.0 * n * n * N + n ** 3 / 3.0, FP64_PEAK_TFS)
    return work


def stage_roofline(stage_ms: dict, work: dict) -> dict:
    stages = {}
    for name, ms in stage_ms.items():
        entry = {"ms": round(ms, 3)}
        if name in work and ms > 0:
            bound, amount, peak = work[name]
            if bound == "hbm":
                ach = amount / (ms * 1e-3) / 1e9
                entry.update(bound="hbm", achieved=round(ach, 1), unit="GB/s", frac=round(ach / peak, 4))
            elif bound == "mfma":
                ach = amount / (ms * 1e-3) / 1e12
                entry.update(bound="mfma", achieved=round(ach, 2), unit="TFLOP/s", frac=round(ach / peak, 4))
            elif bound == "mfma_split":
                # FP64 and FP32 flops: the floor is the sum of both parts at
                # their own peaks; frac = floor / measured time
                floor_ms = sum(f / (pk * 1e12) for f, pk in zip(amount, peak)) * 1e3
                ach = sum(amount) / (ms * 1e-3) / 1e12
                entry.update(bound="mfma", achieved=round(ach, 2), unit="TFLOP/s (FP64 + FP32)",
                             floor_ms=round(floor_ms, 2), frac=round(floor_ms / ms, 4),
                             flops_fp64=amount[0], flops_fp32=amount[1])
            else:
                entry.update(bound=bound)
        stages[name] = entry
    return stages


def cpu_baseline(n_samples, n_target: int, s_a: float, s_b: float):
    """The CPU oracle, as it stands, timed on problems of the same generator
    at the sizes n_samples (about 20 s of host time in all); the time at
    n_target comes from a least-squares fit t = c n^3 over the samples (the
    method's flop count is cubic), labelled as extrapolated.  Also a stronger
    CPU line for context: LAPACK's Hermitian eigensolver (numpy eigh, i.e.
    zheevd) on -iW at the largest sample, with the same cube-law scaling."""
    import oracle
    from bse_inputs import gen_bse
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    pts = []
    for k in n_samples:
        p = gen_bse(k, s_a=s_a, s_b=s_b, seed=3)
        t0 = time.perf_counter()
        r = oracle.solve(p.A, p.B, p.d)
        dt = time.perf_counter() - t0
        assert r.info == 0
        pts.append((k, dt))
        print(f"# cpu oracle n={k}: {dt:.2f} s", file=sys.stderr, flush=True)
    ns = np.array([q[0] for q in pts], dtype=float)
    ts = np.array([q[1] for q in pts])
    c = float(np.sum(ts * ns ** 3) / np.sum(ns ** 6))
    slope = float(np.polyfit(np.log(ns), np.log(ts), 1)[0])
    value = c * n_target ** 3
    # LAPACK zheevd on the Hermitian -iW of the largest sample
    kmax = int(ns.max())
    p = gen_bse(kmax, s_a=s_a, s_b=s_b, seed=3)
    M = oracle.build_M(p.A, p.B)
    L = oracle.cholesky(M)[0]
    W = oracle.form_W(L)
    t0 = time.perf_counter()
    np.linalg.eigh(-1j * W)
    t_eigh = time.perf_counter() - t0
    return {
        "value": value,
        "unit": "s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle.solve (same generator, s_a={s_a}) timed at n=" + ", ".join(f"{k}: {t:.2f} s" for k, t in pts)
                   + f"; least-squares t = c n^3 (c = {c:.3e} s; log-log slope {slope:.2f}) gives n={n_target} "
                   f"(extrapolated)"),
        "fit_points": [[int(k), round(t, 3)] for k, t in pts],
        "loglog_slope": round(slope, 3),
        "lapack_zheevd_line": {
            "what": f"numpy.linalg.eigh (LAPACK zheevd) on -iW, N={2 * kmax}, eigenvalues + vectors, no "
                    f"Cholesky/back-transformation", "seconds": round(t_eigh, 3),
            "at_n_target_s": round(t_eigh * (n_target / kmax) ** 3, 1), "scaling": "cube law (extrapolated)"},
        "host_cpus": os.cpu_count(),
    }


def batched_bench(ctx, steps: int, warmup: int, count: int = 256, lo: int = 64, hi: int = 1024,
                  size_seed: int = 4, s_a: float = 0.1, s_b: float = 0.05, mixed: bool = False):
    """The batched workload: `count` independent problems, n_i log-uniform in
    [lo, hi] (seed size_seed), problem i from seed 1000 + i, one
    bse_solve_batched call per step with inputs resident in HBM, all
    eigenvalues, eigenvectors and weights."""
    import torch
    from bse_inputs import gen_bse, batched_sizes
    from paper_1501_03830_amd import _lib
    from paper_1501_03830_amd.api import to_colmajor

    prec = _lib.BSE_PREC_FP32_REFINE if mixed else _lib.BSE_PREC_FP64

    dev = torch.device("cuda", 0)
    ns = [int(k) for k in batched_sizes(count, lo, hi, seed=size_seed)]
    t0 = time.time()
    Acs, Bcs, ds = [], [], []
    for i, k in enumerate(ns):
        pr = gen_bse(k, s_a=s_a, s_b=s_b, seed=1000 + i, check_definite=False)
        Acs.append(to_colmajor(torch.from_numpy(pr.A), dev))
        Bcs.append(to_colmajor(torch.from_numpy(pr.B), dev))
        ds.append(torch.from_numpy(pr.d).to(dev))
    print(f"# batched: generated {count} problems in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    lams = [torch.empty(k, dtype=torch.float64, device=dev) for k in ns]
    Xs = [torch.empty((k, 2 * k), dtype=torch.complex128, device=dev) for k in ns]
    ws = [torch.empty(k, dtype=torch.complex128, device=dev) for k in ns]
    for i in range(warmup):
        info, rep = ctx.solve_batched_raw(ns, Acs, Bcs, lams, Xs, ds, ws, report=True, prec=prec)
        assert all(v == 0 for v in info), info
        print(f"# batched warmup {i}: {rep['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for i in range(steps):
        info, rep = ctx.solve_batched_raw(ns, Acs, Bcs, lams, Xs, ds, ws, report=True, prec=prec)
        assert all(v == 0 for v in info)
        reps.append(rep)
        print(f"# batched step {i}: {rep['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = {
        "workload": f"{count} independent problems, n log-uniform in [{lo},{hi}] (size seed {size_seed}, "
                    f"problem i seed 1000+i), {'FP32+refine' if mixed else 'FP64'}, eigenvalues + eigenvectors + weights, "
                    f"one bse_solve_batched call",
        "solves_per_s": round(count / dt, 2),
        "s_per_batch": round(dt, 4),
        "device_ms_per_batch": round(float(np.mean([r["total_ms"] for r in reps])), 2),
        "graph_replay": bool(reps[0]["graph"]),
        "sum_n3": float(sum(k ** 3 for k in ns)),
        "n_max": max(ns), "n_min": min(ns),
    }
    if reps[0]["graph"]:
        # a replayed graph records no stage events: the stage split (and the
        # rate without replay) comes from as many steps with plain launches
        ctx.set_graphs(False)
        preps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            info, rep = ctx.solve_batched_raw(ns, Acs, Bcs, lams, Xs, ds, ws, report=True, prec=prec)
            assert all(v == 0 for v in info)
            preps.append(rep)
        torch.cuda.synchronize()
        dtp = (time.perf_counter() - t0) / steps
        ctx.set_graphs(True)
        out["solves_per_s_plain_launches"] = round(count / dtp, 2)
        reps = preps
    out["stage_ms"] = {k: round(float(np.mean([r["stage_ms"][k] for r in reps])), 2) for k in reps[0]["stage_ms"]}
    return out


def serving_bench(big_inputs, count: int = 200, lo: int = 128, hi: int = 2048, big: int = 8192,
                  big_frac: float = 0.02, seed: int = 5, load: float = 0.7, pool_gib: int = 128,
                  slots: int = 4, max_batch: int = 64):
    """Serving workload: a Poisson stream of `count` requests, n log-uniform in
    [lo, hi] with probability 1 - big_frac, else n = big (stream seed `seed`,
    request i from seed 100000 + i; the n = big requests reuse the problem in
    big_inputs).  Inputs are resident in HBM before the clock starts.  Pass 1
    submits every request at once (closed loop) to find the saturation
    throughput; pass 2 replays the arrivals at `load` x that rate (open loop).
    Latency = completion - submission, from the server's own timestamps."""
    import torch
    from bse_inputs import gen_bse, serving_stream
    from paper_1501_03830_amd.api import Context, to_colmajor

    dev = torch.device("cuda", 0)
    _, ns = serving_stream(count, 1.0, lo, hi, big, big_frac, seed)
    ns = [int(k) for k in ns]
    t0 = time.time()
    inputs = []
    for i, k in enumerate(ns):
        if k == big:
            inputs.append(big_inputs)
            continue
        pr = gen_bse(k, seed=100000 + i, check_definite=False)
        inputs.append((to_colmajor(torch.from_numpy(pr.A), dev), to_colmajor(torch.from_numpy(pr.B), dev),
                       torch.from_numpy(pr.d).to(dev)))
    outs = [(torch.empty(k, dtype=torch.float64, device=dev),
             torch.empty((k, 2 * k), dtype=torch.complex128, device=dev),
             torch.empty(k, dtype=torch.complex128, device=dev)) for k in ns]
    torch.cuda.synchronize()
    print(f"# serving: {count} requests ({sum(1 for k in ns if k == big)} at n={big}) prepared in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    def run(arrivals):
        ctx = Context(0)
        ctx.serve_config(pool_gib << 30, slots, max_batch)
        pending = {}
        lat = []
        nxt = 0
        t_start = time.perf_counter()
        while nxt < count or pending:
            now = time.perf_counter() - t_start
            while nxt < count and arrivals[nxt] <= now:
                k = ns[nxt]
                Ac, Bc, d = inputs[nxt]
                lam, X, w = outs[nxt]
                pending[ctx.submit_raw(k, Ac, Bc, lam, X, d, None, w)] = nxt
                nxt += 1
            for t in list(pending):
                st, info = ctx.poll(t)
                if st >= 2:
                    assert info == 0, (pending[t], info)
                    a, _, c = ctx.ticket_times(t)
                    lat.append((c - a) * 1e-3)
                    ctx.release(t)
                    del pending[t]
            time.sleep(0.0005)
        makespan = time.perf_counter() - t_start
        stats = ctx.serve_stats()
        ctx.close()
        return makespan, lat, stats

    span1, lat1, st1 = run([0.0] * count)
    sat = count / span1
    print(f"# serving closed loop: {span1:.2f}s, {sat:.2f} solves/s", file=sys.stderr, flush=True)
    qps = load * sat
    arrivals, _ = serving_stream(count, qps, lo, hi, big, big_frac, seed)
    arrivals = [float(a) - float(arrivals[0]) for a in arrivals]
    span2, lat2, st2 = run(arrivals)
    lat2 = np.array(lat2)
    print(f"# serving open loop at {qps:.2f} req/s: {span2:.2f}s", file=sys.stderr, flush=True)
    return {
        "workload": f"{count} requests, Poisson arrivals, n log-uniform in [{lo},{hi}] w.p. {1 - big_frac:.2f} "
                    f"else n={big} (stream seed {seed}, request i seed 100000+i; n={big} requests reuse the "
                    f"single-solve problem), FP64, eigenvalues + eigenvectors + weights",
        "reduced_from": "2000 requests, n in [128,4096] + 2% at n=16384",
        "slots": slots, "max_batch": max_batch, "pool_gib": pool_gib,
        "saturation_solves_per_s": round(sat, 3),
        "load": load, "qps": round(qps, 3),
        "solves_per_s": round(count / span2, 3),
        "p50_ms": round(float(np.percentile(lat2, 50)), 2),
        "p99_ms": round(float(np.percentile(lat2, 99)), 2),
        "max_ms": round(float(lat2.max()), 2),
        "batches": st2["batches"], "max_inflight": st2["max_inflight"],
        "peak_pool_gib": round(st2["peak_used_bytes"] / 2 ** 30, 2),
    }


def serving_full(count: int = 2000, lo: int = 128, hi: int = 4096, big: int = 16384, big_frac: float = 0.02,
                 seed: int = 5, load: float = 0.7, calib: int = 200, pool_gib: int = 160, slots: int = 4,
                 max_batch: int = 64, max_span_s: float = 780.0, qps: float | None = None):
    """The serving workload as stated: a Poisson stream of `count` requests,
    n log-uniform in [lo, hi] with probability 1 - big_frac, else n = big
    (stream seed `seed`).  Requests of order <= hi are drawn on the device at
    submission (bse_inputs.device, request i from seed 100000 + i); the n = big
    requests solve one closed-form problem (exact eigenvalues known).  The
    saturation rate is measured closed-loop on the first `calib` requests of
    the stream; the timed run replays all `count` arrivals at `load` x that
    rate (open loop; the rate is raised if needed so that the arrivals span
    at most max_span_s).  A given `qps` replaces the calibration and the
    span limit.  Every result is checked: the n = big eigenvalues
    against the closed form, every other request by the residual
    ||H x_j - lambda_j x_j|| / (lambda_max ||x_j||) of all its eigenpairs
    (computed on the device after completion, outside the latency)."""
    import torch
    from bse_inputs import gen_closed_form, serving_stream
    from bse_inputs.device import gen_bse_device
    from paper_1501_03830_amd.api import Context, to_colmajor, from_colmajor

    dev = torch.device("cuda", 0)
    _, ns = serving_stream(count, 1.0, lo, hi, big, big_frac, seed)
    ns = [int(k) for k in ns]
    t0 = time.time()
    pb = gen_closed_form(big, seed=31)
    bigA = to_colmajor(torch.from_numpy(pb.A), dev)
    bigB = to_colmajor(torch.from_numpy(pb.B), dev)
    bigd = torch.from_numpy(pb.d).to(dev)
    exact = torch.from_numpy(np.asarray(pb.exact_lambda)).to(dev)
    del pb
    print(f"# serving (full): {count} requests, {sum(1 for k in ns if k == big)} at n={big}; closed-form "
          f"problem ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    def apply_H(Ac, Bc, X):
        n = Ac.shape[0]
        A = Ac.transpose(0, 1)
        B = Bc.transpose(0, 1)
        x1, x2 = X[:n], X[n:]
        return torch.cat([A @ x1 + B @ x2, -(B.conj() @ x1 + A.conj() @ x2)], 0)

    def run(arrivals, idx, check):
        ctx = Context(0)
        ctx.serve_config(pool_gib << 30, slots, max_batch)
        pending, lat, worst = {}, [], {"resid": 0.0, "big_eig": 0.0}
        nxt, done = 0, 0
        t_start = time.perf_counter()
        while nxt < len(idx) or pending:
            now = time.perf_counter() - t_start
            while nxt < len(idx) and arrivals[nxt] <= now:
                i = idx[nxt]
                k = ns[i]
                if k == big:
                    Ac, Bc, d = bigA, bigB, bigd
                else:
                    Ac, Bc, d = gen_bse_device(k, 100000 + i, dev)
                lam = torch.empty(k, dtype=torch.float64, device=dev)
                X = torch.empty((k, 2 * k), dtype=torch.complex128, device=dev)
                w = torch.empty(k, dtype=torch.complex128, device=dev)
                t = ctx.submit_raw(k, Ac, Bc, lam, X, d, None, w)
                pending[t] = (i, k, Ac, Bc, lam, X)
                nxt += 1
            for t in list(pending):
                st, info = ctx.poll(t)
                if st < 2:
                    continue
                i, k, Ac, Bc, lam, X = pending.pop(t)
                assert info == 0, (i, k, info)
                a, _, c = ctx.ticket_times(t)
                lat.append((c - a) * 1e-3)
                if check:
                    if k == big:
                        e = float((lam - exact).abs().max() / exact.max())
                        worst["big_eig"] = max(worst["big_eig"], e)
                    else:
                        Xl = from_colmajor(X)
                        R = apply_H(Ac, Bc, Xl) - Xl * lam[None, :]
                        r = (torch.linalg.vector_norm(R, dim=0) /
                             (lam.max() * torch.linalg.vector_norm(Xl, dim=0))).max()
                        worst["resid"] = max(worst["resid"], float(r))
                ctx.release(t)
                done += 1
                if done % 100 == 0:
                    print(f"# serving: {done}/{len(idx)} done, {time.perf_counter() - t_start:.0f}s",
                          file=sys.stderr, flush=True)
            time.sleep(0.0005)
        span = time.perf_counter() - t_start
        stats = ctx.serve_stats()
        ctx.close()
        return span, np.array(lat), stats, worst

    cidx = list(range(min(calib, count)))
    sat = None
    if qps is None:
        span1, _, _, _ = run([0.0] * len(cidx), cidx, False)
        sat = len(cidx) / span1
        qps = max(load * sat, count / max_span_s)
    arrivals, _ = serving_stream(count, qps, lo, hi, big, big_frac, seed)
    arrivals = [float(x) - float(arrivals[0]) for x in arrivals]
    print(f"# serving (full): calibration {sat} solves/s on {len(cidx)} requests; open loop at "
          f"{qps:.3f} req/s", file=sys.stderr, flush=True)
    span2, lat, st2, worst = run(arrivals, list(range(count)), True)
    return {
        "workload": f"{count} requests, Poisson arrivals, n log-uniform in [{lo},{hi}] w.p. {1 - big_frac:.2f} else "
                    f"n={big} (stream seed {seed}; n<= {hi} drawn on the device from seed 100000+i, n={big} the "
                    f"closed-form problem), FP64, eigenvalues + eigenvectors + weights",
        "calibration": None if sat is None else {"requests": len(cidx), "solves_per_s": round(sat, 3)},
        "load": load if sat is not None else None, "qps": round(qps, 3), "slots": slots, "max_batch": max_batch, "pool_gib": pool_gib,
        "solves_per_s": round(count / span2, 3), "makespan_s": round(span2, 1),
        "p50_ms": round(float(np.percentile(lat, 50)), 1), "p99_ms": round(float(np.percentile(lat, 99)), 1),
        "max_ms": round(float(lat.max()), 1),
        "max_relative_residual_small": worst["resid"],
        "max_rel_eig_err_big_closed_form": worst["big_eig"],
        "batches": st2["batches"], "max_inflight": st2["max_inflight"],
        "peak_pool_gib": round(st2["peak_used_bytes"] / 2 ** 30, 2),
    }


def calibrate_copy(gib: int = 1, reps: int = 5):
    """A plain device copy of a known size (gib GiB read + gib GiB written per
    launch), for scaling the HBM byte counters of rocprofv3 --pmc
    (FETCH_SIZE, WRITE_SIZE) run on the same command line."""
    import torch
    n = (gib << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy": {"bytes_read_per_launch": n * 8, "bytes_written_per_launch": n * 8,
                                         "launches": reps}}), flush=True)


def mixed_bench(ctx, n, Ac, Bc, drb, lam64, X64, steps: int, warmup: int):
    """The mixed-precision path (FP32 reduction, FP64 refinement) on the same
    resident problem, compared with the FP64 path's result lam64, X64."""
    import torch
    from paper_1501_03830_amd import _lib

    dev = Ac.device
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    X = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev)
    w = torch.empty(n, dtype=torch.complex128, device=dev)
    for i in range(warmup):
        info, rep = ctx.solve_raw(n, Ac, Bc, lam, X, drb, None, w, report=True, prec=_lib.BSE_PREC_FP32_REFINE)
        assert info == 0
        print(f"# mixed warmup {i}: {rep['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for i in range(steps):
        info, rep = ctx.solve_raw(n, Ac, Bc, lam, X, drb, None, w, report=True, prec=_lib.BSE_PREC_FP32_REFINE)
        assert info == 0
        reps.append(rep)
        print(f"# mixed step {i}: {rep['total_ms']:.1f} ms (sweeps {rep['refine_sweeps']}, first correction "
              f"{rep['refine_first_correction']:.2e})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # agreement with the FP64 path: eigenvalues relative to lambda_max, and
    # eigenvectors through |y64_j^H x_j| = 1 (y = S x, y^H x = 1 for each pair)
    lmax = float(lam64.max())
    eig = float((lam - lam64).abs().max()) / lmax
    Xm = X.transpose(0, 1)            # logical 2n x n
    X6 = X64.transpose(0, 1)
    Y6 = torch.cat([X6[:n], -X6[n:]], 0)
    dots = (Y6.conj() * Xm).sum(0).abs()
    vec = (1.0 - dots).abs()
    stage_ms = {k: float(np.mean([r["stage_ms"][k] for r in reps])) for k in reps[0]["stage_ms"]}
    return {
        "workload": f"same problem as the FP64 solve, BSE_PREC_FP32_REFINE",
        "s_per_solve": round(dt, 4),
        "vs_fp64": None,
        "device_ms": round(float(np.mean([r["total_ms"] for r in reps])), 2),
        "stage_ms": {k: round(v, 2) for k, v in stage_ms.items()},
        "stages": stage_roofline(stage_ms, stage_work(n, mixed=True, sweeps=reps[0]["refine_sweeps"])),
        "refine_sweeps": reps[0]["refine_sweeps"],
        "refine_first_correction": reps[0]["refine_first_correction"],
        "refine_last_correction": reps[0]["refine_correction"],
        "eig_err_vs_fp64_rel_lmax": eig,
        "vec_err_vs_fp64_median": float(vec.median()),
        "vec_err_vs_fp64_max": float(vec.max()),
    }


def closed_form_check(ctx, n: int, seed: int = 30):
    """Exact-eigenvalue check at the benchmark size: the closed-form
    generator (A = U0 diag(a) U0^H, B = U0 diag(b) U0^T, eigenvalues
    sqrt(a_k^2 - |b_k|^2)), solved by the one-stage and the two-stage
    reduction, eigenvalues only, and by the two-stage one with eigenvectors;
    and a real closed-form problem through Algorithm 2 with eigenvectors.  Errors are max |lambda - lambda_exact|
    relative to lambda_max (at most ||H||_2)."""
    import torch
    from bse_inputs import gen_closed_form
    from paper_1501_03830_amd import _lib
    from paper_1501_03830_amd.api import to_colmajor

    t0 = time.time()
    p = gen_closed_form(n, seed=seed)
    dev = torch.device("cuda", 0)
    Ac = to_colmajor(torch.from_numpy(p.A), dev)
    Bc = to_colmajor(torch.from_numpy(p.B), dev)
    exact = torch.from_numpy(np.asarray(p.exact_lambda)).to(dev)
    del p
    lmax = float(exact.max())
    out = {"workload": f"closed-form generator n={n} (seed {seed}), eigenvalues only", "lambda_max": lmax}
    # eigenvalue-only calls: the mixed policy runs the FP64 path for them;
    # the two-stage reduction is the third line
    for key, prec, fl in (("fp64", _lib.BSE_PREC_FP64, 0), ("fp64_two_stage", _lib.BSE_PREC_FP64, _lib.BSE_TWO_STAGE)):
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        info, rep = ctx.solve_raw(n, Ac, Bc, lam, None, None, None, None, report=True, prec=prec, extra_flags=fl)
        assert info == 0, info
        out[key] = {"max_rel_eig_err": float((lam - exact).abs().max()) / lmax,
                    "device_ms": round(rep["total_ms"], 2), "sktrd_ms": round(rep["stage_ms"]["sktrd"], 2)}
    # the two-stage reduction with eigenvectors (both stages' reflectors
    # applied back): exact eigenvalues and residuals of 32 sampled eigenpairs
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    X = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev)
    info, rep = ctx.solve_raw(n, Ac, Bc, lam, X, None, None, None, report=True, extra_flags=_lib.BSE_TWO_STAGE)
    assert info == 0, info
    A = Ac.transpose(0, 1)
    B = Bc.transpose(0, 1)
    Af = torch.tril(A) + torch.tril(A, -1).conj().transpose(0, 1)
    Bf = torch.tril(B) + torch.tril(B, -1).transpose(0, 1)
    cols = torch.arange(0, n, max(1, n // 32), device=dev)
    Xs = X[cols].transpose(0, 1)
    x1, x2 = Xs[:n], Xs[n:]
    lc = lam[cols][None, :]
    r = torch.cat([Af @ x1 + Bf @ x2 - x1 * lc, -(Bf.conj() @ x1) - (Af.conj() @ x2) - x2 * lc])
    out["fp64_two_stage_vectors"] = {
        "max_rel_eig_err": float((lam - exact).abs().max()) / lmax,
        "max_rel_residual_sampled": float(r.abs().max()) / lmax,
        "device_ms": round(rep["total_ms"], 2), "sktrd_ms": round(rep["stage_ms"]["sktrd"], 2),
        "apply_U_ms": round(rep["stage_ms"]["apply_U"], 2)}
    del X, Af, Bf, Xs, x1, x2, r
    # Algorithm 2 (real A, B) on a real closed-form problem of the same order,
    # with eigenvectors
    from bse_inputs import gen_real_closed_form
    pr = gen_real_closed_form(n, seed=41)
    exact_r = torch.from_numpy(np.asarray(pr.exact_lambda)).to(dev)
    res = ctx.solve_real(torch.from_numpy(pr.A.real.copy()), torch.from_numpy(pr.B.real.copy()),
                         vectors=True, report=True)
    assert res["info"] == 0, res["info"]
    out["real_fp64"] = {"workload": f"real closed-form generator n={n} (seed 41), bse_solve_real, eigenvalues "
                                    f"+ eigenvectors",
                        "max_rel_eig_err": float((res["lam"] - exact_r).abs().max() / exact_r.max()),
                        "device_ms": round(res["report"]["total_ms"], 2)}
    del pr, res
    print(f"# closed form n={n}: {out} ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    return out


def device_info():
    import torch
    pr = torch.cuda.get_device_properties(0)
    return {"name": pr.name, "compute_units": pr.multi_processor_count,
            "hbm_gib": round(pr.total_memory / 2 ** 30, 1), "gcn_arch": getattr(pr, "gcnArchName", None)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--s_a", type=float, default=0.3)
    ap.add_argument("--s_b", type=float, default=0.05)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--cpu-sample-n", type=str, default="256,384,512,768,1024",
                    help="comma-separated oracle sample sizes for the cube-law fit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="skip per-launch kernel events")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workload")
    ap.add_argument("--batched-only", action="store_true", help="only the batched workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision solve")
    ap.add_argument("--no-closed-form", action="store_true", help="skip the exact-eigenvalue check")
    ap.add_argument("--serving-count", type=int, default=200)
    ap.add_argument("--serving-full", action="store_true",
                    help="only the serving workload as stated (2000 requests, n in [128,4096] + 2%% at 16384)")
    ap.add_argument("--sf-count", type=int, default=2000)
    ap.add_argument("--sf-hi", type=int, default=4096)
    ap.add_argument("--sf-big", type=int, default=16384)
    ap.add_argument("--sf-calib", type=int, default=200)
    ap.add_argument("--sf-qps", type=float, default=None, help="arrival rate (skips the calibration)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    a = ap.parse_args()

    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); a multi-GPU solve is not "
              f"part of this build", file=sys.stderr)
        sys.exit(2)

    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.serving_full:
        print(json.dumps({"serving_full": serving_full(count=a.sf_count, hi=a.sf_hi, big=a.sf_big,
                                                       calib=a.sf_calib, qps=a.sf_qps)}), flush=True)
        return

    import torch
    from bse_inputs import gen_bse
    from paper_1501_03830_amd.api import Context, to_colmajor

    if a.batched_only:
        ctx = Context(0)
        print(json.dumps({"batched": batched_bench(ctx, a.steps, a.warmup)}), flush=True)
        ctx.close()
        return

    n = a.n
    t0 = time.time()
    p = gen_bse(n, s_a=a.s_a, s_b=a.s_b, seed=a.seed, check_definite=False)
    print(f"# generated n={n} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    ctx = Context(0)
    Ac = to_colmajor(torch.from_numpy(p.A), dev)
    Bc = to_colmajor(torch.from_numpy(p.B), dev)
    drb = torch.from_numpy(p.d).to(dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Xbuf = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev)
    w = torch.empty(n, dtype=torch.complex128, device=dev)
    # the timed steps run without per-launch events; the roofline of the
    # dominant kernel is measured afterwards in steps of its own
    ctx.set_timing(False)
    torch.cuda.synchronize()

    for i in range(a.warmup):
        info, rep = ctx.solve_raw(n, Ac, Bc, lam, Xbuf, drb, None, w, report=True)
        assert info == 0, f"solve returned info={info}"
        print(f"# warmup {i}: {rep['total_ms']:.1f} ms", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        info, rep = ctx.solve_raw(n, Ac, Bc, lam, Xbuf, drb, None, w, report=True)
        assert info == 0
        reps.append(rep)
        print(f"# step {i}: {rep['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s_per_solve = elapsed / a.steps

    # stage roofline: a replayed graph records no stage events, so the split
    # comes from steps with plain launches (mean over them)
    sreps = reps
    plain_ms = None
    if reps[0]["graph"]:
        ctx.set_graphs(False)
        sreps = []
        for i in range(max(1, min(2, a.steps))):
            info, rep = ctx.solve_raw(n, Ac, Bc, lam, Xbuf, drb, None, w, report=True)
            assert info == 0
            sreps.append(rep)
            print(f"# plain-launch step {i}: {rep['total_ms']:.1f} ms", file=sys.stderr, flush=True)
        ctx.set_graphs(True)
        plain_ms = float(np.mean([r["total_ms"] for r in sreps]))
    stages = stage_roofline({k: float(np.mean([r["stage_ms"][k] for r in sreps])) for k in sreps[0]["stage_ms"]},
                            stage_work(n))

    roofline = None
    if not a.no_timing:
        ctx.set_timing(True)
        treps = []
        for i in range(max(1, min(2, a.steps))):
            info, rep = ctx.solve_raw(n, Ac, Bc, lam, Xbuf, drb, None, w, report=True)
            assert info == 0
            treps.append(rep)
            print(f"# roofline step {i}: {rep['total_ms']:.1f} ms, sk_symv {rep['symv_ms']:.1f} ms over "
                  f"{rep['symv_launches']} launches", file=sys.stderr, flush=True)
        ctx.set_timing(False)
    if not a.no_timing and treps[0]["symv_launches"] > 0:
        sym_ms = float(np.mean([r["symv_ms"] for r in treps]))
        sym_bytes = treps[0]["symv_bytes"]
        launches = treps[0]["symv_launches"]
        avg_ms = sym_ms / launches
        ach = (sym_bytes / launches) / (avg_ms * 1e-3) / 1e9
        roofline = {
            "kernel": "sk_symv (tiled skew matrix-vector product, Algorithm 3 step 1)",
            "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "launches_per_step": launches, "avg_launch_us": round(avg_ms * 1e3, 3),
            "algorithmic_bytes_per_step": sym_bytes, "kernel_ms_per_step": round(sym_ms, 2),
            "measured": "hipEvents around every launch on the solver's stream, in separate steps after the "
                        "timed ones (the timed steps record no per-launch events)",
        }

    out = {
        "metric": "full BSE eigensolve s at n=8192 (FP64 vs FP32+refine); batched solves/s, p99",
        "value": round(s_per_solve, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(s_per_solve * 1e3, 2),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single BSE eigensolve n={n} (real {2 * n}x{2 * n} Hamiltonian form), FP64 path, "
                               f"all eigenvalues, right/left eigenvectors and absorption weights",
                   "n": n, "s_a": a.s_a, "s_b": a.s_b, "seed": a.seed, "precision": "fp64"},
        "solves_per_s": round(1.0 / s_per_solve, 4),
        "device_ms_per_step": round(float(np.mean([r["total_ms"] for r in reps])), 2),
        "graph_replay": bool(reps[0]["graph"]),
        "device_ms_plain_launches": None if plain_ms is None else round(plain_ms, 2),
        "stages": stages,
        "roofline": roofline,
        "cpu_baseline": None,
        "device": device_info(),
    }
    if not a.no_mixed:
        out["fp32_refine"] = mixed_bench(ctx, n, Ac, Bc, drb, lam.clone(), Xbuf.clone(), a.steps, a.warmup)
        out["fp32_refine"]["vs_fp64"] = round(s_per_solve / out["fp32_refine"]["s_per_solve"], 4)
    del Xbuf
    if not a.no_closed_form:
        out["closed_form"] = closed_form_check(ctx, n)
    if not a.no_batched:
        out["batched"] = batched_bench(ctx, a.steps, a.warmup)
        if not a.no_mixed:
            bm = batched_bench(ctx, a.steps, a.warmup, mixed=True)
            out["batched_fp32_refine"] = {k: bm[k] for k in ("workload", "solves_per_s", "s_per_batch",
                                                            "device_ms_per_batch", "stage_ms")}
    if not a.no_serving:
        out["serving"] = serving_bench((Ac, Bc, drb), count=a.serving_count, big=n)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline([int(k) for k in a.cpu_sample_n.split(",")], n, a.s_a, a.s_b)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
