"""Autotuner of the tile table of the tridiagonalisation's skew matrix-vector
kernel (row tiles per strip workgroup, by trailing size bucket and storage
type; bse_set_tile_table).

    python -m paper_1501_03830_amd.autotune [--out tuning.json] [--quick]

Coordinate descent over the table's tile counts, on the workloads they
decide: the bottom bucket (below 33 row blocks, every problem of the batched
workload) on that workload (256 problems, n log-uniform in [64, 1024], FP64
and FP32 + refinement), the four buckets above it on single n = 8192 solves
(FP64 and FP32 + refinement; the reduction's own time).  Each candidate is timed as the median device time
of a few calls after a warm-up; a bucket keeps its current count unless a
candidate is at least 1% faster.  The chosen table, the device and every
measurement are written to the output (JSON), which the Python binding
applies to each context it creates (tuning.json next to this file).
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_OUT = os.path.join(HERE, "tuning.json")

# bucket layout of a table row: [t0 t1 t2 t3 v0 v1 v2 v3 v4]
SMALL_SPLIT = 33      # t3: batched problems (n <= 1024) have nblk <= 32
CANDIDATES = {"small": [2, 3, 4, 6, 8], "mid": [3, 4, 6, 8], "large": [8, 12, 16]}


def get_table(lib):
    t = (ctypes.c_int * 18)()
    assert lib.bse_get_tile_table(t) == 0
    return [list(t[:9]), list(t[9:])]


def set_table(lib, ctx, table):
    arr = (ctypes.c_int * 18)(*(table[0] + table[1]))
    rc = lib.bse_set_tile_table(ctx.h, arr)
    if rc != 0:
        from . import _lib
        raise RuntimeError(f"bse_set_tile_table: {rc} {_lib.last_error()}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="batched buckets only")
    a = ap.parse_args()

    sys.path.insert(0, ROOT)
    import torch
    from bse_inputs import gen_bse, batched_sizes
    from . import _lib
    from .api import Context, to_colmajor

    ctx = Context(0, apply_tuning=False)
    lib = ctx.lib
    dev = ctx.device
    table = get_table(lib)
    # Split the bottom bucket at SMALL_SPLIT so that the batched sizes get
    # counts of their own, keeping every other size's count: a row whose
    # lowest threshold in use is t2 (t3 = 0) gets t3 = SMALL_SPLIT; one that
    # already ends at t1 (t2 = t3 = 0) moves its bottom count to v3 and leaves
    # the v2 bucket empty (t2 = t1).
    for row in table:
        if row[3] == 0:
            if row[2] == 0:
                row[2], row[7], row[6] = row[1], row[6], row[5]
            row[3] = SMALL_SPLIT
            row[8] = row[7]
    set_table(lib, ctx, table)

    def bucket_used(row, slot):
        """v_i (slot 4 + i) covers [t_i, t_{i-1}): empty when they are equal."""
        i = slot - 4
        hi = row[i - 1] if i > 0 else 1 << 30
        lo = row[i] if i < 4 else 0
        return hi > lo

    # the batched workload, resident in HBM
    ns = [int(k) for k in batched_sizes(256, 64, 1024, seed=4)]
    Acs, Bcs, ds = [], [], []
    for i, k in enumerate(ns):
        p = gen_bse(k, s_a=0.1, s_b=0.05, seed=1000 + i, check_definite=False)
        Acs.append(to_colmajor(torch.from_numpy(p.A), dev))
        Bcs.append(to_colmajor(torch.from_numpy(p.B), dev))
        ds.append(torch.from_numpy(p.d).to(dev))
    lams = [torch.empty(k, dtype=torch.float64, device=dev) for k in ns]
    Xs = [torch.empty((k, 2 * k), dtype=torch.complex128, device=dev) for k in ns]
    ws = [torch.empty(k, dtype=torch.complex128, device=dev) for k in ns]
    big = None
    if not a.quick:
        p = gen_bse(8192, s_a=0.3, s_b=0.05, seed=3, check_definite=False)
        big = (to_colmajor(torch.from_numpy(p.A), dev), to_colmajor(torch.from_numpy(p.B), dev))
        del p
    lam8 = torch.empty(8192, dtype=torch.float64, device=dev)
    X8 = torch.empty((8192, 16384), dtype=torch.complex128, device=dev) if big is not None else None

    def time_batched(prec):
        ms = []
        for r in range(a.reps + 1):
            info, rep = ctx.solve_batched_raw(ns, Acs, Bcs, lams, Xs, ds, ws, report=True, prec=prec)
            assert all(v == 0 for v in info)
            if r > 0:
                ms.append(rep["total_ms"])
        return float(np.median(ms))

    def time_single(prec):
        # plain launches, so that the reduction's own stage events are recorded
        ctx.set_graphs(False)
        ms = []
        for r in range(2):
            info, rep = ctx.solve_raw(8192, big[0], big[1], lam8, X8, report=True, prec=prec)
            assert info == 0
            ms.append(rep["stage_ms"]["sktrd"])
        ctx.set_graphs(True)
        return float(np.median(ms))

    log = []
    precs = [("fp64", _lib.BSE_PREC_FP64, 0), ("fp32_refine", _lib.BSE_PREC_FP32_REFINE, 1)]
    # the bottom bucket v4 (nblk < t3: every batched problem) on the batched
    # workload
    for name, prec, row in precs:
        for slot in (8,):
            if not bucket_used(table[row], slot):
                continue
            best_v = table[row][slot]
            set_table(lib, ctx, table)
            best_ms = time_batched(prec)
            log.append({"workload": "batched", "prec": name, "slot": slot, "tiles": best_v, "ms": best_ms})
            for v in CANDIDATES["small"]:
                if v == table[row][slot]:
                    continue
                trial = [r[:] for r in table]
                trial[row][slot] = v
                set_table(lib, ctx, trial)
                ms = time_batched(prec)
                log.append({"workload": "batched", "prec": name, "slot": slot, "tiles": v, "ms": ms})
                print(f"# batched {name} slot {slot} tiles {v}: {ms:.2f} ms (best {best_ms:.2f})", flush=True)
                if ms < 0.99 * best_ms:
                    best_ms, best_v = ms, v
            table[row][slot] = best_v
    # v0 .. v3 on single n = 8192 solves (the reduction): trailing orders
    # from 16384 down to about 2100
    if big is not None:
        for name, prec, row in precs:
            for slot in (4, 5, 6, 7):
                if not bucket_used(table[row], slot):
                    continue
                best_v = table[row][slot]
                set_table(lib, ctx, table)
                best_ms = time_single(prec)
                log.append({"workload": "n8192", "prec": name, "slot": slot, "tiles": best_v, "ms": best_ms})
                for v in CANDIDATES["mid" if slot == 7 else "large"]:
                    if v == table[row][slot]:
                        continue
                    trial = [r[:] for r in table]
                    trial[row][slot] = v
                    set_table(lib, ctx, trial)
                    ms = time_single(prec)
                    log.append({"workload": "n8192", "prec": name, "slot": slot, "tiles": v, "ms": ms})
                    print(f"# n=8192 {name} slot {slot} tiles {v}: {ms:.1f} ms (best {best_ms:.1f})", flush=True)
                    if ms < 0.99 * best_ms:
                        best_ms, best_v = ms, v
                table[row][slot] = best_v
    set_table(lib, ctx, table)
    pr = torch.cuda.get_device_properties(0)
    out = {
        "what": "tile table of the skew matrix-vector kernel (bse_set_tile_table): rows FP64, FP32; "
                "[t0 t1 t2 t3 v0 v1 v2 v3 v4]: nblk >= t0 -> v0, >= t1 -> v1, >= t2 -> v2, >= t3 -> v3, else v4",
        "table": table,
        "device": {"name": pr.name, "gcn_arch": getattr(pr, "gcnArchName", None),
                   "compute_units": pr.multi_processor_count},
        "command": "python -m paper_1501_03830_amd.autotune" + (" --quick" if a.quick else ""),
        "date": time.strftime("%Y-%m-%d"),
        "measurements": log,
    }
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"table": table}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
