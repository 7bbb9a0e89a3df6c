"""Write the stored expected values used by the GPU parity tests.

Every value here comes from the CPU oracle (oracle/) applied to the seeded
generator (bse_inputs/); nothing is read from the GPU path.  Run from the
repository root:

    python tests/golden/make_golden.py [--n 2048] [--seed 2]

The dense config-2 problem (n = 2048, A = diag(U[1,10]) + 0.1/sqrt(n) GUE-like
kernel, B = 0.05/sqrt(n) complex-symmetric Gaussian, unit complex dipole
d_r = d_l) takes a few minutes of CPU time in the unblocked oracle, which is
why its results are stored rather than recomputed inside a GPU test.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from bse_inputs import gen_bse  # noqa: E402

SAMPLE_COLS = [0, 1, 2, 511, 1023, 1024, 1536, 2046, 2047]
SAMPLE_ROWS = 64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--s_a", type=float, default=0.1)
    ap.add_argument("--s_b", type=float, default=0.05)
    a = ap.parse_args()
    p = gen_bse(a.n, s_a=a.s_a, s_b=a.s_b, seed=a.seed)
    t0 = time.time()
    r = oracle.solve(p.A, p.B, p.d)
    dt = time.time() - t0
    assert r.info == 0
    tag = f"config2_n{a.n}_seed{a.seed}"
    np.savetxt(os.path.join(HERE, f"{tag}_lambda.txt"), r.lam, fmt="%.17e",
               header=f"oracle eigenvalues, gen_bse(n={a.n}, s_a={a.s_a}, s_b={a.s_b}, seed={a.seed})")
    np.savetxt(os.path.join(HERE, f"{tag}_weights.txt"), np.column_stack([r.w.real, r.w.imag]), fmt="%.17e",
               header="oracle absorption weights w_j (re, im), d_r = d_l = generator dipole")
    rng = np.random.default_rng(123)
    cols = [c for c in SAMPLE_COLS if c < a.n]
    rows = np.sort(rng.choice(2 * a.n, size=min(SAMPLE_ROWS, 2 * a.n), replace=False))
    samp = r.X[np.ix_(rows, cols)]
    meta = {"n": a.n, "seed": a.seed, "s_a": a.s_a, "s_b": a.s_b, "oracle_seconds": dt,
            "sample_cols": cols, "sample_rows": rows.tolist(),
            "x_re": samp.real.tolist(), "x_im": samp.imag.tolist(),
            "note": "entries of oracle eigenvectors (canonical phase) at sampled rows/cols"}
    with open(os.path.join(HERE, f"{tag}_vectors.json"), "w") as f:
        json.dump(meta, f)
    print(f"wrote {tag} in {dt:.1f}s")


if __name__ == "__main__":
    main()
