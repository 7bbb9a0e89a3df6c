"""The order in which the GPU applies the bulge chase's reflectors to the
eigenvector basis (Q2 Z), checked on the CPU against the plain definition.

The chase makes reflector (s, t) (sweep s, step t) on rows
s + 1 + 64 t .. s + 64 + 64 t, and Q2 is their product in the order they are
made, so Q2 Z applies them last first, one at a time (the oracle's
reflector list, oracle/sbr.py).  The GPU instead applies groups: group
(sb, t) holds step t of the 64 sweeps 64 sb .. 64 sb + 63 as one block
reflector I - V T V^T (T from dlarft, forward); sweep blocks go last first,
and inside a block the steps go first to last.  This test restates that
schedule in numpy (blocks, steps, the group's window of 127 rows, its V and
T) and checks that it gives the same Q2 Z as the sequential definition.
"""

import numpy as np
import pytest

from oracle import sbr

B = 64


def chase_reflectors(N, seed):
    rng = np.random.default_rng(seed)
    g = np.tril(rng.standard_normal((N, N)), -1)
    Wsk = g - g.T
    band, _ = sbr.band_reduce(Wsk, B)
    _, _, refl = sbr.band_to_tridiag(band, B)
    # (s, t) of each reflector, in the order the chase made them
    out = {}
    k = 0
    for s in range(N - 2):
        r0, t = s + 1, 0
        while r0 < N - 1:
            rr0, v, tau = refl[k]
            assert rr0 == r0
            out[(s, t)] = (r0, v, tau)
            k += 1
            r0 += v.shape[0]
            t += 1
    assert k == len(refl)
    return refl, out


def apply_sequential(Z, refl):
    Z = Z.copy()
    for r0, v, tau in reversed(refl):
        sl = slice(r0, r0 + v.shape[0])
        Z[sl, :] -= tau * np.outer(v, v @ Z[sl, :])
    return Z


def apply_grouped(Z, N, refl_st):
    Z = Z.copy()
    nsb = (N - 2 + B - 1) // B if N > 2 else 0
    for sb in range(nsb - 1, -1, -1):
        s0 = B * sb
        for t in range(nsb - sb):
            R0 = s0 + 1 + B * t
            rows = np.arange(R0, min(N, R0 + 2 * B - 1))
            V = np.zeros((rows.shape[0], B))
            tau = np.zeros(B)
            for l in range(B):
                key = (s0 + l, t)
                if key not in refl_st:
                    continue
                r0, v, tv = refl_st[key]
                assert r0 == R0 + l
                V[l:l + v.shape[0], l] = v
                tau[l] = tv
            S = V.T @ V
            T = np.zeros((B, B))
            for j in range(B):
                T[:j, j] = -tau[j] * (T[:j, :j] @ S[:j, j])
                T[j, j] = tau[j]
            Zw = Z[rows, :]
            Z[rows, :] = Zw - V @ (T @ (V.T @ Zw))
    return Z


@pytest.mark.parametrize("N", [3, 4, 5, 66, 67, 130, 131, 200])
def test_grouped_order_equals_sequential(N):
    refl, refl_st = chase_reflectors(N, seed=N)
    Z = np.random.default_rng(100 + N).standard_normal((N, N))
    ref = apply_sequential(Z, refl)
    got = apply_grouped(Z, N, refl_st)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_other_orders_differ():
    """The check has teeth: applying the steps of a block last to first (or
    the sweeps of a group first to last) breaks the equality."""
    N = 200
    refl, refl_st = chase_reflectors(N, seed=7)
    Z = np.random.default_rng(8).standard_normal((N, N))
    ref = apply_sequential(Z, refl)
    # steps last to first inside each sweep block
    Zs = Z.copy()
    nsb = (N - 2 + B - 1) // B
    for sb in range(nsb - 1, -1, -1):
        for t in range(nsb - sb - 1, -1, -1):
            for l in range(B - 1, -1, -1):
                key = (B * sb + l, t)
                if key in refl_st:
                    r0, v, tau = refl_st[key]
                    sl = slice(r0, r0 + v.shape[0])
                    Zs[sl, :] -= tau * np.outer(v, v @ Zs[sl, :])
    assert np.max(np.abs(Zs - ref)) > 1e-6
    # sweeps first to last inside each group
    Zg = Z.copy()
    for sb in range(nsb - 1, -1, -1):
        for t in range(nsb - sb):
            for l in range(B):
                key = (B * sb + l, t)
                if key in refl_st:
                    r0, v, tau = refl_st[key]
                    sl = slice(r0, r0 + v.shape[0])
                    Zg[sl, :] -= tau * np.outer(v, v @ Zg[sl, :])
    assert np.max(np.abs(Zg - ref)) > 1e-6
