"""Host-only dry run of the launch plan (bse_plan_check): the sequence of
kernel launches the library would issue for a solve or a batch, checked
against the dispatch limits without a GPU, at the benchmark and serving
sizes (n = 8192 and 16384, both precision policies) and for the 256-problem
batch.  Also checks launch counts that follow from the method: one skew
matvec and one update per reflector column (N - 2 per problem of order
N = 2n), one bisection launch, and the mixed path's FP32 products."""

import ctypes

import pytest

from bse_inputs import batched_sizes
from paper_1501_03830_amd import _lib


def plan(ns, prec, flags=_lib.BSE_WANT_VECTORS | _lib.BSE_WANT_WEIGHTS):
    lib = _lib.load()
    buf = ctypes.create_string_buffer(1 << 16)
    arr = (ctypes.c_int * len(ns))(*ns)
    rc = lib.bse_plan_check(len(ns), arr, prec, flags, buf, len(buf))
    lines = buf.value.decode().strip().splitlines()
    head = lines[0].split()
    kern = {}
    for ln in lines[1:]:
        name, rest = ln.split(" launches ")
        f = rest.split()
        kern[name] = {"launches": int(f[0]), "grid_min": tuple(map(int, f[2:5])),
                      "grid_max": tuple(map(int, f[6:9])), "block_max": int(f[10]), "kernarg_max": int(f[12])}
    return rc, int(head[3]), int(head[5]), kern


def count(kern, prefix):
    return sum(v["launches"] for k, v in kern.items() if k.lstrip("(").startswith(prefix))


@pytest.mark.parametrize("n", [1, 2, 64, 2048, 8192, 16384])
@pytest.mark.parametrize("prec", [_lib.BSE_PREC_FP64, _lib.BSE_PREC_FP32_REFINE])
def test_plan_within_dispatch_limits(n, prec):
    rc, total, ws, kern = plan([n], prec)
    assert rc == 0, _lib.last_error()
    N = 2 * n
    assert count(kern, "sk_symv") == max(N - 2, 0)
    assert count(kern, "sk_update") == max(N - 2, 0)
    # one bisection launch (k_bisect<L>: L the lanes per eigenvalue as log2)
    assert count(kern, "k_bisect") == 1
    if prec == _lib.BSE_PREC_FP32_REFINE:
        assert count(kern, "gemm_f32_kernel") > 0
        assert kern["k_ref_F"]["launches"] >= 1
    else:
        assert count(kern, "gemm_f32_kernel") == 0
    for name, v in kern.items():
        assert min(v["grid_min"]) >= 1, name
        assert v["grid_max"][0] * v["block_max"] <= 0xFFFFFFFF, name
        assert v["block_max"] <= 1024, name
        assert v["kernarg_max"] <= 4096, name
    assert ws == _lib.load().bse_footprint_bytes(n, prec, 3)


@pytest.mark.parametrize("n", [1, 2, 33, 100, 2048, 8192])
def test_plan_cholesky_sub_panels(n):
    """The blocked Cholesky factorisations run one diagonal-block factor
    (k_potf2) per 64-column sub-panel and one row solve (k_trsm_rows) per
    sub-panel with rows below it: for M (order N = 2n) and for the cluster
    reorthogonalisation's Gram matrix (order n), whose second pass is issued
    always and skipped on the device when the first suffices."""
    rc, total, ws, kern = plan([n], _lib.BSE_PREC_FP64)
    assert rc == 0, _lib.last_error()
    N = 2 * n
    blocks = lambda m: (m + 63) // 64
    assert kern["k_potf2"]["launches"] == blocks(N) + 2 * blocks(n)
    assert count(kern, "k_trsm_rows<true>") == (blocks(N) - 1) + 2 * (blocks(n) - 1)


@pytest.mark.parametrize("n", [1, 2, 33, 64, 2048, 8192, 16384])
def test_plan_two_stage_with_vectors(n):
    """The two-stage reduction with eigenvectors: panels, one chase, the
    fill-zone copies, the Q2 factors of all nsb (nsb + 1) / 2 groups in one
    launch (nsb = ceil((N - 2) / 64) sweep blocks), Q2 on ceil(N / 64) column
    panels, then the block back-transformation of the band reduction's
    N - 65 reflectors; every launch within the dispatch limits."""
    rc, total, ws, kern = plan([n], _lib.BSE_PREC_FP64,
                               _lib.BSE_WANT_VECTORS | _lib.BSE_WANT_WEIGHTS | _lib.BSE_TWO_STAGE)
    assert rc == 0, _lib.last_error()
    N = 2 * n
    assert count(kern, "sk_symv") == 0
    nsb = (N - 2 + 63) // 64 if N > 2 else 0
    if nsb:
        assert kern["k_sbr_chase"]["launches"] == 1
        assert kern["k_sbr_q2T"]["launches"] == 1
        assert kern["k_sbr_q2T"]["grid_max"][0] == nsb * (nsb + 1) // 2
        assert kern["k_sbr_q2"]["grid_max"][0] == (N + 63) // 64
        assert kern["k_sbr_fill"]["launches"] == 2
    if N - 65 > 0:
        assert kern["k_extract_V"]["launches"] == (N - 65 + 255) // 256
    for name, v in kern.items():
        assert min(v["grid_min"]) >= 1, name
        assert v["grid_max"][0] * v["block_max"] <= 0xFFFFFFFF, name
        assert v["block_max"] <= 1024, name
        assert v["kernarg_max"] <= 4096, name


@pytest.mark.parametrize("prec", [_lib.BSE_PREC_FP64, _lib.BSE_PREC_FP32_REFINE])
def test_plan_of_the_256_problem_batch(prec):
    ns = [int(k) for k in batched_sizes(256, 64, 1024, seed=4)]
    rc, total, ws, kern = plan(ns, prec)
    assert rc == 0, _lib.last_error()
    # one launch per reflector column of the largest problem serves the batch
    assert count(kern, "sk_symv") == 2 * max(ns) - 2
    assert ws == _lib.load().bse_footprint_batched_bytes(len(ns), (ctypes.c_int * len(ns))(*ns), prec, 3)


def test_plan_eigenvalues_only_skips_vectors():
    rc, total, ws, kern = plan([4096], _lib.BSE_PREC_FP64, flags=0)
    assert rc == 0
    assert "k_invit" not in kern and "k_finish_X" not in kern


def test_plan_rejects_bad_arguments():
    lib = _lib.load()
    arr = (ctypes.c_int * 1)(0)
    assert lib.bse_plan_check(1, arr, 0, 0, None, 0) == -2
    arr = (ctypes.c_int * 1)(8)
    assert lib.bse_plan_check(1, arr, 7, 0, None, 0) == -3
    assert lib.bse_plan_check(0, arr, 0, 0, None, 0) == -1
