"""bse_solve_noalloc (the solve on the library's fixed workspace array, for
callers that cannot allocate) against bse_solve, through the C ABI.

Two calls in a row, the second on a smaller problem, so that the second runs
on the array as the first left it; eigenvalues, eigenvectors and weights
must equal bse_solve's bit for bit (the same kernels with the same launch
shapes).  A problem whose workspace exceeds the array is rejected.
"""

import numpy as np
import pytest
import torch

from bse_inputs import gen_bse

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def tt(a):
    return torch.from_numpy(np.ascontiguousarray(a))


@pytest.fixture(scope="module")
def ctx():
    from paper_1501_03830_amd.api import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec_name", ["fp64", "fp32_refine"])
def test_noalloc_equals_solve_two_calls(ctx, prec_name):
    from paper_1501_03830_amd import _lib
    prec = _lib.BSE_PREC_FP64 if prec_name == "fp64" else _lib.BSE_PREC_FP32_REFINE
    sizes = (300, 97) if prec_name == "fp64" else (250, 70)
    for k, n in enumerate(sizes):
        p = gen_bse(n, s_a=0.3, s_b=0.05, seed=4100 + k)
        say(f"[noalloc] {prec_name} call {k + 1}: n={n}")
        a = ctx.solve_noalloc(tt(p.A), tt(p.B), d_r=tt(p.d), prec=prec)
        torch.cuda.synchronize()
        b = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), prec=prec)
        torch.cuda.synchronize()
        assert a["info"] == 0 and b["info"] == 0
        assert torch.equal(a["lam"], b["lam"])
        assert torch.equal(a["X"], b["X"])
        assert torch.equal(a["w"], b["w"])
        # eigenvalue-only call on the same array (the mixed policy runs the
        # FP64 path for it, as bse_solve does)
        c = ctx.solve_noalloc(tt(p.A), tt(p.B), vectors=False, prec=prec)
        torch.cuda.synchronize()
        e = ctx.solve(tt(p.A), tt(p.B), vectors=False, prec=prec)
        torch.cuda.synchronize()
        assert c["info"] == 0 and torch.equal(c["lam"], e["lam"])


def test_noalloc_two_stage_equals_solve(ctx):
    """The two-stage reduction with eigenvectors on the fixed array (its
    chase reflectors, fill-zone copy and Q2 factors all live in the
    problem's workspace): bit for bit bse_solve with the same flag, on two
    calls in a row, the second smaller."""
    from paper_1501_03830_amd import _lib
    for k, n in enumerate((260, 90)):
        p = gen_bse(n, s_a=0.3, s_b=0.05, seed=4200 + k)
        say(f"[noalloc] two-stage call {k + 1}: n={n}")
        a = ctx.solve_noalloc(tt(p.A), tt(p.B), d_r=tt(p.d), extra_flags=_lib.BSE_TWO_STAGE)
        torch.cuda.synchronize()
        b = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), extra_flags=_lib.BSE_TWO_STAGE)
        torch.cuda.synchronize()
        assert a["info"] == 0 and b["info"] == 0
        assert torch.equal(a["lam"], b["lam"])
        assert torch.equal(a["X"], b["X"])
        assert torch.equal(a["w"], b["w"])


def test_noalloc_rejects_oversized(ctx):
    from paper_1501_03830_amd import _lib
    lib = ctx.lib
    cap = lib.bse_noalloc_max_bytes()
    assert cap == 64 << 20
    # the limits stated in the header
    assert lib.bse_footprint_bytes(544, _lib.BSE_PREC_FP64, 3) <= cap
    assert lib.bse_footprint_bytes(545, _lib.BSE_PREC_FP64, 3) > cap
    assert lib.bse_footprint_bytes(416, _lib.BSE_PREC_FP32_REFINE, 3) <= cap
    assert lib.bse_footprint_bytes(417, _lib.BSE_PREC_FP32_REFINE, 3) > cap
    n = 545
    dev = ctx.device
    A = torch.zeros((n, n), dtype=torch.complex128, device=dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    rc = lib.bse_solve_noalloc(ctx.h, n, A.data_ptr(), n, A.data_ptr(), n, _lib.BSE_PREC_FP64, 0,
                               lam.data_ptr(), None, 2 * n, None, None, None)
    assert rc == _lib.BSE_ENOMEM
    assert "no-alloc" in _lib.last_error()
