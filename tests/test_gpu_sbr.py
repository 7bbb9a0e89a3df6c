"""Two-stage skew tridiagonalisation (BSE_TWO_STAGE, bse_sktrd2: dense to
band on the matrix cores, then bulge chasing) against the oracle, through the
C ABI.

Both the one-stage and the two-stage reduction keep U e_1 = e_1, so by the
implicit-Q argument they give the same |alpha| (tolerance 1e-10 of max|alpha|:
forward errors of the two reductions, ~N eps kappa, at the sizes here), and
the same eigenvalues (1e-13 lambda_max end to end, as the one-stage parity
tests).  Sizes span one and several 64-column panels with ragged tails;
random skew matrices of odd order check the reduction alone.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import bse_oracle as bo
from bse_inputs import gen_bse, gen_closed_form

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def tt(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def npc(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    from paper_1501_03830_amd.api import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 2, 33, 64, 65, 100, 150])
def test_sktrd2_alpha_matches_one_stage(ctx, n):
    say(f"[sktrd2] n={n}")
    p = gen_bse(n, seed=30 + n)
    Lo, _ = bo.cholesky(bo.build_M(p.A, p.B))
    Wo = bo.form_W(Lo)
    ao, _, _ = bo.skew_tridiagonalize(Wo)
    a2 = npc(ctx.sktrd2(tt(Wo)))
    d = float(np.max(np.abs(np.abs(a2) - np.abs(ao)))) / float(np.max(np.abs(ao)))
    lam_o = bo.bisect_positive(ao)
    lam, _ = ctx.tridiag_eig(torch.from_numpy(a2), vectors=False)
    el = float(np.max(np.abs(npc(lam) - lam_o))) / float(lam_o.max())
    say(f"  |alpha| {d:.2e}  eigenvalues {el:.2e}")
    assert d <= 1e-10 and el <= 1e-13


@pytest.mark.parametrize("N", [3, 5, 129, 131, 257])
def test_sktrd2_random_skew(ctx, N):
    g = np.random.default_rng(N).standard_normal((N, N))
    W = g - g.T
    ao, _, _ = bo.skew_tridiagonalize(W)
    a2 = npc(ctx.sktrd2(tt(W)))
    d = float(np.max(np.abs(np.abs(a2) - np.abs(ao)))) / float(np.max(np.abs(ao)))
    say(f"[sktrd2] random skew N={N}: |alpha| {d:.2e}")
    assert d <= 1e-10


@pytest.mark.parametrize("n", [1, 2, 33, 64, 100, 300])
def test_two_stage_solve_matches_oracle(ctx, n):
    from paper_1501_03830_amd import _lib
    p = gen_bse(n, s_a=0.3, s_b=0.05, seed=800 + n)
    r = ctx.solve(tt(p.A), tt(p.B), vectors=False, extra_flags=_lib.BSE_TWO_STAGE)
    assert r["info"] == 0
    lo = oracle.solve(p.A, p.B).lam
    el = float(np.max(np.abs(npc(r["lam"]) - lo))) / float(lo.max())
    say(f"[two-stage solve] n={n}: eig {el:.2e}")
    assert el <= 1e-13


@pytest.mark.parametrize("n", [2048, 8192])
def test_two_stage_closed_form(ctx, n):
    from paper_1501_03830_amd import _lib
    p = gen_closed_form(n, seed=30)
    exact = np.asarray(p.exact_lambda)
    r = ctx.solve(tt(p.A), tt(p.B), vectors=False, extra_flags=_lib.BSE_TWO_STAGE, report=True)
    assert r["info"] == 0
    err = float(np.max(np.abs(npc(r["lam"]) - exact))) / float(exact.max())
    say(f"[two-stage closed form] n={n}: eig {err:.2e}, {r['report']['total_ms']:.1f} ms "
        f"(sktrd {r['report']['stage_ms']['sktrd']:.1f} ms)")
    assert err <= 1e-10


@pytest.mark.parametrize("n", [300, 2048])
def test_two_stage_after_mixed_solve(ctx, n):
    """Regression: a mixed-precision solve leaves its refinement state word
    (the sweep it converged in) in the context's workspace header.  The
    two-stage products once took it for theirs and skipped every panel past
    that sweep number, so a two-stage solve after a mixed one on the same
    context returned wrong eigenvalues.  Same context and order; the mixed
    solve afterwards must give the same bits as before."""
    from paper_1501_03830_amd import _lib
    p = gen_closed_form(n, seed=32)
    exact = np.asarray(p.exact_lambda)
    A, B = tt(p.A), tt(p.B)
    mixed = ctx.solve(A, B, vectors=True, prec=_lib.BSE_PREC_FP32_REFINE, report=True)
    assert mixed["info"] == 0 and mixed["report"]["refine_sweeps"] >= 1
    for rep in range(2):
        r = ctx.solve(A, B, vectors=False, extra_flags=_lib.BSE_TWO_STAGE)
        assert r["info"] == 0
        err = float(np.max(np.abs(npc(r["lam"]) - exact))) / float(exact.max())
        say(f"[two-stage after mixed] n={n} call {rep}: eig {err:.2e}")
        assert err <= 1e-10
    mixed2 = ctx.solve(A, B, vectors=True, prec=_lib.BSE_PREC_FP32_REFINE)
    assert torch.equal(mixed2["lam"], mixed["lam"]) and torch.equal(mixed2["X"], mixed["X"])


def _check_vectors(A, B, d, r, ro, tag):
    """Eigenvalues, eigenvectors (up to phase and cluster span), the residual
    and normalisation metrics and the weights against the oracle, with the
    one-stage parity suite's tolerances."""
    from oracle import metrics
    lam, X, w = npc(r["lam"]), npc(r["X"]), npc(r["w"])
    As, Bs = bo.symmetrize_lower(A, B)
    normH = np.linalg.norm(metrics.H_matrix(As, Bs), 2)
    el = float(np.max(np.abs(lam - ro.lam))) / normH
    gap = 1e-6 * normH
    ev = metrics.compare_eigvecs(ro.X, X, ro.lam, gap)
    r1, r2 = metrics.table1_metrics(As, Bs, lam, X)
    we = metrics.compare_weights(ro.w, w, ro.lam, gap)
    say(f"  {tag}: eig {el:.2e} vec {ev:.2e} table1 {r1:.2e} {r2:.2e} weights {we:.2e}")
    assert el <= 1e-13
    assert ev <= 1e-9
    assert r1 <= 1e-12 and r2 <= 1e-12
    assert metrics.normalization_error(X) <= 1e-12
    assert we <= 1e-10


@pytest.mark.parametrize("n", [1, 2, 3, 33, 64, 65, 100, 200])
def test_two_stage_vectors_match_oracle(ctx, n):
    """Eigenvectors through both stages' reflectors (the chase's as 64-sweep
    block reflectors, then the band reduction's at row offset 64): the same
    bar as the one-stage path.  Orders below and above one sweep block, one
    band and several of each."""
    from paper_1501_03830_amd import _lib
    p = gen_bse(n, s_a=0.3, s_b=0.05, seed=900 + n)
    ro = oracle.solve(p.A, p.B, p.d)
    r = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), extra_flags=_lib.BSE_TWO_STAGE)
    assert r["info"] == 0
    _check_vectors(p.A, p.B, p.d, r, ro, f"[two-stage vectors] n={n}")


def test_two_stage_vectors_equal_one_stage(ctx):
    """n = 300 (N = 600: ten sweep blocks, nine bands): the two paths'
    eigenvectors agree to the forward error of the two reductions."""
    from paper_1501_03830_amd import _lib
    from oracle import metrics
    p = gen_bse(300, s_a=0.3, s_b=0.05, seed=77)
    A, B = tt(p.A), tt(p.B)
    r1 = ctx.solve(A, B)
    r2 = ctx.solve(A, B, extra_flags=_lib.BSE_TWO_STAGE)
    lam1 = npc(r1["lam"])
    el = float(np.max(np.abs(npc(r2["lam"]) - lam1))) / float(lam1.max())
    ev = metrics.compare_eigvecs(npc(r1["X"]), npc(r2["X"]), lam1, 1e-6 * float(lam1.max()))
    rr1, rr2 = metrics.table1_metrics(*bo.symmetrize_lower(p.A, p.B), npc(r2["lam"]), npc(r2["X"]))
    say(f"[two-stage vs one-stage] n=300: eig {el:.2e} vec {ev:.2e} table1 {rr1:.2e} {rr2:.2e}")
    assert el <= 1e-13 and ev <= 1e-9 and rr1 <= 1e-12 and rr2 <= 1e-12


def test_two_stage_vectors_closed_form_2048(ctx):
    """n = 2048 with eigenvectors: exact eigenvalues, and the eigenpairs'
    residual certificate on a sample of columns."""
    from paper_1501_03830_amd import _lib
    from oracle import metrics
    p = gen_closed_form(2048, seed=33)
    exact = np.asarray(p.exact_lambda)
    r = ctx.solve(tt(p.A), tt(p.B), extra_flags=_lib.BSE_TWO_STAGE, report=True)
    assert r["info"] == 0
    lam, X = npc(r["lam"]), npc(r["X"])
    err = float(np.max(np.abs(lam - exact))) / float(exact.max())
    As, Bs = bo.symmetrize_lower(p.A, p.B)
    H = metrics.H_matrix(As, Bs)
    cols = np.random.default_rng(5).choice(2048, 48, replace=False)
    res = max(float(np.linalg.norm(H @ X[:, j] - lam[j] * X[:, j]) / np.linalg.norm(X[:, j])) for j in cols)
    res /= float(exact.max())
    say(f"[two-stage vectors closed form] n=2048: eig {err:.2e} residual {res:.2e}, "
        f"{r['report']['total_ms']:.1f} ms (apply_U {r['report']['stage_ms']['apply_U']:.1f} ms)")
    assert err <= 1e-10 and res <= 1e-12


def test_two_stage_vectors_closed_form_8192(ctx):
    """The benchmark order (n = 8192, N = 16384) through the two-stage
    reduction with eigenvectors, in the launch configuration the benchmark
    uses: exact eigenvalues, and the residuals of 32 sampled eigenpairs
    computed on the device from the logical A and B."""
    from paper_1501_03830_amd import _lib
    from paper_1501_03830_amd.api import to_colmajor
    n = 8192
    p = gen_closed_form(n, seed=30)
    dev = torch.device("cuda", 0)
    Ac = to_colmajor(torch.from_numpy(p.A), dev)
    Bc = to_colmajor(torch.from_numpy(p.B), dev)
    exact = torch.from_numpy(np.asarray(p.exact_lambda)).to(dev)
    del p
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    X = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev)
    info, rep = ctx.solve_raw(n, Ac, Bc, lam, X, report=True, extra_flags=_lib.BSE_TWO_STAGE)
    assert info == 0
    lmax = float(exact.max())
    err = float((lam - exact).abs().max()) / lmax
    A = Ac.transpose(0, 1)
    B = Bc.transpose(0, 1)
    Af = torch.tril(A) + torch.tril(A, -1).conj().transpose(0, 1)
    Bf = torch.tril(B) + torch.tril(B, -1).transpose(0, 1)
    cols = torch.arange(0, n, n // 32, device=dev)
    Xs = X[cols].transpose(0, 1)
    x1, x2 = Xs[:n], Xs[n:]
    lc = lam[cols][None, :]
    r = torch.cat([Af @ x1 + Bf @ x2 - x1 * lc, -(Bf.conj() @ x1) - (Af.conj() @ x2) - x2 * lc])
    res = float(r.abs().max()) / lmax
    say(f"[two-stage vectors] n={n}: eig {err:.2e} sampled residual {res:.2e}, {rep['total_ms']:.0f} ms")
    assert err <= 1e-10 and res <= 1e-12


def test_two_stage_with_twisted_vectors(ctx):
    """BSE_TWO_STAGE together with BSE_EIGVEC_TWISTED: the tridiagonal
    eigenvectors by twisted factorisations, back through both stages."""
    from paper_1501_03830_amd import _lib
    for n in (50, 130):
        p = gen_bse(n, s_a=0.3, s_b=0.05, seed=950 + n)
        ro = oracle.solve(p.A, p.B, p.d)
        r = ctx.solve(tt(p.A), tt(p.B), d_r=tt(p.d), extra_flags=_lib.BSE_TWO_STAGE | _lib.BSE_EIGVEC_TWISTED)
        assert r["info"] == 0
        _check_vectors(p.A, p.B, p.d, r, ro, f"[two-stage + twisted] n={n}")


def test_two_stage_real_path(ctx):
    """Algorithm 2 (real A, B) through the two-stage reduction and its
    back-transformation: eigenvalues, eigenvectors and weights against the
    real oracle."""
    from paper_1501_03830_amd import _lib
    from bse_inputs import gen_real
    from oracle import metrics
    n = 120
    p = gen_real(n, seed=12)
    lo, Xo, info = oracle.solve_real(p.A, p.B)
    assert info == 0
    r = ctx.solve_real(tt(p.A.real), tt(p.B.real), d_r=tt(p.d), extra_flags=_lib.BSE_TWO_STAGE)
    assert r["info"] == 0
    lam, X, w = npc(r["lam"]), npc(r["X"]), npc(r["w"])
    normH = float(lo.max())
    el = float(np.max(np.abs(lam - lo))) / normH
    ev = metrics.compare_eigvecs(Xo.astype(np.complex128), X.astype(np.complex128), lo, 1e-6 * normH)
    wo = oracle.absorption_weights(Xo.astype(np.complex128), p.d, p.d)
    we = metrics.compare_weights(wo, w, lo, 1e-6 * normH)
    say(f"[two-stage real] n={n}: eig {el:.2e} vec {ev:.2e} w {we:.2e}")
    assert el <= 1e-13 and ev <= 1e-9 and we <= 1e-10


def test_two_stage_flag_limits(ctx):
    from paper_1501_03830_amd import _lib
    p = gen_bse(20, seed=3)
    with pytest.raises(_lib.BseError) as e:
        ctx.solve(tt(p.A), tt(p.B), vectors=False, prec=_lib.BSE_PREC_FP32_REFINE, extra_flags=_lib.BSE_TWO_STAGE)
    assert e.value.code == _lib.BSE_EUNSUPPORTED
    with pytest.raises(_lib.BseError) as e:
        ctx.solve(tt(p.A), tt(p.B), vectors=True, prec=_lib.BSE_PREC_FP32_REFINE, extra_flags=_lib.BSE_TWO_STAGE)
    assert e.value.code == _lib.BSE_EUNSUPPORTED
