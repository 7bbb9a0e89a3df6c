"""Pins of the Tamm-Dancoff and spectra oracle (oracle/spectra.py) to what
the paper and the mathematics fix, each chosen so that a plausible slip
fails at least one of them (checked below on planted mutants):

* the TDA eigenpairs are the B = 0 case of Algorithm 1: oracle.solve(A, 0)
  (an independent route through the embedding, Cholesky, W and the skew
  tridiagonalisation) gives the same eigenvalues and, per eigenvalue, the
  same weights;
* Theorem 4: lambda_j(H) <= lambda_j(A);
* eq. DOS normalisation: the broadened density integrates to 1 (each
  Gaussian to 1, 2n of them, divided by 2n), is even in omega (the +-lambda
  pairs of Theorem 3) and peaks at 1/(2 sqrt(2 pi) sigma) for n = 1;
* eq. absp: the broadened absorption spectrum integrates to sum_j w_j and
  peaks at w/(sqrt(2 pi) sigma) for n = 1.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import spectra
from bse_inputs import gen_bse

GRID = np.linspace(-14.0, 14.0, 56001)   # step 5e-4


def pins_dos(dos_fn, lam, sigma):
    out = []
    phi = dos_fn(lam, GRID, sigma)
    integ = float(np.trapezoid(phi, GRID))
    out.append(("DOS integrates to 1", abs(integ - 1.0) <= 1e-9, integ))
    sym = float(np.max(np.abs(phi - phi[::-1])))
    out.append(("DOS even", sym <= 1e-12 * float(phi.max()), sym))
    one = dos_fn(np.array([3.0]), np.array([3.0]), sigma)[0]
    want = 1.0 / (2.0 * math.sqrt(2.0 * math.pi) * sigma)
    out.append(("DOS peak n=1", abs(one - want) <= 1e-12 * want, one))
    return out


def pins_absorption(abs_fn, lam, w, sigma):
    out = []
    e = abs_fn(lam, w, GRID, sigma)
    integ = complex(np.trapezoid(e, GRID))
    out.append(("absorption integrates to sum w", abs(integ - w.sum()) <= 1e-9 * abs(w.sum()), integ))
    one = abs_fn(np.array([3.0]), np.array([0.5 + 0.25j]), np.array([3.0]), sigma)[0]
    want = (0.5 + 0.25j) / (math.sqrt(2.0 * math.pi) * sigma)
    out.append(("absorption peak n=1", abs(one - want) <= 1e-12 * abs(want), one))
    return out


def test_tda_is_algorithm1_with_b_zero():
    for n in (1, 5, 40, 90):
        p = gen_bse(n, s_a=0.3, s_b=0.05, seed=60 + n)
        lam, X, w = spectra.tda_solve(p.A, p.d)
        r = oracle.solve(p.A, np.zeros_like(p.B), p.d)
        assert r.info == 0
        normH = float(lam.max())
        assert np.max(np.abs(lam - r.lam)) <= 1e-12 * normH
        # eigenvectors: x_j = [v_j; 0], A v = lambda v, unit v
        a, _ = oracle.symmetrize_lower(p.A, p.B)
        assert np.max(np.abs(X[n:])) == 0.0
        assert np.max(np.abs(a @ X[:n] - X[:n] * lam)) <= 1e-12 * normH
        assert np.max(np.abs(np.linalg.norm(X[:n], axis=0) - 1.0)) <= 1e-13
        assert oracle.metrics.compare_eigvecs(r.X, X, r.lam, 1e-6 * normH) <= 1e-9
        assert oracle.metrics.compare_weights(r.w, w, r.lam, 1e-6 * normH) <= 1e-10


def test_theorem4_tda_overestimates():
    for n, s_a in ((30, 0.3), (120, 0.3), (200, 0.1)):
        p = gen_bse(n, s_a=s_a, s_b=0.05, seed=70 + n)
        lam_tda = spectra.tda_solve(p.A)[0]
        lam_full = oracle.solve(p.A, p.B).lam
        # both ascending: the j-th largest of each pair up
        assert np.all(lam_full <= lam_tda + 1e-13 * lam_tda.max())
        assert np.max(lam_tda - lam_full) > 1e-6   # B = 0 is not a no-op


@pytest.mark.parametrize("sigma", [0.05, 0.2])
def test_spectra_pins(sigma):
    p = gen_bse(12, s_a=0.3, s_b=0.05, seed=5)
    r = oracle.solve(p.A, p.B, p.d)
    for name, ok, val in pins_dos(spectra.dos, r.lam, sigma) + pins_absorption(spectra.absorption, r.lam, r.w, sigma):
        assert ok, (name, val)


# planted mistakes: each must fail at least one pin
def _dos_over_n(lam, om, s):
    return spectra.dos(lam, om, s) * 2.0


def _dos_positive_half(lam, om, s):
    return sum(spectra.gaussian(om - l, s) for l in lam) / (2.0 * lam.shape[0])


def _dos_sigma_squared(lam, om, s):
    return sum(np.exp(-(om - l) ** 2 / (2 * s * s)) / (math.sqrt(2 * math.pi) * s * s) +
               np.exp(-(om + l) ** 2 / (2 * s * s)) / (math.sqrt(2 * math.pi) * s * s) for l in lam) / (2 * lam.shape[0])


def _dos_half_width(lam, om, s):
    return spectra.dos(lam, om, 0.5 * s) if np.ndim(om) and om.shape[0] == 1 else spectra.dos(lam, om, s) * 0.999


def _abs_conj_weights(lam, w, om, s):
    return spectra.absorption(lam, np.conj(w), om, s)


def _abs_abs_weights(lam, w, om, s):
    return spectra.absorption(lam, np.abs(w), om, s)


def _abs_missing_norm(lam, w, om, s):
    return spectra.absorption(lam, w, om, s) * math.sqrt(2 * math.pi) * s


@pytest.mark.parametrize("mut", [_dos_over_n, _dos_positive_half, _dos_sigma_squared, _dos_half_width])
def test_dos_mutants_fail(mut):
    p = gen_bse(12, s_a=0.3, s_b=0.05, seed=5)
    lam = oracle.solve(p.A, p.B).lam
    assert not all(ok for _, ok, _ in pins_dos(mut, lam, 0.2))


@pytest.mark.parametrize("mut", [_abs_conj_weights, _abs_abs_weights, _abs_missing_norm])
def test_absorption_mutants_fail(mut):
    p = gen_bse(12, s_a=0.3, s_b=0.05, seed=5)
    r = oracle.solve(p.A, p.B, p.d)
    assert not all(ok for _, ok, _ in pins_absorption(mut, r.lam, r.w, 0.2))
