"""Oracle for the Tamm-Dancoff solve and the broadened spectra.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Tamm-Dancoff approximation (Section 2.2): the Bethe-Salpeter Hamiltonian
  with B = 0 is blkdiag(A, -conj A); its positive eigenpairs are those of the
  Hermitian A, lambda_j(A) with x_j = [v_j; 0].  Theorem 4 states that, under
  eq. cond, lambda_j(H) <= lambda_j(A) with both sorted the same way.  The
  plain definition is the Hermitian eigendecomposition of A (a library
  routine, numpy.linalg.eigh, serves as that step).
* Density of states, eq. DOS: phi(omega) = 1/(2n) sum over the 2n
  eigenvalues of delta(omega - lambda_j); absorption spectrum, eq. absp:
  eps+(omega) = sum_{j=1}^n w_j delta(omega - lambda_j).  Section 4 replaces
  the delta function by a Gaussian of standard deviation sigma
  (5e-4 there).  Written out as explicit sums.
"""

from __future__ import annotations

import math

import numpy as np

from .bse_oracle import absorption_weights, canonical_phase, symmetrize_lower


def tda_solve(A: np.ndarray, d_r: np.ndarray | None = None, d_l: np.ndarray | None = None):
    """Eigenvalues of A ascending, eigenvectors as [v_j; 0] with unit v_j and
    the canonical phase, and the TDA weights of eq. absp (y_j = S x_j).
    Only the lower triangle of A is read."""
    a, _ = symmetrize_lower(A, np.zeros_like(A))
    lam, V = np.linalg.eigh(a)
    n = A.shape[0]
    X = np.zeros((2 * n, n), dtype=np.complex128)
    X[:n] = V
    X = canonical_phase(X)
    w = None
    if d_r is not None:
        w = absorption_weights(X, d_r, d_r if d_l is None else d_l)
    return lam, X, w


def gaussian(t, sigma: float):
    """The broadened delta function of Section 4."""
    return np.exp(-np.asarray(t) ** 2 / (2.0 * sigma * sigma)) / (math.sqrt(2.0 * math.pi) * sigma)


def dos(lam: np.ndarray, omega: np.ndarray, sigma: float) -> np.ndarray:
    """phi(omega) of eq. DOS over the 2n eigenvalues +-lambda_j of H (the
    negative half from Theorem 3), each delta broadened by the Gaussian."""
    n = lam.shape[0]
    out = np.zeros(omega.shape[0])
    for l in lam:
        out += gaussian(omega - l, sigma)
        out += gaussian(omega + l, sigma)
    return out / (2.0 * n)


def absorption(lam: np.ndarray, w: np.ndarray, omega: np.ndarray, sigma: float) -> np.ndarray:
    """eps+(omega) of eq. absp: the weights of the positive eigenvalues, each
    at its eigenvalue, broadened by the Gaussian (complex weights give a
    complex spectrum)."""
    out = np.zeros(omega.shape[0], dtype=np.complex128)
    for l, wj in zip(lam, w):
        out += wj * gaussian(omega - l, sigma)
    return out
