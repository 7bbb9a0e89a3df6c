"""Oracle of the two-stage (successive band reduction) skew
tridiagonalisation that Section 3.3 names as the way to cut the Level-2
cost of the reduction.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Stage 1 (dense to band): for each panel of b columns starting at k0, a
Householder reflector per column (the LAPACK dlarfg convention) annihilates
the panel below row k0 + b + j; each is applied from both sides, so the
result B = Q1^T W Q1 is skew with bandwidth b.  Stage 2 (band to
tridiagonal, bulge chasing): for each column s a reflector on rows
s+1 .. s+b annihilates the column below its subdiagonal; applied from both
sides it fills a block below the band, whose first column is annihilated
by a reflector on the next b rows, and so on down the matrix.  Every
reflector acts on rows >= 1, so U e_1 = e_1 for U = Q1 Q2, and by the
implicit-Q argument the tridiagonal T = U^T W U has the same |alpha| as the
one-stage reduction (unreduced case).  Plain O(N^2) two-sided application
per reflector: for small N only.
"""

from __future__ import annotations

import numpy as np

from .bse_oracle import _larfg


def _apply_two_sided(A: np.ndarray, r0: int, v: np.ndarray, tau: float) -> None:
    """A <- H A H with H = I - tau v v^T acting on indices r0 .. r0+len(v)-1."""
    sl = slice(r0, r0 + v.shape[0])
    A[sl, :] -= tau * np.outer(v, v @ A[sl, :])
    A[:, sl] -= tau * np.outer(A[:, sl] @ v, v)


def band_reduce(W: np.ndarray, b: int):
    """Stage 1.  Returns (B, refl) with B = Q1^T W Q1 of bandwidth b and
    refl = [(row0, v, tau), ...] in application order (Q1 = H_1 H_2 ...)."""
    A = np.array(W, dtype=np.float64)
    N = A.shape[0]
    refl = []
    for k0 in range(0, N, b):
        r0 = k0 + b
        if r0 >= N - 1:
            break
        for j in range(b):
            if r0 + j >= N - 1:
                break
            _beta, tau, v = _larfg(A[r0 + j:, k0 + j].copy())
            _apply_two_sided(A, r0 + j, v, tau)
            refl.append((r0 + j, v, tau))
    return A, refl


def band_to_tridiag(B: np.ndarray, b: int):
    """Stage 2.  Returns (T, alpha, refl): T = Q2^T B Q2 tridiagonal,
    alpha[k] = T[k+1, k] and the reflectors in application order."""
    A = np.array(B, dtype=np.float64)
    N = A.shape[0]
    refl = []
    for s in range(N - 2):
        col, r0 = s, s + 1
        while r0 < N - 1:
            r1 = min(r0 + b - 1, N - 1)
            _beta, tau, v = _larfg(A[r0:r1 + 1, col].copy())
            _apply_two_sided(A, r0, v, tau)
            refl.append((r0, v, tau))
            col, r0 = r0, r1 + 1
    alpha = np.array([A[k + 1, k] for k in range(N - 1)])
    return A, alpha, refl


def two_stage_tridiagonalize(W: np.ndarray, b: int):
    """W = U T U^T by the two stages; returns (alpha, U) (U explicit)."""
    N = W.shape[0]
    B, r1 = band_reduce(W, b)
    T, alpha, r2 = band_to_tridiag(B, b)
    U = np.eye(N)
    for r0, v, tau in r1 + r2:
        sl = slice(r0, r0 + v.shape[0])
        U[:, sl] -= tau * np.outer(U[:, sl] @ v, v)
    return alpha, U
