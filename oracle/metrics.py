"""Accuracy measures fixed by the paper, plus phase- and basis-invariant
comparisons of eigenvector sets.

TEST INFRASTRUCTURE ONLY.  Used to assess both the oracle and the GPU path;
none of it is part of the solver.
"""

from __future__ import annotations

import math

import numpy as np


def H_matrix(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """H = [[A, B], [-conj B, -conj A]]  (eq. H-complex), from full A, B."""
    return np.block([[A, B], [-B.conj(), -A.conj()]])


def omega_matrix(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Omega = [[A, B], [conj B, conj A]]  (eq. cond)."""
    return np.block([[A, B], [B.conj(), A.conj()]])


def full_eigvecs(X: np.ndarray):
    """All right and left eigenvectors from [X1; X2] (Theorem 3):
    X = [[X1, conj X2], [X2, conj X1]],  Y = [[X1, -conj X2], [-X2, conj X1]]."""
    n = X.shape[1]
    X1, X2 = X[:n], X[n:]
    Xf = np.block([[X1, X2.conj()], [X2, X1.conj()]])
    Yf = np.block([[X1, -X2.conj()], [-X2, X1.conj()]])
    return Xf, Yf


def table1_metrics(A: np.ndarray, B: np.ndarray, lam: np.ndarray, X: np.ndarray):
    """The two accuracy measures of Table 1:
    ||Y^H H X - Lambda||_F / ||H||_F   and   ||Y^H X - I_2n||_F / sqrt(2n)."""
    H = H_matrix(A, B)
    Xf, Yf = full_eigvecs(X)
    Lam = np.diag(np.concatenate([lam, -lam]))
    r1 = np.linalg.norm(Yf.conj().T @ H @ Xf - Lam) / np.linalg.norm(H)
    n2 = Xf.shape[0]
    r2 = np.linalg.norm(Yf.conj().T @ Xf - np.eye(n2)) / math.sqrt(n2)
    return float(r1), float(r2)


def normalization_error(X: np.ndarray) -> float:
    """max |X1^H X1 - X2^H X2 - I|  (eq. normalization)."""
    n = X.shape[1]
    X1, X2 = X[:n], X[n:]
    return float(np.max(np.abs(X1.conj().T @ X1 - X2.conj().T @ X2 - np.eye(n))))


def eig_residual(A: np.ndarray, B: np.ndarray, lam: np.ndarray, X: np.ndarray) -> float:
    """max_j ||H x_j - lam_j x_j|| / (||H||_F ||x_j||)."""
    H = H_matrix(A, B)
    R = H @ X - X * lam[None, :]
    return float(np.max(np.linalg.norm(R, axis=0) / (np.linalg.norm(H) * np.linalg.norm(X, axis=0))))


def Q_matrix(n: int) -> np.ndarray:
    """Q = (1/sqrt 2) [[I, -iI], [I, iI]]  (proof of Theorem 2)."""
    i = np.eye(n)
    return np.block([[i, -1j * i], [i, 1j * i]]) / math.sqrt(2.0)


def residual_certificate(A: np.ndarray, B: np.ndarray, lam_j: float, x_j: np.ndarray,
                         M: np.ndarray) -> float:
    """Bound on the distance from lam_j to the spectrum of H.

    H = Q (-i J M) Q^H (Theorem 2).  With M = L L^T, u = Q^H x, s = Q^H r for
    r = H x - lam x and z = L^T u one gets (-i L^T J L) z - lam z = L^T s,
    and -i L^T J L is Hermitian, so
        min_k |lam_k - lam| <= ||L^T Q^H r|| / ||L^T Q^H x||
    which in turn is at most sqrt(kappa(M)) ||r|| / ||x||.  Needs only FP64
    matrix-vector products with H; L comes from LAPACK's Cholesky of M."""
    n = A.shape[0]
    H = H_matrix(A, B)
    r = H @ x_j - lam_j * x_j
    L = np.linalg.cholesky(M)
    Qh = Q_matrix(n).conj().T
    return float(np.linalg.norm(L.T @ (Qh @ r)) / np.linalg.norm(L.T @ (Qh @ x_j)))


def clusters(lam: np.ndarray, gap: float):
    """Index ranges [s, e) of consecutive eigenvalues closer than `gap`."""
    out = []
    s = 0
    for j in range(1, lam.shape[0] + 1):
        if j == lam.shape[0] or lam[j] - lam[j - 1] > gap:
            out.append((s, j))
            s = j
    return out


def compare_eigvecs(X_ref: np.ndarray, X: np.ndarray, lam: np.ndarray, gap: float):
    """Basis-invariant distance between two eigenvector sets.

    Inside each cluster (consecutive eigenvalues closer than `gap`) the part
    of X_c that lies outside the reference cluster's eigenspace is
    E = X_c - X_ref,c (Y_ref,c^H X_c), with Y = S X the left eigenvectors
    (Theorem 3), i.e. (I - P_ref) X_c for the oblique spectral projector
    P_ref = X_ref,c Y_ref,c^H.  It does not depend on the phase or on the
    basis chosen inside a cluster.  Returns max over clusters of
    ||E||_F / ||X_c||_F."""
    n = X.shape[1]
    worst = 0.0
    for s, e in clusters(lam, gap):
        Xr, Xc = X_ref[:, s:e], X[:, s:e]
        Yr = Xr.copy()
        Yr[n:] *= -1
        E = Xc - Xr @ (Yr.conj().T @ Xc)
        worst = max(worst, float(np.linalg.norm(E) / np.linalg.norm(Xc)))
    return worst


def compare_weights(w_ref: np.ndarray, w: np.ndarray, lam: np.ndarray, gap: float) -> float:
    """Max over clusters of |sum w - sum w_ref| / max(|sum w_ref|, sum|w_ref|).
    Weights summed over a cluster do not depend on the basis chosen for it."""
    worst = 0.0
    scale = float(np.sum(np.abs(w_ref))) or 1.0
    for s, e in clusters(lam, gap):
        worst = max(worst, abs(np.sum(w[s:e]) - np.sum(w_ref[s:e])) / scale)
    return worst


def weights_all_pairs(X: np.ndarray, d_r: np.ndarray, d_l: np.ndarray) -> np.ndarray:
    """Absorption-type weights over all 2n eigenpairs, using the negative
    eigenvectors of Theorem 3.  Their sum is d_r^H d_l because Y^H X = I."""
    Xf, Yf = full_eigvecs(X)
    num = (d_r.conj() @ Xf) * (Yf.conj().T @ d_l)
    den = np.einsum("ij,ij->j", Yf.conj(), Xf)
    return num / den
