"""Plain FP64 oracle of Algorithm 1 (complex Bethe-Salpeter eigenproblem),
carried out the way Algorithm 3 organises steps 4 and 5.

TEST INFRASTRUCTURE ONLY -- imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.

Every step is unblocked and follows the paper's order and notation:

  Algorithm 1, step 1   M = [[Re(A+B), Im(A-B)], [-Im(A+B), Re(A-B)]]   (eq. embedding)
  Algorithm 1, step 2   M = L L^T                                         (textbook Cholesky)
  Algorithm 1, step 3   W = L^T J_n L                                     (eq. J)
  Algorithm 3, step 1   W = U T U^T  by Householder reflections           (Section 3.3, remark 1)
  Algorithm 3, step 2   -i D^H T D = tridiag(alpha, 0, alpha); bisection for the
                        positive eigenvalues, inverse iteration for V_+,
                        reorthogonalised inside clusters                  (Section 3.3, remark 2)
  Algorithm 3, step 3   Phi = L U  (reflections applied to L)
  Algorithm 3, step 4   Y_hat = Q Phi D                                   (remark 3, O(n^2))
  Algorithm 3, step 5   Y_+ = Y_hat V_+, real and imaginary parts apart   (remark 4)
  Algorithm 3, step 6   [X1; X2] = S Y_+ Lambda_+^{-1/2}                  (Algorithm 1, step 5)

Readings taken where the paper is silent (each also listed in the design
notes): D = diag(i^k) for k = 0..2n-1; Algorithm 3 omits the Lambda_+^{-1/2}
scaling of Algorithm 1 step 5, which is applied here (it is what makes
X1^H X1 - X2^H X2 = I hold); reflectors follow LAPACK's dlarfg convention;
the lower triangles of A and B are the ones read; bisection stops at a
relative width of 2 eps; clusters for reorthogonalisation are consecutive
eigenvalues closer than 1e-3 * ||T_s||_1 (LAPACK dstein's criterion) and are
Gram-Schmidt orthogonalised in ascending order; eigenvectors get a canonical
phase (largest-modulus entry, lowest index on ties, made real positive).

Library primitives used as single steps: matrix products, vector norms,
square roots.  No LAPACK eigensolver is called.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

EPS = np.finfo(np.float64).eps          # 2^-52
SAFMIN = np.finfo(np.float64).tiny


# --------------------------------------------------------------------------
# Algorithm 1, step 1 (Theorem 2, eq. embedding)
# --------------------------------------------------------------------------

def symmetrize_lower(A: np.ndarray, B: np.ndarray):
    """Full A (Hermitian) and B (complex symmetric) from their lower
    triangles (eq. symmetry: A = A^H, B = B^T)."""
    lo_a = np.tril(A)
    lo_b = np.tril(B)
    a = lo_a + np.tril(A, -1).conj().T
    a = a - np.diag(1j * np.diag(a).imag)   # Hermitian: real diagonal
    b = lo_b + np.tril(B, -1).T
    return a, b


def build_M(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """M = [[Re(A+B), Im(A-B)], [-Im(A+B), Re(A-B)]]  (Theorem 2, eq. embedding).
    Only the lower triangles of A and B are read."""
    a, b = symmetrize_lower(A, B)
    return np.block([[(a + b).real, (a - b).imag],
                     [-(a + b).imag, (a - b).real]]).astype(np.float64)


# --------------------------------------------------------------------------
# Algorithm 1, step 2
# --------------------------------------------------------------------------

def cholesky(M: np.ndarray):
    """Textbook left-looking column Cholesky M = L L^T.

    Returns (L, info).  info = 0 on success; info = k > 0 when the leading
    k x k minor of M is not positive definite, i.e. the condition eq. cond of
    the paper does not hold (Algorithm 1 requires it)."""
    N = M.shape[0]
    L = np.zeros_like(M, dtype=np.float64)
    for j in range(N):
        s = M[j, j] - L[j, :j] @ L[j, :j]
        if not (s > 0.0) or not np.isfinite(s):
            return L, j + 1
        ljj = math.sqrt(s)
        L[j, j] = ljj
        if j + 1 < N:
            L[j + 1:, j] = (M[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / ljj
    return L, 0


# --------------------------------------------------------------------------
# Algorithm 1, step 3
# --------------------------------------------------------------------------

def J_matrix(n: int) -> np.ndarray:
    """J_n = [[0, I_n], [-I_n, 0]]  (eq. J)."""
    z = np.zeros((n, n))
    i = np.eye(n)
    return np.block([[z, i], [-i, z]])


def form_W(L: np.ndarray) -> np.ndarray:
    """W = L^T J_n L, a real skew-symmetric matrix (Section 3.1)."""
    n = L.shape[0] // 2
    return L.T @ (J_matrix(n) @ L)


# --------------------------------------------------------------------------
# Algorithm 3, step 1: skew-symmetric Householder tridiagonalisation
# --------------------------------------------------------------------------

def _larfg(x: np.ndarray):
    """Householder reflector H = I - tau v v^T with H x = beta e_1 and v[0]=1
    (LAPACK dlarfg convention)."""
    alpha = x[0]
    xnorm = np.linalg.norm(x[1:]) if x.shape[0] > 1 else 0.0
    v = np.zeros_like(x)
    v[0] = 1.0
    if xnorm == 0.0:
        return alpha, 0.0, v
    beta = -math.copysign(math.hypot(alpha, xnorm), alpha)
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return beta, tau, v


def skew_tridiagonalize(W: np.ndarray):
    """W = U T U^T with U = H_0 H_1 ... H_{N-3}, T skew tridiagonal.

    Reflector H_k = I - tau_k v_k v_k^T acts on rows/columns k+1..N-1 and
    zeroes W[k+2:, k].  For a skew matrix S and p = tau S v one has
    v^T S v = 0, so H S H = S + v p^T - p v^T (no extra rank-one term as in
    the symmetric case; Section 3.3, remark 1).

    Returns (alpha, vs, taus): alpha[k] = T[k, k+1] (the paper's
    superdiagonal, so T[k+1, k] = -alpha[k]), vs[k] the reflector vector on
    rows k+1.., taus[k] its scalar.
    """
    Wk = np.array(W, dtype=np.float64, copy=True)
    N = Wk.shape[0]
    alpha = np.zeros(N - 1)
    vs, taus = [], []
    for k in range(N - 1):
        x = Wk[k + 1:, k].copy()
        if k == N - 2:
            beta, tau, v = x[0], 0.0, np.ones(1)
        else:
            beta, tau, v = _larfg(x)
        alpha[k] = -beta
        vs.append(v)
        taus.append(tau)
        if k == N - 2:
            break
        Wk[k + 1:, k] = 0.0
        Wk[k + 1, k] = beta
        Wk[k, k + 1:] = 0.0
        Wk[k, k + 1] = -beta
        if tau != 0.0:
            S = Wk[k + 1:, k + 1:]
            p = tau * (S @ v)
            S += np.outer(v, p) - np.outer(p, v)
    return alpha, vs, np.array(taus)


def householder_matrix(vs, taus, N: int) -> np.ndarray:
    """U = H_0 H_1 ... H_{N-2} as an explicit N x N orthogonal matrix."""
    U = np.eye(N)
    for k in range(len(vs) - 1, -1, -1):
        v = np.zeros(N)
        v[k + 1:] = vs[k]
        U -= taus[k] * np.outer(v, v @ U)
    return U


def tridiag_T(alpha: np.ndarray) -> np.ndarray:
    """Explicit skew tridiagonal T with T[k,k+1] = alpha[k], T[k+1,k] = -alpha[k]."""
    return np.diag(alpha, 1) - np.diag(alpha, -1)


def tridiag_T_s(alpha: np.ndarray) -> np.ndarray:
    """T_s = -i D^H T D = tridiag(alpha, 0, alpha) with D = diag(i^k)
    (Section 3.3, remark 2)."""
    return np.diag(alpha, 1) + np.diag(alpha, -1)


# --------------------------------------------------------------------------
# Algorithm 3, step 2: bisection + inverse iteration (remark 2)
# --------------------------------------------------------------------------

def _pivmin(e2: np.ndarray) -> float:
    return SAFMIN * max(1.0, float(np.max(e2)) if e2.size else 1.0)


def sturm_count(alpha: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Number of eigenvalues of T_s = tridiag(alpha, 0, alpha) smaller than x
    (Sturm sequence of the LDL^T factorisation of T_s - x I), vectorised over
    the shifts x."""
    e2 = alpha * alpha
    pivmin = _pivmin(e2)
    x = np.asarray(x, dtype=np.float64)
    q = -x.copy()
    q = np.where(np.abs(q) < pivmin, -pivmin, q)
    cnt = (q < 0).astype(np.int64)
    for k in range(1, alpha.shape[0] + 1):
        q = -x - e2[k - 1] / q
        q = np.where(np.abs(q) < pivmin, -pivmin, q)
        cnt += q < 0
    return cnt


def gershgorin_bound(alpha: np.ndarray) -> float:
    """max_k |alpha_{k-1}| + |alpha_k|, an upper bound of |eig(T_s)| = ||T_s||_1."""
    a = np.abs(alpha)
    left = np.concatenate(([0.0], a))
    right = np.concatenate((a, [0.0]))
    return float(np.max(left + right))


def bisect_positive(alpha: np.ndarray, max_iter: int = 200) -> np.ndarray:
    """The n positive eigenvalues of T_s (N = 2n), ascending, by bisection.

    T_s is nonsingular (W = L^T J L is), so exactly n eigenvalues lie below 0.
    The j-th positive eigenvalue is the (n+j)-th smallest overall; every
    interval starts as [0, Gershgorin bound] and is halved until its width is
    at most 2 eps max(|lo|, |hi|) (or 4 pivmin)."""
    N = alpha.shape[0] + 1
    n = N // 2
    e2 = alpha * alpha
    pivmin = _pivmin(e2)
    target = n + np.arange(n)               # eigenvalue index in ascending order
    lo = np.zeros(n)
    hi = np.full(n, gershgorin_bound(alpha) * (1.0 + 4.0 * EPS) + 4.0 * pivmin)
    active = np.ones(n, dtype=bool)
    for _ in range(max_iter):
        tol = np.maximum(2.0 * EPS * np.maximum(np.abs(lo), np.abs(hi)), 4.0 * pivmin)
        active = (hi - lo) > tol
        if not np.any(active):
            break
        idx = np.nonzero(active)[0]
        mid = 0.5 * (lo[idx] + hi[idx])
        stuck = (mid <= lo[idx]) | (mid >= hi[idx])
        c = sturm_count(alpha, mid)
        go_up = c <= target[idx]
        lo[idx] = np.where(go_up & ~stuck, mid, lo[idx])
        hi[idx] = np.where(~go_up & ~stuck, mid, hi[idx])
        done = idx[stuck]
        hi[done] = lo[done]
    return 0.5 * (lo + hi)


def _tridiag_lu_solve(alpha: np.ndarray, shift: np.ndarray, rhs: np.ndarray,
                      pert: float) -> np.ndarray:
    """Solve (T_s - shift_j I) x_j = rhs_j for every column j by Gaussian
    elimination with partial pivoting (the LAPACK dgttrf/dgttrs scheme),
    vectorised over the columns.  Pivots smaller than `pert` in modulus are
    replaced by +-pert, as inverse iteration does for a (nearly) singular
    shifted matrix."""
    N = alpha.shape[0] + 1
    m = shift.shape[0]
    d = np.tile(-shift, (N, 1))                       # diagonal, per column
    du = np.tile(alpha[:, None], (1, m)) if N > 1 else np.zeros((0, m))
    dl = alpha
    du2 = np.zeros((max(N - 2, 0), m))
    lmul = np.zeros((max(N - 1, 0), m))
    swap = np.zeros((max(N - 1, 0), m), dtype=bool)
    for k in range(N - 1):
        sw = np.abs(d[k]) < abs(dl[k])
        swap[k] = sw
        # no interchange
        dk = np.where(np.abs(d[k]) < pert, np.where(d[k] < 0, -pert, pert), d[k])
        l_ns = dl[k] / np.where(sw, 1.0, dk)
        # interchange rows k, k+1
        l_sw = d[k] / (dl[k] if dl[k] != 0.0 else 1.0)
        dkp1_old = d[k + 1].copy()
        duk_old = du[k].copy()
        du_next_old = du[k + 1].copy() if k + 1 < N - 1 else None
        lmul[k] = np.where(sw, l_sw, l_ns)
        d[k] = np.where(sw, dl[k], dk)
        du[k] = np.where(sw, dkp1_old, duk_old)
        d[k + 1] = np.where(sw, duk_old - l_sw * dkp1_old, dkp1_old - l_ns * duk_old)
        if k < N - 2:
            du2[k] = np.where(sw, du_next_old, 0.0)
            du[k + 1] = np.where(sw, -l_sw * du_next_old, du_next_old)
    d = np.where(np.abs(d) < pert, np.where(d < 0, -pert, pert), d)
    b = np.array(rhs, dtype=np.float64, copy=True)
    for k in range(N - 1):
        sw = swap[k]
        bk = b[k].copy()
        bk1 = b[k + 1].copy()
        b[k] = np.where(sw, bk1, bk)
        b[k + 1] = np.where(sw, bk - lmul[k] * bk1, bk1 - lmul[k] * bk)
    x = np.zeros_like(b)
    x[N - 1] = b[N - 1] / d[N - 1]
    if N > 1:
        x[N - 2] = (b[N - 2] - du[N - 2] * x[N - 1]) / d[N - 2]
    for k in range(N - 3, -1, -1):
        x[k] = (b[k] - du[k] * x[k + 1] - du2[k] * x[k + 2]) / d[k]
    return x


def inverse_iteration(alpha: np.ndarray, lam: np.ndarray, seed: int = 12345,
                      iters: int = 3) -> np.ndarray:
    """Eigenvectors of T_s for the (ascending) eigenvalues lam by inverse
    iteration: `iters` solves with T_s - sigma_j I from a random start,
    normalised after each solve.  Shifts closer than 10 eps |lam_j| to the
    previous one are pushed apart by that amount (as LAPACK dstein does) so
    that equal eigenvalues get independent directions."""
    N = alpha.shape[0] + 1
    m = lam.shape[0]
    tnorm = gershgorin_bound(alpha)
    pert = EPS * max(tnorm, SAFMIN)
    shift = lam.astype(np.float64).copy()
    for j in range(1, m):
        pertol = 10.0 * EPS * abs(shift[j])
        if shift[j] - shift[j - 1] < pertol:
            shift[j] = shift[j - 1] + pertol
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1.0, 1.0, size=(N, m))
    for _ in range(iters):
        x = _tridiag_lu_solve(alpha, shift, b, pert)
        b = x / np.linalg.norm(x, axis=0, keepdims=True)
    return b


def reorthogonalize_clusters(V: np.ndarray, lam: np.ndarray, ortol: float) -> np.ndarray:
    """Gram-Schmidt inside clusters: consecutive eigenvalues with gap <= ortol
    form a cluster whose vectors are orthogonalised in ascending order, each
    against the earlier ones of its cluster (two classical passes), then
    normalised."""
    V = np.array(V, dtype=np.float64, copy=True)
    m = lam.shape[0]
    start = 0
    for j in range(m):
        if j > 0 and lam[j] - lam[j - 1] > ortol:
            start = j
        v = V[:, j]
        if j > start:
            P = V[:, start:j]
            for _ in range(2):
                v = v - P @ (P.T @ v)
        V[:, j] = v / np.linalg.norm(v)
    return V


def eigenvectors_T_s(alpha: np.ndarray, lam: np.ndarray, seed: int = 12345) -> np.ndarray:
    """V_+ (N x n): inverse iteration plus cluster reorthogonalisation."""
    V = inverse_iteration(alpha, lam, seed=seed)
    ortol = 1e-3 * gershgorin_bound(alpha)
    return reorthogonalize_clusters(V, lam, ortol)


# --------------------------------------------------------------------------
# Algorithm 3, steps 3-6
# --------------------------------------------------------------------------

def phi_LU(L: np.ndarray, vs, taus) -> np.ndarray:
    """Phi = L U = L H_0 H_1 ... H_{N-2} (Algorithm 3, step 3).

    Computed as its transpose Phi^T = ... H_1 H_0 L^T, i.e. the reflections
    applied to the rows of L^T in the order H_0, H_1, ... (row-major storage
    keeps each update contiguous)."""
    Pt = np.array(L.T, dtype=np.float64, copy=True, order="C")
    for k in range(len(vs)):
        if taus[k] == 0.0:
            continue
        v = vs[k]
        blk = Pt[k + 1:, :]
        blk -= taus[k] * np.outer(v, v @ blk)
    return Pt.T


def back_transform(Phi: np.ndarray, V: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """[X1; X2] = S Q Phi D V_+ Lambda_+^{-1/2}  (Algorithm 3 steps 4-6 with
    Algorithm 1 step 5's scaling).

    Y_hat = Q Phi D is formed in O(n^2) (remark 3): Q = (1/sqrt 2)[[I, -iI],
    [I, iI]] combines row blocks, D = diag(i^k) scales columns.  Y_+ =
    Y_hat V_+ is two real products, one for the real and one for the imaginary
    part (remark 4)."""
    N = Phi.shape[0]
    n = N // 2
    Phi1, Phi2 = Phi[:n], Phi[n:]
    Qphi = np.vstack([Phi1 - 1j * Phi2, Phi1 + 1j * Phi2]) / math.sqrt(2.0)
    dk = np.array([1j ** (k % 4) for k in range(N)])
    Y_hat = Qphi * dk[None, :]
    Y_plus = (np.ascontiguousarray(Y_hat.real) @ V) + 1j * (np.ascontiguousarray(Y_hat.imag) @ V)
    X = Y_plus.copy()
    X[n:] = -X[n:]
    return X / np.sqrt(lam)[None, :]


def canonical_phase(X: np.ndarray) -> np.ndarray:
    """Scale each column by a unit phase so that its largest-modulus entry
    (lowest index on ties) is real and positive."""
    X = np.array(X, copy=True)
    idx = np.argmax(np.abs(X), axis=0)
    piv = X[idx, np.arange(X.shape[1])]
    ph = np.where(np.abs(piv) > 0, np.conj(piv) / np.abs(piv), 1.0)
    return X * ph[None, :]


def absorption_weights(X: np.ndarray, d_r: np.ndarray, d_l: np.ndarray) -> np.ndarray:
    """w_j = (d_r^H x_j)(y_j^H d_l) / (y_j^H x_j) with y_j = S x_j (eq. absp,
    left eigenvectors from Theorem 3)."""
    n = X.shape[1]
    Y = X.copy()
    Y[n:] = -Y[n:]
    num = (d_r.conj() @ X) * (Y.conj().T @ d_l)
    den = np.einsum("ij,ij->j", Y.conj(), X)
    return num / den


@dataclasses.dataclass
class OracleResult:
    lam: np.ndarray            # n positive eigenvalues, ascending
    X: np.ndarray              # (2n, n) complex, [X1; X2], canonical phase
    w: np.ndarray | None       # absorption weights or None
    info: int                  # 0, or k > 0 when eq. cond fails at minor k
    M: np.ndarray | None = None
    L: np.ndarray | None = None
    W: np.ndarray | None = None
    alpha: np.ndarray | None = None
    V: np.ndarray | None = None


def solve(A: np.ndarray, B: np.ndarray, d_r: np.ndarray | None = None,
          d_l: np.ndarray | None = None, keep: bool = False, seed: int = 12345) -> OracleResult:
    """Algorithm 1 end to end.  A, B: complex (n, n), only lower triangles
    read.  Returns the positive eigenvalues (ascending), the right
    eigenvectors [X1; X2] normalised so that X1^H X1 - X2^H X2 = I, and the
    absorption weights when dipole vectors are given."""
    n = A.shape[0]
    M = build_M(A, B)
    L, info = cholesky(M)
    if info != 0:
        return OracleResult(np.zeros(0), np.zeros((2 * n, 0), complex), None, info)
    W = form_W(L)
    alpha, vs, taus = skew_tridiagonalize(W)
    lam = bisect_positive(alpha)
    V = eigenvectors_T_s(alpha, lam, seed=seed)
    Phi = phi_LU(L, vs, taus)
    X = canonical_phase(back_transform(Phi, V, lam))
    w = None
    if d_r is not None:
        w = absorption_weights(X, d_r, d_r if d_l is None else d_l)
    if keep:
        return OracleResult(lam, X, w, 0, M=M, L=L, W=W, alpha=alpha, V=V)
    return OracleResult(lam, X, w, 0)
