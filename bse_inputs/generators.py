"""Seeded generators for Bethe-Salpeter test and benchmark problems.

A Bethe-Salpeter Hamiltonian is H = [[A, B], [-conj(B), -conj(A)]] with A
Hermitian and B complex symmetric (eq. H-complex and eq. symmetry of the
paper).  The structure-preserving method needs the definiteness condition
Omega = [[A, B], [conj(B), conj(A)]] > 0 (eq. cond).

The physical matrices the paper measures (naphthalene, GaAs and BN, Section 4)
are not available, so every problem here is synthetic with their structure: a
dense Hermitian A dominated by a positive diagonal (quasiparticle energy
differences), a weaker dense Hermitian kernel added to it, and a smaller
complex-symmetric coupling B (Section 1).

All random draws use numpy's PCG64 generator (``numpy.random.default_rng``)
in a fixed order, so a (generator, n, seed) triple always yields the same
matrices.  Matrices are returned as complex128 arrays in C order; callers that
need column-major storage transpose explicitly.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

# Seed offset used when a draw must be rejected (Omega not positive definite).
REJECT_SEED_STRIDE = 1_000_003


@dataclasses.dataclass
class BseProblem:
    """One Bethe-Salpeter problem.

    A, B  : complex128 (n, n); A Hermitian, B complex symmetric (full storage).
    d     : complex128 (2n,) unit dipole vector, used as d_r = d_l.
    seed  : the seed that produced the accepted draw.
    exact_lambda : the exact positive eigenvalues (ascending) when the
                   generator knows them in closed form, else None.
    """

    A: np.ndarray
    B: np.ndarray
    d: np.ndarray
    seed: int
    exact_lambda: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.A.shape[0]


def omega_is_positive_definite(A: np.ndarray, B: np.ndarray) -> bool:
    """True when Omega = [[A, B], [conj B, conj A]] is Hermitian positive
    definite (eq. cond).  Uses LAPACK's complex Cholesky on Omega itself, which
    is the definition of the condition, not the solver's real embedding."""
    omega = np.block([[A, B], [B.conj(), A.conj()]])
    try:
        np.linalg.cholesky(omega)
    except np.linalg.LinAlgError:
        return False
    return True


def _complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / math.sqrt(2.0)


def _unit_dipole(rng: np.random.Generator, n: int) -> np.ndarray:
    g = _complex_gaussian(rng, (2 * n,))
    return g / np.linalg.norm(g)


def gen_bse(n: int, s_a: float = 0.1, s_b: float = 0.05, seed: int = 0,
            check_definite: bool = True, max_tries: int = 16) -> BseProblem:
    """Dense synthetic problem with the structure of the paper's workloads.

    Draw order (PCG64, ``default_rng(seed)``):
      1. u ~ U[1, 10]^n                         (diagonal energies)
      2. G1 complex Gaussian n x n;  A = diag(u) + (s_a/sqrt n) (G1 + G1^H)/sqrt 2
      3. G2 complex Gaussian n x n;  B = (s_b/sqrt n) (G2 + G2^T)/sqrt 2
      4. g complex Gaussian 2n;      d = g / |g|
    A draw whose Omega is not positive definite is rejected and the next seed
    tried is seed + 1,000,003.
    """
    if n <= 0:
        raise ValueError("n must be positive")
    cur = seed
    for _ in range(max_tries):
        rng = np.random.default_rng(cur)
        u = rng.uniform(1.0, 10.0, size=n)
        g1 = _complex_gaussian(rng, (n, n))
        a = np.diag(u).astype(np.complex128) + (s_a / math.sqrt(n)) * (g1 + g1.conj().T) / math.sqrt(2.0)
        g2 = _complex_gaussian(rng, (n, n))
        b = (s_b / math.sqrt(n)) * (g2 + g2.T) / math.sqrt(2.0)
        d = _unit_dipole(rng, n)
        # enforce exact symmetry of the stored matrices
        a = 0.5 * (a + a.conj().T)
        b = 0.5 * (b + b.T)
        if not check_definite or omega_is_positive_definite(a, b):
            return BseProblem(a, b, d, cur)
        cur += REJECT_SEED_STRIDE
    raise RuntimeError("no positive definite draw found")


def _haar_unitary(rng: np.random.Generator, m: int) -> np.ndarray:
    z = _complex_gaussian(rng, (m, m))
    q, r = np.linalg.qr(z)
    ph = np.diag(r).copy()
    ph = np.where(np.abs(ph) > 0, ph / np.abs(ph), 1.0)
    return q * ph[None, :]


def _split_factors(n: int) -> tuple[int, int]:
    """n = n1 * n2 with n1 <= n2 as balanced as possible."""
    best = (1, n)
    for f in range(1, int(math.isqrt(n)) + 1):
        if n % f == 0:
            best = (f, n // f)
    return best


def gen_closed_form(n: int, seed: int = 30, b_ratio: float = 0.05,
                    kron_above: int = 2048, planted=()) -> BseProblem:
    """Problem with eigenvalues known in closed form.

    With a unitary U0, A = U0 diag(a) U0^H and B = U0 diag(b) U0^T, the
    Hamiltonian decouples into n 2x2 problems [[a_k, b_k], [-conj b_k, -a_k]]
    whose positive eigenvalue is sqrt(a_k^2 - |b_k|^2).

    Draw order: a ~ U[1,10]^n; |b| = b_ratio * a * U[0,1]; arg b ~ U[0, 2pi);
    then U0.  For n <= kron_above, U0 is Haar (QR of a complex Gaussian with
    the R-diagonal phases removed).  Above it, U0 = P (Ua kron Ub) with Haar
    Ua, Ub of sizes n1*n2 = n and a random permutation P, which keeps the
    generation O(n^2 (n1 + n2)) while A and B stay dense.

    planted: pairs (k, g) applied after the draws: a[k+1] = (1+g) a[k] and
    b[k+1] = (1+g) b[k], so the eigenvalue of index k+1 (draw order) is
    (1+g) times that of index k: a near-degenerate pair of relative gap g
    (g = 0: an exactly degenerate one).
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(1.0, 10.0, size=n)
    bmag = b_ratio * a * rng.uniform(0.0, 1.0, size=n)
    bph = rng.uniform(0.0, 2.0 * math.pi, size=n)
    b = bmag * np.exp(1j * bph)
    for k, g in planted:
        if not 0 <= k < n - 1:
            raise ValueError("planted pair index out of range")
        a[k + 1] = (1.0 + g) * a[k]
        b[k + 1] = (1.0 + g) * b[k]
    if n <= kron_above:
        u0 = _haar_unitary(rng, n)
        amat = (u0 * a[None, :]) @ u0.conj().T
        bmat = (u0 * b[None, :]) @ u0.T
    else:
        n1, n2 = _split_factors(n)
        ua = _haar_unitary(rng, n1)
        ub = _haar_unitary(rng, n2)
        perm = rng.permutation(n)
        amat = _kron_congruence(ua, ub, a.astype(np.complex128), conj_right=True)
        bmat = _kron_congruence(ua, ub, b, conj_right=False)
        amat = amat[np.ix_(perm, perm)]
        bmat = bmat[np.ix_(perm, perm)]
    amat = 0.5 * (amat + amat.conj().T)
    bmat = 0.5 * (bmat + bmat.T)
    d = _unit_dipole(rng, n)
    lam = np.sort(np.sqrt(a * a - np.abs(b) ** 2))
    return BseProblem(amat, bmat, d, seed, exact_lambda=lam)


def _kron_congruence(ua: np.ndarray, ub: np.ndarray, diag: np.ndarray,
                     conj_right: bool) -> np.ndarray:
    """K diag(v) K^H (conj_right) or K diag(v) K^T with K = ua kron ub."""
    n1, n2 = ua.shape[0], ub.shape[0]
    dv = diag.reshape(n1, n2)
    ubr = ub.conj() if conj_right else ub
    uar = ua.conj() if conj_right else ua
    # t[k1, i2, j2] = sum_k2 ub[i2,k2] d[k1,k2] ubr[j2,k2]
    t = np.einsum("ik,ak,jk->aij", ub, dv, ubr, optimize=True)
    # out[i1, i2, j1, j2] = sum_k1 ua[i1,k1] uar[j1,k1] t[k1,i2,j2]
    out = np.einsum("pk,qk,kij->piqj", ua, uar, t, optimize=True)
    return out.reshape(n1 * n2, n1 * n2)


def gen_b_zero(n: int, seed: int = 0, s_a: float = 0.1) -> BseProblem:
    """B = 0: H = diag(A, -conj A) so the positive eigenvalues are eig(A)."""
    p = gen_bse(n, s_a=s_a, s_b=0.0, seed=seed)
    return BseProblem(p.A, np.zeros_like(p.A), p.d, p.seed)


def gen_real(n: int, seed: int = 0, s_a: float = 0.1, s_b: float = 0.05) -> BseProblem:
    """Real symmetric A and B (the real Bethe-Salpeter case, eq. H-real)."""
    cur = seed
    for _ in range(16):
        rng = np.random.default_rng(cur)
        u = rng.uniform(1.0, 10.0, size=n)
        g1 = rng.standard_normal((n, n))
        a = np.diag(u) + (s_a / math.sqrt(n)) * (g1 + g1.T) / math.sqrt(2.0)
        g2 = rng.standard_normal((n, n))
        b = (s_b / math.sqrt(n)) * (g2 + g2.T) / math.sqrt(2.0)
        d = _unit_dipole(rng, n)
        a = a.astype(np.complex128)
        b = b.astype(np.complex128)
        if omega_is_positive_definite(a, b):
            return BseProblem(a, b, d, cur)
        cur += REJECT_SEED_STRIDE
    raise RuntimeError("no positive definite draw found")


def gen_real_closed_form(n: int, seed: int = 40, b_ratio: float = 0.5, planted=()) -> BseProblem:
    """Real problem with eigenvalues known in closed form.

    With a real orthogonal Q0, A = Q0 diag(a) Q0^T and B = Q0 diag(b) Q0^T
    decouple H into n 2x2 problems [[a_k, b_k], [-b_k, -a_k]] whose positive
    eigenvalue is sqrt(a_k^2 - b_k^2).  Draw order: a ~ U[1,10]^n,
    b = b_ratio * a * U[-1,1], then Q0 (QR of a Gaussian with the R-diagonal
    signs removed), then a unit complex dipole.  planted: pairs (k, g) set
    a[k+1] = (1+g) a[k], b[k+1] = (1+g) b[k] after the draws (g = 0: an
    exactly degenerate eigenvalue)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(1.0, 10.0, size=n)
    b = b_ratio * a * rng.uniform(-1.0, 1.0, size=n)
    for k, g in planted:
        if not 0 <= k < n - 1:
            raise ValueError("planted pair index out of range")
        a[k + 1] = (1.0 + g) * a[k]
        b[k + 1] = (1.0 + g) * b[k]
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    q = q * np.sign(np.diag(r))[None, :]
    amat = (q * a[None, :]) @ q.T
    bmat = (q * b[None, :]) @ q.T
    amat = 0.5 * (amat + amat.T)
    bmat = 0.5 * (bmat + bmat.T)
    d = _unit_dipole(rng, n)
    lam = np.sort(np.sqrt(a * a - b * b))
    return BseProblem(amat.astype(np.complex128), bmat.astype(np.complex128), d, seed, exact_lambda=lam)


def gen_not_definite(n: int, k: int, seed: int = 0) -> BseProblem:
    """A problem whose Omega fails to be positive definite.

    A = diag(u), B = diag(b) with |b_j| < u_j except at index k (0-based),
    where |b_k| = 2 u_k.  The 2x2 block [[u_k, b_k], [conj b_k, u_k]] of Omega
    is then indefinite.
    """
    if not 0 <= k < n:
        raise ValueError("k out of range")
    rng = np.random.default_rng(seed)
    u = rng.uniform(1.0, 10.0, size=n)
    bm = 0.5 * u * rng.uniform(0.0, 1.0, size=n)
    bm[k] = 2.0 * u[k]
    ph = np.exp(1j * rng.uniform(0.0, 2.0 * math.pi, size=n))
    a = np.diag(u).astype(np.complex128)
    b = np.diag(bm * ph)
    d = _unit_dipole(rng, n)
    return BseProblem(a, b, d, seed)


def batched_sizes(count: int = 256, lo: int = 64, hi: int = 1024, seed: int = 4) -> np.ndarray:
    """Problem sizes n_i = round(exp(U[ln lo, ln hi])), one draw per problem."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.rint(np.exp(x)).astype(np.int64), lo, hi)


def serving_stream(count: int = 2000, qps: float = 10.0, lo: int = 128, hi: int = 4096,
                   big: int = 16384, big_frac: float = 0.02, seed: int = 5):
    """Poisson arrival times (s) and sizes for a request stream.

    Sizes are log-uniform in [lo, hi] with probability 1 - big_frac, else big.
    Returns (arrival_times, sizes)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps)
    x = rng.uniform(math.log(lo), math.log(hi), size=count)
    sizes = np.rint(np.exp(x)).astype(np.int64)
    is_big = rng.uniform(0.0, 1.0, size=count) < big_frac
    sizes = np.where(is_big, big, sizes)
    return t, sizes
