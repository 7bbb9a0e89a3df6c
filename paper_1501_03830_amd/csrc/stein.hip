// Eigenpairs of the real symmetric tridiagonal T_s = -i D^H T D =
// tridiag(alpha, 0, alpha), D = diag(i^k) (Algorithm 3 step 2; Section 3.3,
// remark 2).  Only the n positive eigenvalues and their eigenvectors are
// computed, as in the paper:
//
//  * bisection with Sturm counts, one eigenvalue per thread.  The recurrence
//    q_0 = -x,  q_k = -x - alpha_{k-1}^2 / q_{k-1}  (pivots smaller than
//    pivmin replaced by -pivmin) counts the eigenvalues below x; T_s is
//    nonsingular, so exactly n eigenvalues are negative and the j-th positive
//    one is the (n+j)-th smallest.  Intervals start at [0, Gershgorin bound]
//    and are halved to a relative width of 2 eps.
//  * inverse iteration, one eigenvector per thread: Gaussian elimination with
//    partial pivoting of T_s - sigma I (factors kept in HBM, interleaved over
//    the eigenvectors so that every access is coalesced), three solves from a
//    pseudo-random start.  Shifts closer than 10 eps |lambda| are pushed apart.
//  * reorthogonalisation inside clusters (eigenvalues closer than
//    1e-3 ||T_s||_1): Gram-Schmidt in ascending order, realised as a Cholesky
//    QR of the Gram matrix with the entries between different clusters
//    removed (the Q factor of that QR is exactly the Gram-Schmidt result).
//    Inside a cluster, pairs farther apart than REORTH_BAND ||T_s||_1 are
//    removed too: inverse iteration already leaves them orthogonal to about
//    eps / REORTH_BAND, the Gram matrix becomes banded in eigenvalue order,
//    its Cholesky factor has no fill outside the band, and the products skip
//    the tiles outside it (a long chain of close eigenvalues, e.g. most of
//    the spectrum at n = 8192, no longer costs a dense n x n Cholesky QR).
#include <cfloat>

#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr double EPS = DBL_EPSILON;   // 2^-52
constexpr double SAFMIN = DBL_MIN;

// scal[0] = pivmin, scal[1] = Gershgorin bound ||T_s||_1, scal[2] = max alpha^2
__global__ __launch_bounds__(1024) void k_tridiag_prep(const Prob* __restrict__ probs) {
  __shared__ double smax[16], sg[16];
  const Prob& P = probs[blockIdx.z];
  const int N = P.N;
  const BSE_GLOBAL double* __restrict__ alpha = gbl(P.alpha);
  BSE_GLOBAL double* __restrict__ e2 = gbl(P.e2);
  BSE_GLOBAL double* __restrict__ scal = gbl(P.scal);
  double m = 0.0, g = 0.0;
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const double a = (k < N - 1) ? alpha[k] : 0.0;
    if (k < N - 1) e2[k] = a * a;
    m = fmax(m, a * a);
    const double left = (k > 0) ? fabs(alpha[k - 1]) : 0.0;
    g = fmax(g, left + fabs(a));
  }
  for (int off = 32; off >= 1; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off, 64));
    g = fmax(g, __shfl_xor(g, off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smax[w] = m;
    sg[w] = g;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0, gg = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      mm = fmax(mm, smax[i]);
      gg = fmax(gg, sg[i]);
    }
    scal[0] = SAFMIN * fmax(1.0, mm);
    scal[1] = gg;
    scal[2] = mm;
  }
}

// The loads of alpha^2 are issued eight steps at a time, ahead of the
// dependent divisions; the arithmetic and its order are those of the plain
// recurrence.
template <class Ptr>
__device__ inline int sturm_count(Ptr e2, int N, double x, double pivmin) {
  double q = -x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  int k = 1;
  for (; k + 8 <= N; k += 8) {
    double e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = e2[k - 1 + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      q = -x - e[u] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
    }
  }
  for (; k < N; ++k) {
    q = -x - e2[k - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Bisection for eigenvalue j of T_s (the (n+j)-th smallest), run as
// multisection by a group of 2^L lanes with results bit for bit those of
// plain bisection: each round, lane g evaluates the Sturm count at node g + 1
// of the next L levels of the bisection tree (heap order, midpoints formed
// exactly as the sequential loop forms them), then every lane replays the L
// bisection steps -- tolerance test, midpoint, count, half -- reading each
// count from the lane that owns the node.  One round costs one Sturm count
// instead of L; with 8 lanes per eigenvalue (L = 3) a solve of order n runs
// n/8 wavefronts, about one per SIMD at n = 8192 (16 lanes gave two per SIMD
// and fewer rounds, and measured slower: the counts are chains of dependent
// divisions).  The 2^L - 1 counts of a round buy L levels, so multisection
// spends (2^L)/L lane-counts per level against 1 for plain bisection: a
// launch with enough eigenvalues to fill the device (a batch) runs L = 0,
// one lane per eigenvalue and the plain loop, with the same results.
template <int L>
__global__ __launch_bounds__(64) void k_bisect(const Prob* __restrict__ probs) {
  constexpr int LANES = 1 << L;
  const Prob& P = probs[blockIdx.z];
  const int N = P.N, n = P.n;
  const int lane = threadIdx.x & 63;
  const int g = lane % LANES;
  const int base = lane - g;   // first lane of this eigenvalue's group
  const int j = (int)(((long)blockIdx.x * blockDim.x + threadIdx.x) / LANES);
  if (j >= n) return;   // the whole group
  const BSE_CONST double* __restrict__ e2 = ro(P.e2);
  const BSE_CONST double* __restrict__ scal = ro(P.scal);
  BSE_GLOBAL double* __restrict__ lam = gbl(P.lambda);
  const double pivmin = scal[0];
  double lo = 0.0;
  double hi = scal[1] * (1.0 + 4.0 * EPS) + 4.0 * pivmin;
  const int target = n + j;
  if constexpr (L == 0) {
    for (int steps = 0;; ++steps) {
      const double tol = fmax(2.0 * EPS * fmax(fabs(lo), fabs(hi)), 4.0 * pivmin);
      if (hi - lo <= tol || steps >= 200) break;
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) {
        hi = lo;
        break;
      }
      if (sturm_count(e2, N, mid, pivmin) <= target) lo = mid;
      else hi = mid;
    }
    lam[j] = 0.5 * (lo + hi);
    return;
  } else {
    const int node = g + 1;
    const int depth = 31 - __clz(node);
    int steps = 0;
    bool done = false;
    while (!done) {   // uniform inside the group
      double a = lo, b = hi;
      for (int lev = depth - 1; lev >= 0; --lev) {
        const double m = 0.5 * (a + b);
        if ((node >> lev) & 1) a = m;
        else b = m;
      }
      const int c = (node < (1 << L)) ? sturm_count(e2, N, 0.5 * (a + b), pivmin) : 0;
      int nd = 1;
      for (int lev = 0; lev < L; ++lev) {
        const double tol = fmax(2.0 * EPS * fmax(fabs(lo), fabs(hi)), 4.0 * pivmin);
        if (hi - lo <= tol || steps >= 200) {
          done = true;
          break;
        }
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) {
          hi = lo;
          done = true;
          break;
        }
        const int cn = __shfl(c, base + nd - 1, 64);
        ++steps;
        if (cn <= target) {
          lo = mid;
          nd = 2 * nd + 1;
        } else {
          hi = mid;
          nd = 2 * nd;
        }
      }
    }
    if (g == 0) lam[j] = 0.5 * (lo + hi);
  }
}

__global__ void k_shifts(const Prob* __restrict__ probs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const Prob& P = probs[blockIdx.z];
  const int n = P.n;
  const BSE_CONST double* __restrict__ lam = ro(P.lambda);
  BSE_GLOBAL double* __restrict__ shift = gbl(P.shift);
  double prev = lam[0];
  shift[0] = prev;
  for (int j = 1; j < n; ++j) {
    double sj = lam[j];
    const double pertol = 10.0 * EPS * fabs(sj);
    if (sj - prev < pertol) sj = prev + pertol;
    shift[j] = sj;
    prev = sj;
  }
}

__device__ inline double hash_uniform(unsigned long long key) {
  // splitmix64 finaliser, mapped to [-1, 1)
  unsigned long long z = key + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__device__ inline double perturb(double d, double pert) {
  return (fabs(d) < pert) ? (d < 0.0 ? -pert : pert) : d;
}

// Eigenvalues closer than this many eps |lambda| to a neighbour are
// numerically degenerate for the twisted factorisations (both would see the
// same shifted matrix and return the same vector): inverse iteration, whose
// pushed-apart shifts and independent starts separate them, computes those.
constexpr double TWIST_DEGEN = 1000.0;

__device__ inline bool twist_degenerate(const BSE_CONST double* __restrict__ lam, int j, int n) {
  const double lj = lam[j];
  const double tol = TWIST_DEGEN * EPS * fabs(lj);
  return (j > 0 && lj - lam[j - 1] <= tol) || (j + 1 < n && lam[j + 1] - lj <= tol);
}

// Workspace per eigenvector j (n of them), element k at [k*n + j]:
//   fd (U diagonal), fu (first superdiagonal), fu2 (second), fl (multiplier),
//   fs (row interchange flag).  Vt holds the iterate.
__global__ __launch_bounds__(64) void k_invit(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  const int N = P.N, n = P.n;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  // with BSE_EIGVEC_TWISTED, only the degenerate eigenvalues (k_twisted
  // computed every other vector)
  if ((P.flags & BSE_EIGVEC_TWISTED) && !twist_degenerate(ro(P.lambda), j, n)) return;
  const BSE_CONST double* __restrict__ alpha = ro(P.alpha);
  const BSE_CONST double* __restrict__ scal = ro(P.scal);
  const BSE_GLOBAL double* __restrict__ shift = gbl(P.shift);
  const long sz = (long)N * n;
  BSE_GLOBAL double* __restrict__ fd = gbl(P.inv);
  BSE_GLOBAL double* __restrict__ fu = gbl(P.inv + sz);
  BSE_GLOBAL double* __restrict__ fu2 = gbl(P.inv + 2 * sz);
  BSE_GLOBAL double* __restrict__ fl = gbl(P.inv + 3 * sz);
  BSE_GLOBAL unsigned char* __restrict__ fs = gbl(reinterpret_cast<unsigned char*>(P.inv + 4 * sz));
  BSE_GLOBAL double* __restrict__ Vt = gbl(P.Vt);
  const long ldn = n;
  const double pert = EPS * fmax(scal[1], SAFMIN);
  const double sh = shift[j];

  // factorisation (LAPACK dgttrf scheme) of T_s - sh I
  double cur_d = -sh;
  double cur_du = (N > 1) ? alpha[0] : 0.0;
  for (int k = 0; k < N - 1; ++k) {
    const double dlk = alpha[k];
    const double next_d = -sh;
    const double next_du = (k + 1 < N - 1) ? alpha[k + 1] : 0.0;
    const long o = (long)k * ldn + j;
    if (fabs(cur_d) >= fabs(dlk)) {
      const double dk = perturb(cur_d, pert);
      const double l = dlk / dk;
      fd[o] = dk;
      fu[o] = cur_du;
      fu2[o] = 0.0;
      fl[o] = l;
      fs[o] = 0;
      cur_d = next_d - l * cur_du;
      cur_du = next_du;
    } else {
      const double l = cur_d / dlk;
      fd[o] = perturb(dlk, pert);
      fu[o] = next_d;
      fu2[o] = next_du;
      fl[o] = l;
      fs[o] = 1;
      cur_d = cur_du - l * next_d;
      cur_du = -l * next_du;
    }
  }
  fd[(long)(N - 1) * ldn + j] = perturb(cur_d, pert);

  // start vector
  for (int k = 0; k < N; ++k)
    Vt[(long)k * ldn + j] = hash_uniform(((unsigned long long)j << 32) ^ (unsigned long long)k ^ 0x5bd1e995ull);

  // Both solves run in blocks of 32 steps whose loads (the factors and
  // the entries of the iterate not yet overwritten) are issued before the
  // dependent arithmetic; the arithmetic is that of the step-by-step loops.
  constexpr int UB = 32;
  for (int it = 0; it < 3; ++it) {
    // forward: apply the row interchanges and multipliers
    double cur = Vt[j];
    int k = 0;
    for (; k + UB <= N - 1; k += UB) {
      double nx[UB], lv[UB];
      unsigned char sv[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const long o = (long)(k + u) * ldn + j;
        nx[u] = Vt[o + ldn];
        lv[u] = fl[o];
        sv[u] = fs[o];
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        double outk;
        if (sv[u]) {
          outk = nx[u];
          cur = cur - lv[u] * nx[u];
        } else {
          outk = cur;
          cur = nx[u] - lv[u] * cur;
        }
        Vt[(long)(k + u) * ldn + j] = outk;
      }
    }
    for (; k < N - 1; ++k) {
      const long o = (long)k * ldn + j;
      const double nxt = Vt[o + ldn];
      const double l = fl[o];
      double outk;
      if (fs[o]) {
        outk = nxt;
        cur = cur - l * nxt;
      } else {
        outk = cur;
        cur = nxt - l * cur;
      }
      Vt[o] = outk;
    }
    Vt[(long)(N - 1) * ldn + j] = cur;
    // back substitution with the upper factor
    double x2 = 0.0, x1 = 0.0, ss = 0.0;
    k = N - 1;
    for (; k - UB + 1 >= 0; k -= UB) {
      double vv[UB], u1[UB], u2[UB], dd[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const long o = (long)(k - u) * ldn + j;
        vv[u] = Vt[o];
        u1[u] = fu[o];
        u2[u] = fu2[o];
        dd[u] = fd[o];
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int kk = k - u;
        double v = vv[u];
        if (kk <= N - 2) v -= u1[u] * x1;
        if (kk <= N - 3) v -= u2[u] * x2;
        const double x = v / dd[u];
        Vt[(long)kk * ldn + j] = x;
        ss += x * x;
        x2 = x1;
        x1 = x;
      }
    }
    for (; k >= 0; --k) {
      const long o = (long)k * ldn + j;
      double v = Vt[o];
      if (k <= N - 2) v -= fu[o] * x1;
      if (k <= N - 3) v -= fu2[o] * x2;
      const double x = v / fd[o];
      Vt[o] = x;
      ss += x * x;
      x2 = x1;
      x1 = x;
    }
    const double inv = 1.0 / sqrt(ss);
    // normalise, UB loads in flight at a time (a load-multiply-store chain per
    // element waits out a full memory round trip each)
    k = 0;
    for (; k + UB <= N; k += UB) {
      double vv[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) vv[u] = Vt[(long)(k + u) * ldn + j];
#pragma unroll
      for (int u = 0; u < UB; ++u) Vt[(long)(k + u) * ldn + j] = vv[u] * inv;
    }
    for (; k < N; ++k) Vt[(long)k * ldn + j] *= inv;
  }
}

// Eigenvector j of T_s by a twisted factorisation (the per-vector step of
// MRRR, Section 3.3's alternative to inverse iteration), one thread per
// eigenvalue, for problems with BSE_EIGVEC_TWISTED:
//   d+_0 = -lam,  d+_{k+1} = -lam - alpha_k^2 / d+_k       (top down)
//   d-_{N-1} = -lam,  d-_k = -lam - alpha_k^2 / d-_{k+1}   (bottom up)
//   gamma_k = d+_k + d-_k + lam,  r = argmin |gamma_k|
//   z_r = 1, z_k = -(alpha_k / d+_k) z_{k+1} (k < r),
//   z_{k+1} = -(alpha_k / d-_{k+1}) z_k (k >= r), then normalised.
// Pivots below pivmin in modulus become -pivmin (as in the Sturm count); a
// recurrence that meets z = 0 takes the row equation two entries away (0
// where that row's coupling is exactly zero, a split of T_s).  d+
// and d- go to the first two factor arrays of inverse iteration ([k*n + j],
// coalesced over the eigenvalues); loads are issued UB steps ahead of the
// dependent arithmetic.  Degenerate eigenvalues are left to inverse
// iteration (k_invit runs after this kernel and writes only those).
__global__ __launch_bounds__(64) void k_twisted(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  if (!(P.flags & BSE_EIGVEC_TWISTED)) return;   // uniform
  const int N = P.N, n = P.n;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const BSE_CONST double* __restrict__ alpha = ro(P.alpha);
  const BSE_CONST double* __restrict__ lamv = ro(P.lambda);
  if (twist_degenerate(lamv, j, n)) return;
  const double pivmin = ro(P.scal)[0];
  const long sz = (long)N * n;
  BSE_GLOBAL double* __restrict__ dp = gbl(P.inv);
  BSE_GLOBAL double* __restrict__ dm = gbl(P.inv + sz);
  BSE_GLOBAL double* __restrict__ Vt = gbl(P.Vt);
  const long ldn = n;
  const double lam = lamv[j];
  auto fix = [&](double q) { return fabs(q) < pivmin ? -pivmin : q; };
  constexpr int UB = 32;

  // top down
  double d = fix(-lam);
  dp[j] = d;
  {
    int k = 0;
    for (; k + UB <= N - 1; k += UB) {
      double a[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) a[u] = alpha[k + u];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        d = fix(-lam - a[u] * a[u] / d);
        dp[(long)(k + u + 1) * ldn + j] = d;
      }
    }
    for (; k < N - 1; ++k) {
      const double a = alpha[k];
      d = fix(-lam - a * a / d);
      dp[(long)(k + 1) * ldn + j] = d;
    }
  }
  // bottom up, with the twists
  d = fix(-lam);
  dm[(long)(N - 1) * ldn + j] = d;
  double gmin = fabs(dp[(long)(N - 1) * ldn + j] + d + lam);
  int r = N - 1;
  {
    int k = N - 2;
    for (; k - UB + 1 >= 0; k -= UB) {
      double a[UB], pk[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        a[u] = alpha[k - u];
        pk[u] = dp[(long)(k - u) * ldn + j];
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        d = fix(-lam - a[u] * a[u] / d);
        dm[(long)(k - u) * ldn + j] = d;
        const double g = fabs(pk[u] + d + lam);
        if (g < gmin) {
          gmin = g;
          r = k - u;
        }
      }
    }
    for (; k >= 0; --k) {
      const double a = alpha[k];
      d = fix(-lam - a * a / d);
      dm[(long)k * ldn + j] = d;
      const double g = fabs(dp[(long)k * ldn + j] + d + lam);
      if (g < gmin) {
        gmin = g;
        r = k;
      }
    }
  }
  // the vector: upwards from r, then downwards, UB steps of loads at a time
  // (a step's factor does not depend on the vector, only its use does)
  double ss = 1.0;
  Vt[(long)r * ldn + j] = 1.0;
  {
    double z1 = 1.0, z2 = 0.0;   // z_{k+1}, z_{k+2}
    int k = r - 1;
    for (; k - UB + 1 >= 0; k -= UB) {
      double pk[UB], a[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        pk[u] = dp[(long)(k - u) * ldn + j];
        a[u] = alpha[k - u];
      }
      const double a_top = (k + 1 <= N - 2) ? alpha[k + 1] : 0.0;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const double an = (u == 0) ? a_top : a[u - 1];   // alpha_{k-u+1}
        const double z = (z1 != 0.0) ? -(a[u] / pk[u]) * z1 : (a[u] != 0.0 ? -(an / a[u]) * z2 : 0.0);
        Vt[(long)(k - u) * ldn + j] = z;
        ss += z * z;
        z2 = z1;
        z1 = z;
      }
    }
    for (; k >= 0; --k) {
      const double a = alpha[k];
      const double an = (k + 1 <= N - 2) ? alpha[k + 1] : 0.0;
      const double z = (z1 != 0.0) ? -(a / dp[(long)k * ldn + j]) * z1 : (a != 0.0 ? -(an / a) * z2 : 0.0);
      Vt[(long)k * ldn + j] = z;
      ss += z * z;
      z2 = z1;
      z1 = z;
    }
  }
  {
    double z1 = 1.0, z0 = 0.0;   // z_k, z_{k-1}
    int k = r;
    for (; k + UB <= N - 1; k += UB) {
      double mk[UB], a[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        mk[u] = dm[(long)(k + u + 1) * ldn + j];
        a[u] = alpha[k + u];
      }
      const double a_bot = (k >= 1) ? alpha[k - 1] : 0.0;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const double ap = (u == 0) ? a_bot : a[u - 1];   // alpha_{k+u-1}
        const double z = (z1 != 0.0) ? -(a[u] / mk[u]) * z1 : (a[u] != 0.0 ? -(ap / a[u]) * z0 : 0.0);
        Vt[(long)(k + u + 1) * ldn + j] = z;
        ss += z * z;
        z0 = z1;
        z1 = z;
      }
    }
    for (; k < N - 1; ++k) {
      const double a = alpha[k];
      const double ap = (k >= 1) ? alpha[k - 1] : 0.0;
      const double z = (z1 != 0.0) ? -(a / dm[(long)(k + 1) * ldn + j]) * z1 : (a != 0.0 ? -(ap / a) * z0 : 0.0);
      Vt[(long)(k + 1) * ldn + j] = z;
      ss += z * z;
      z0 = z1;
      z1 = z;
    }
  }
  const double inv = 1.0 / sqrt(ss);
  int k = 0;
  for (; k + UB <= N; k += UB) {
    double vv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) vv[u] = Vt[(long)(k + u) * ldn + j];
#pragma unroll
    for (int u = 0; u < UB; ++u) Vt[(long)(k + u) * ldn + j] = vv[u] * inv;
  }
  for (; k < N; ++k) Vt[(long)k * ldn + j] *= inv;
}

// cid[j] = index of the cluster of eigenvalue j (consecutive gaps <= ortol)
__global__ __launch_bounds__(1024) void k_cluster_ids(const Prob* __restrict__ probs) {
  __shared__ int sums[1024];
  const Prob& P = probs[blockIdx.z];
  const int n = P.n;
  const BSE_GLOBAL double* __restrict__ lam = gbl(P.lambda);
  const BSE_CONST double* __restrict__ scal = ro(P.scal);
  BSE_GLOBAL int* __restrict__ cid = gbl(P.cid);
  const bool mixed = P.prec == BSE_PREC_FP32_REFINE;
  const double ortol = (mixed ? 1e-10 : 1e-3) * scal[1];
  const int T = blockDim.x;
  const int chunk = (n + T - 1) / T;
  const int b = threadIdx.x * chunk, e = min(n, b + chunk);
  int local = 0;
  for (int jj = b; jj < e; ++jj)
    if (jj > 0 && lam[jj] - lam[jj - 1] > ortol) ++local;
  sums[threadIdx.x] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < T; ++t) {
      const int v = sums[t];
      sums[t] = run;
      run += v;
    }
    // run = gaps above ortol; fewer than n - 1 means a cluster
    *gbl(P.reorth) = (!mixed || run < n - 1) ? 1 : 0;
    *gbl(P.gdef) = 0.0;
    gbl(P.info)[1] = 0;   // no Gram-Schmidt failure yet (it may be skipped)
  }
  __syncthreads();
  int run = sums[threadIdx.x];
  for (int jj = b; jj < e; ++jj) {
    if (jj > 0 && lam[jj] - lam[jj - 1] > ortol) ++run;
    cid[jj] = run;
  }
}

__global__ __launch_bounds__(256) void k_mask_gram(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  if (*gbl(P.reorth) == 0) return;   // uniform: no cluster to orthogonalise
  const int n = P.n;
  const long ldg = n;
  BSE_GLOBAL double* __restrict__ G = gbl(P.inv);
  const BSE_GLOBAL int* __restrict__ cid = gbl(P.cid);
  const BSE_GLOBAL double* __restrict__ lam = gbl(P.lambda);
  const double band = REORTH_BAND * gbl(P.scal)[1];
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  __shared__ double wmax[4];
  double def = 0.0;   // largest |G - I| over this thread's entries inside a cluster
  const int cr = r < n ? cid[r] : -1;
  const double lr = r < n ? lam[r] : 0.0;
  for (int q = 0; q < 16 && r < n; ++q) {
    const long c = c0 + q;
    if (c >= n || c > r) break;
    // entries between clusters, and pairs farther apart than the band (whose
    // tiles the Gram product may have skipped), are dropped
    if (cid[c] != cr || lr - lam[c] > band) G[r + c * ldg] = 0.0;
    else def = fmax(def, fabs(G[r + c * ldg] - (c == r ? 1.0 : 0.0)));
  }
  // the workgroup's largest defect joins the problem's (non-negative doubles
  // order like their bit patterns)
  for (int off = 32; off >= 1; off >>= 1) def = fmax(def, __shfl_xor(def, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = def;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    if (m > 0.0)
      __hip_atomic_fetch_max((BSE_GLOBAL unsigned long long*)P.gdef, (unsigned long long)__double_as_longlong(m),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The second Cholesky QR pass runs only where the first Gram matrix was far
// from the identity.  Its error after one pass grows like u cond(V)^2, and
// ||G - I||_2 <= n max |G_ij - delta_ij| <= 1e-2 bounds cond(V)^2 by 1.03.
__global__ void k_reorth_gate(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.x];
  if (threadIdx.x == 0 && *gbl(P.reorth) != 0 && (double)P.n * *gbl(P.gdef) <= 1e-2) *gbl(P.reorth) = 0;
}

__global__ __launch_bounds__(256) void k_transpose(int rows, int cols, const double* __restrict__ src, long lds,
                                                   double* __restrict__ dst, long ldd) {
  __shared__ double t[64][65];
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int i = idx & 63, jj = idx >> 6;
    const int r = r0 + i, c = c0 + jj;
    t[jj][i] = (r < rows && c < cols) ? src[(long)r + (long)c * lds] : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int i = idx & 63, jj = idx >> 6;   // dst row = c0 + i, dst col = r0 + jj
    const int dr = c0 + i, dc = r0 + jj;
    if (dr < cols && dc < rows) dst[(long)dr + (long)dc * ldd] = t[i][jj];
  }
}

}  // namespace

int bisect_batched(hipStream_t s, const Batch& b) {
  if (b.count <= 0) return 0;
  const int n0 = b.maxn();
  BSE_LAUNCH(k_tridiag_prep, dim3(1, 1, (unsigned)b.count), 1024, 0, s, b.dev);
  // eigenvalues of the launch: multisection (8 lanes each) while it leaves
  // the device at most two wavefronts per SIMD, else plain bisection
  long neig = 0;
  for (int i = 0; i < b.count; ++i) neig += b.host[i].n;
  if (neig * 8 <= 131072)
    BSE_LAUNCH(k_bisect<3>, dim3((unsigned)(((long)n0 * 8 + 63) / 64), 1, (unsigned)b.count), 64, 0, s, b.dev);
  else
    BSE_LAUNCH(k_bisect<0>, dim3((unsigned)((n0 + 63) / 64), 1, (unsigned)b.count), 64, 0, s, b.dev);
  return 0;
}

int invit_batched(hipStream_t s, const Batch& b) {
  if (b.count <= 0) return 0;
  const int n0 = b.maxn();
  // launched whatever the flags (its problems without BSE_EIGVEC_TWISTED
  // exit at once): the launch sequence depends on the shape alone, as a
  // captured graph of the chain requires
  BSE_LAUNCH(k_twisted, dim3((unsigned)((n0 + 63) / 64), 1, (unsigned)b.count), 64, 0, s, b.dev);
  BSE_LAUNCH(k_shifts, dim3(1, 1, (unsigned)b.count), 64, 0, s, b.dev);
  BSE_LAUNCH(k_invit, dim3((unsigned)((n0 + 63) / 64), 1, (unsigned)b.count), 64, 0, s, b.dev);
  return 0;
}

int reorth_batched(hipStream_t s, const Batch& b, const int* dflags, int* hflags, int nslots) {
  if (b.count <= 0) return 0;
  const int n0 = b.maxn();
  BSE_LAUNCH(k_cluster_ids, dim3(1, 1, (unsigned)b.count), 1024, 0, s, b.dev);
  if (b.host[0].prec == BSE_PREC_FP32_REFINE) {
    // skip the launches altogether when no problem has a near-degenerate
    // cluster (otherwise the kernels skip the problems without one)
    BSE_HIP(hipMemcpyAsync(hflags, dflags, nslots * sizeof(int), hipMemcpyDeviceToHost, s));
    BSE_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int i = 0; i < b.count; ++i) any = any || hflags[b.host[i].reorth - dflags] != 0;
    if (!any) return 0;
  }
  // Two passes of Cholesky QR ("twice is enough"): the second restores full
  // orthogonality when a degenerate cluster's start vectors were close, and
  // is skipped (its kernels return at once) when the first Gram matrix shows
  // the vectors were already close to orthonormal.
  const dim3 g2((unsigned)((n0 + 63) / 64), (unsigned)((n0 + 63) / 64), (unsigned)b.count);
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      BSE_LAUNCH(k_reorth_gate, dim3((unsigned)b.count), 64, 0, s, b.dev);
    }
    // G = Vt Vt^T (lower, band tiles), then drop the entries between
    // clusters and outside the band
    BSE_TRY(gemm_batched(s, b, b.count, GOP_GRAM, 0));
    BSE_LAUNCH(k_mask_gram, g2, 256, 0, s, b.dev);
    BSE_TRY(potrf_batched(s, b, 1, pass == 0));
    // Vt <- L^{-1} Vt: blocked forward substitution over 128-row blocks, each
    // two direct solves with 64 x 64 diagonal blocks around the update of the
    // block's second half, then one update (K = 128) of the rows below
    auto count_above = [&](int from, int k) {
      int c = 0;
      while (c < from && b.host[c].n > k) ++c;
      return c;
    };
    for (int b0 = 0; b0 < n0; b0 += 128) {
      const int nact = count_above(b.count, b0);
      BSE_TRY(trsm_cols_batched(s, b, nact, b0));
      const int nrest = count_above(nact, b0 + 64);
      if (nrest == 0) continue;
      BSE_TRY(gemm_batched(s, b, nrest, GOP_GRAM_UPD_PANEL, b0));
      BSE_TRY(trsm_cols_batched(s, b, nrest, b0 + 64));
      const int nrest2 = count_above(nrest, b0 + 128);
      if (nrest2 == 0) continue;
      BSE_TRY(gemm_batched(s, b, nrest2, GOP_GRAM_UPD, b0));
    }
  }
  return 0;
}

int transpose_to(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst, long ldd) {
  dim3 g((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
  BSE_LAUNCH(k_transpose, g, 256, 0, s, rows, cols, src, lds, dst, ldd);
  return 0;
}

}  // namespace bse
