// Real embedding, Cholesky factorisation and the skew-symmetric W.
//
//   Algorithm 1 step 1 (Theorem 2, eq. embedding):
//       M = [Re(A+B)  Im(A-B); -Im(A+B)  Re(A-B)]
//   Algorithm 1 step 2:  M = L L^T   (blocked, right-looking, lower)
//   Algorithm 1 step 3:  W = L^T J L  with J = [0 I; -I 0]
//
// With L = [L11 0; L21 L22] the blocks of W are
//       W11 = L11^T L21 - (L11^T L21)^T,   W21 = -L22^T L11,   W22 = 0,
// so W costs two triangular-by-dense products instead of a full N^3 product
// (the zero W22 block follows from the block form of L^T J L).
#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int TB = 64;
// the sub-panel index rides in the low bits of the panel products' step
static_assert(CHOL_PANEL % TB == 0 && CHOL_PANEL / TB < TB, "Cholesky panel of whole 64-column sub-panels");

__global__ __launch_bounds__(256) void k_build_M(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  const int n = P.n, N = P.N;
  const int r = blockIdx.x * TB + (threadIdx.x & 63);
  const int cbase = blockIdx.y * TB + (threadIdx.x >> 6) * 16;
  if (r >= N) return;
  const BSE_GLOBAL double* __restrict__ A = gbl(P.A);
  // no B: the Tamm-Dancoff Hamiltonian (B = 0)
  const BSE_GLOBAL double* __restrict__ B = gbl(P.B);
  const bool hasB = P.B != nullptr;
  // real A, B (eq. H-real): M = blkdiag(A + B, A - B), whose Cholesky
  // factor is blkdiag(L1, L2) with the two factors of Algorithm 2 step 1
  const bool real_in = (P.flags & FLAG_REAL_IN) != 0;
  const long lda = P.lda, ldb = P.ldb, ldm = P.ld;
  BSE_GLOBAL double* __restrict__ M = gbl(P.L);
  for (int q = 0; q < 16; ++q) {
    const int c = cbase + q;
    if (c >= N) break;
    double val = 0.0;
    if (r >= c) {
      const int bi = r >= n, bj = c >= n;
      const int i = r - bi * n, j = c - bj * n;
      double ar, ai, br, bim;
      if (real_in) {
        const long ia = (i >= j) ? (long)i + (long)j * lda : (long)j + (long)i * lda;
        const long ib = (i >= j) ? (long)i + (long)j * ldb : (long)j + (long)i * ldb;
        ar = A[ia];
        ai = 0.0;
        br = B[ib];
        bim = 0.0;
      } else if (i >= j) {
        const long ia = 2 * ((long)i + (long)j * lda), ib = 2 * ((long)i + (long)j * ldb);
        ar = A[ia];
        ai = A[ia + 1];
        br = hasB ? B[ib] : 0.0;
        bim = hasB ? B[ib + 1] : 0.0;
      } else {  // upper triangle: A[i,j] = conj(A[j,i]), B[i,j] = B[j,i]
        const long ia = 2 * ((long)j + (long)i * lda), ib = 2 * ((long)j + (long)i * ldb);
        ar = A[ia];
        ai = -A[ia + 1];
        br = hasB ? B[ib] : 0.0;
        bim = hasB ? B[ib + 1] : 0.0;
      }
      if (i == j) ai = 0.0;  // a Hermitian diagonal is real
      if (!bi && !bj) val = ar + br;          // Re(A+B)
      else if (bi && !bj) val = -(ai + bim);  // -Im(A+B)
      else val = ar - br;                     // Re(A-B)
    }
    M[(long)r + (long)c * ldm] = val;
  }
}

__global__ void k_reset_info(const Prob* __restrict__ probs, int sel) {
  if (threadIdx.x == 0) gbl(probs[blockIdx.z].info)[sel] = 0;
}

__device__ inline void chol_matrix(const Prob& P, int sel, BSE_GLOBAL double*& M, long& ld, int& N) {
  if (sel == 0) {
    M = gbl(P.L);
    ld = P.ld;
    N = P.N;
  } else {
    M = gbl(P.inv);
    ld = P.n;
    N = P.n;
  }
}

// Unblocked Cholesky of the diagonal block at (k0, k0): one wavefront, lane
// t holds row t of the block in registers.  Step j publishes column j in LDS
// (double-buffered, so one barrier per step), every lane takes the pivot from
// there, scales its own entry by the reciprocal of the root (as dpotf2 does)
// and subtracts its rank-1 share from its entries right of j; lane c's entry
// of the scaled column is formed by the other lanes with the same expression,
// so all lanes use identical values.  Entries above the diagonal are scratch
// and are never stored.
// x of lane l, bit for bit, in every lane (the readlane builtin moves one
// 32-bit word, so a double goes as its two halves)
__device__ inline double readlane_f64(double x, int l) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffLL), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(TB) void k_potf2(const Prob* __restrict__ probs, int sel, int k0) {
  const Prob& P = probs[blockIdx.z];
  BSE_GLOBAL double* M;
  long ld;
  int N;
  chol_matrix(P, sel, M, ld, N);
  BSE_GLOBAL int* info = gbl(P.info + sel);
  if (k0 >= N || *info != 0) return;
  if (sel == 1 && *gbl(P.reorth) == 0) return;   // no cluster Gram-Schmidt
  const int nbk = min(TB, N - k0);
  const int t = threadIdx.x;
  // one wavefront, lane t holding row t: column j's entries reach every lane
  // by readlane (no LDS round trip and no barrier per column)
  double a[TB];
#pragma unroll
  for (int c = 0; c < TB; ++c)
    a[c] = (t < nbk && c <= t) ? M[(long)(k0 + t) + (long)(k0 + c) * ld] : 0.0;
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    if (j < nbk) {   // uniform
      const double colj = a[j];   // column j before scaling (row t)
      const double piv = readlane_f64(colj, j);
      if (!(piv > 0.0) || !isfinite(piv)) {
        if (t == 0) *info = k0 + j + 1;
        return;  // uniform: every lane read the same pivot
      }
      const double ljj = sqrt(piv);
      const double rinv = 1.0 / ljj;
      a[j] = (t == j) ? ljj : colj * rinv;
      // L[c][j] is lane c's scaled entry (the same product colj * rinv)
#pragma unroll
      for (int c = j + 1; c < TB; ++c) a[c] -= a[j] * readlane_f64(a[j], c);
    }
  }
#pragma unroll
  for (int c = 0; c < TB; ++c)
    if (t < nbk && c <= t) M[(long)(k0 + t) + (long)(k0 + c) * ld] = a[c];
}

// For every lower tile pair (R, C), R >= C, of the leading nrows x nrows
// part of P.W (nrows = n in mode 0, N in mode 1):
//  mode 0: lower <- T1 - T2^T  (T1 = tile (R,C), T2 = tile (C,R)); diagonal 0;
//          with `full` the upper triangle receives the negated transpose.
//  mode 1: upper <- -lower^T (completion of a skew matrix from its lower part)
__global__ __launch_bounds__(256) void k_skew_pairs(const Prob* __restrict__ probs, int mode, int full) {
  __shared__ double t1[TB][TB + 1];
  __shared__ double t2[TB][TB + 1];
  const Prob& P = probs[blockIdx.z];
  const int nrows = (mode == 0) ? P.n : P.N;
  const long nt = (nrows + TB - 1) / TB;
  if ((long)blockIdx.x >= nt * (nt + 1) / 2) return;
  BSE_GLOBAL double* __restrict__ W = gbl(P.W);
  const long ld = P.ld;
  int R, C;
  tri_index(blockIdx.x, R, C);
  const int tid = threadIdx.x;
  const int r0 = R * TB, c0 = C * TB;
  for (int idx = tid; idx < TB * TB; idx += 256) {
    const int i = idx & 63, j = idx >> 6;
    const int gi = r0 + i, gj = c0 + j;  // element of T1
    t1[j][i] = (gi < nrows && gj < nrows) ? W[(long)gi + (long)gj * ld] : 0.0;
    const int hi = c0 + i, hj = r0 + j;  // element of T2
    t2[j][i] = (mode == 0 && hi < nrows && hj < nrows) ? W[(long)hi + (long)hj * ld] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < TB * TB; idx += 256) {
    const int i = idx & 63, j = idx >> 6;
    const int gi = r0 + i, gj = c0 + j;
    if (gi >= nrows || gj >= nrows) continue;
    if (gi < gj) continue;
    double lo;
    if (gi == gj) lo = 0.0;
    else lo = (mode == 0) ? (t1[j][i] - t2[i][j]) : t1[j][i];
    if (mode == 0) W[(long)gi + (long)gj * ld] = lo;
    if (full || mode == 1) W[(long)gj + (long)gi * ld] = -lo;
  }
}

// W22 = 0
__global__ __launch_bounds__(256) void k_zero_W22(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  const long n = P.n;
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= n) return;
  BSE_GLOBAL double* W22 = gbl(P.W + n + n * P.ld);
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    if (c >= n) break;
    W22[r + c * P.ld] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_copy(int m, int n, const double* __restrict__ src, long lds,
                                              double* __restrict__ dst, long ldd) {
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= m) return;
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    if (c >= n) break;
    dst[r + c * ldd] = src[r + c * lds];
  }
}

__global__ __launch_bounds__(256) void k_zero_upper(int n, double* __restrict__ dst, long ldd) {
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= n) return;
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    if (c >= n) break;
    if (r < c) dst[r + c * ldd] = 0.0;
  }
}

dim3 grid2d(long m, long n, int z = 1) {
  return dim3((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64), (unsigned)z);
}

}  // namespace

int build_M_batched(hipStream_t s, const Batch& b) {
  if (b.count <= 0) return 0;
  const long N = b.maxN();
  BSE_LAUNCH(k_build_M, grid2d(N, N, b.count), 256, 0, s, b.dev);
  return 0;
}

int copy_matrix(hipStream_t s, int m, int n, const double* src, long lds, double* dst, long ldd) {
  if (m <= 0 || n <= 0) return 0;
  BSE_LAUNCH(k_copy, grid2d(m, n), 256, 0, s, m, n, src, lds, dst, ldd);
  return 0;
}

int zero_upper(hipStream_t s, int N, double* A, long lda) {
  if (N <= 0) return 0;
  BSE_LAUNCH(k_zero_upper, grid2d(N, N), 256, 0, s, N, A, lda);
  return 0;
}

int potrf_batched(hipStream_t s, const Batch& b, int sel, bool reset_info) {
  if (b.count <= 0) return 0;
  if (reset_info) {
    BSE_LAUNCH(k_reset_info, dim3(1, 1, (unsigned)b.count), 64, 0, s, b.dev, sel);
  }
  // order of the factored matrix: N (sel 0) or n (sel 1); both sort with N
  auto order = [sel](const Prob& P) { return sel == 0 ? P.N : P.n; };
  const int Nmax = order(b.host[0]);
  const int SOPS = sel == 0 ? GOP_POTRF_SYRK : GOP_GRAM_SYRK;
  const int POPS = sel == 0 ? GOP_POTRF_PANEL : GOP_GRAM_PANEL;
  auto count_above = [&](int from, int k) {
    int c = 0;
    while (c < from && order(b.host[c]) > k) ++c;
    return c;
  };
  // Panels of CHOL_PANEL columns, each factored in 64-column sub-panels:
  // sub-panel h is first brought up to date with the sub-panels before it
  // (one product with K = 64 h), then its diagonal block is factored
  // (k_potf2) and the rows below it are solved (trsm_rows_batched).  The
  // trailing update then runs once per panel with K = CHOL_PANEL, so that
  // the product's tiles carry enough work to hide their loads and stores.
  for (int k0 = 0; k0 < Nmax; k0 += CHOL_PANEL) {
    int nact = b.count;
    bool rows_below = true;
    for (int h = 0; h < CHOL_PANEL / TB; ++h) {
      const int kh = k0 + h * TB;
      nact = count_above(nact, kh);   // problems with a diagonal block at kh
      if (nact == 0) { rows_below = false; break; }
      if (h > 0) BSE_TRY(gemm_batched(s, b, nact, POPS, k0 + h));
      BSE_LAUNCH(k_potf2, dim3(1, 1, (unsigned)nact), TB, 0, s, b.dev, sel, kh);
      nact = count_above(nact, kh + TB);   // problems with rows below it
      if (nact == 0) { rows_below = false; break; }
      BSE_TRY(trsm_rows_batched(s, b, nact, sel, kh));
    }
    if (!rows_below) break;
    const int nrest = count_above(nact, k0 + CHOL_PANEL);
    if (nrest > 0) BSE_TRY(gemm_batched(s, b, nrest, SOPS, k0));
  }
  return 0;
}

int form_W_batched(hipStream_t s, const Batch& b, bool full) {
  if (b.count <= 0) return 0;
  const long n = b.maxn(), N = b.maxN();
  // C = L11^T L21 into W11, then W11 = C - C^T
  BSE_TRY(gemm_batched(s, b, b.count, GOP_FORMW_C, 0));
  const long nt = (n + TB - 1) / TB;
  BSE_LAUNCH(k_skew_pairs, dim3((unsigned)(nt * (nt + 1) / 2), 1, (unsigned)b.count), 256, 0, s, b.dev, 0, full ? 1 : 0);
  // W21 = -L22^T L11
  BSE_TRY(gemm_batched(s, b, b.count, GOP_FORMW_21, 0));
  BSE_LAUNCH(k_zero_W22, grid2d(n, n, b.count), 256, 0, s, b.dev);
  if (full) {
    const long Nt = (N + TB - 1) / TB;
    BSE_LAUNCH(k_skew_pairs, dim3((unsigned)(Nt * (Nt + 1) / 2), 1, (unsigned)b.count), 256, 0, s, b.dev, 1, 1);
  }
  return 0;
}

}  // namespace bse
