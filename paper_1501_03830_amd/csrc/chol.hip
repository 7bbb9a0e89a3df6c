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

__global__ __launch_bounds__(256) void k_build_M(int n, const double* __restrict__ A, long lda,
                                                 const double* __restrict__ B, long ldb,
                                                 double* __restrict__ M, long ldm) {
  const int N = 2 * n;
  const int r = blockIdx.x * TB + (threadIdx.x & 63);
  const int cbase = blockIdx.y * TB + (threadIdx.x >> 6) * 16;
  if (r >= N) return;
  for (int q = 0; q < 16; ++q) {
    const int c = cbase + q;
    if (c >= N) break;
    double val = 0.0;
    if (r >= c) {
      const int bi = r >= n, bj = c >= n;
      const int i = r - bi * n, j = c - bj * n;
      double ar, ai, br, bim;
      if (i >= j) {
        const long ia = 2 * ((long)i + (long)j * lda), ib = 2 * ((long)i + (long)j * ldb);
        ar = A[ia];
        ai = A[ia + 1];
        br = B[ib];
        bim = B[ib + 1];
      } else {  // upper triangle: A[i,j] = conj(A[j,i]), B[i,j] = B[j,i]
        const long ia = 2 * ((long)j + (long)i * lda), ib = 2 * ((long)j + (long)i * ldb);
        ar = A[ia];
        ai = -A[ia + 1];
        br = B[ib];
        bim = B[ib + 1];
      }
      if (i == j) ai = 0.0;  // a Hermitian diagonal is real
      if (!bi && !bj) val = ar + br;          // Re(A+B)
      else if (bi && !bj) val = -(ai + bim);  // -Im(A+B)
      else val = ar - br;                     // Re(A-B)
    }
    M[(long)r + (long)c * ldm] = val;
  }
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Unblocked Cholesky of the nb x nb diagonal block at (k0, k0), in LDS.
__global__ __launch_bounds__(256) void k_potf2(double* __restrict__ M, long ld, int N, int k0,
                                               int* __restrict__ info) {
  __shared__ double a[TB][TB + 1];  // a[col][row]
  if (*info != 0) return;
  const int nbk = min(TB, N - k0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < TB * TB; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    a[c][r] = (r < nbk && c < nbk && r >= c) ? M[(long)(k0 + r) + (long)(k0 + c) * ld] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nbk; ++j) {
    const double piv = a[j][j];
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (tid == 0) *info = k0 + j + 1;
      return;  // uniform: every thread read the same pivot
    }
    const double ljj = sqrt(piv);
    __syncthreads();
    for (int r = j + 1 + tid; r < nbk; r += 256) a[j][r] /= ljj;
    if (tid == 0) a[j][j] = ljj;
    __syncthreads();
    const int nc = nbk - j - 1;
    for (int idx = tid; idx < nc * nc; idx += 256) {
      const int r = j + 1 + idx % nc, c = j + 1 + idx / nc;
      if (r >= c) a[c][r] -= a[j][r] * a[j][c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < TB * TB; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    if (r < nbk && c < nbk && r >= c) M[(long)(k0 + r) + (long)(k0 + c) * ld] = a[c][r];
  }
}

// Inverse of the lower-triangular nbk x nbk diagonal block at (b0, b0) into
// Linv (64 x 64, ld 64): thread c solves L y = e_c by forward substitution,
// with y kept in LDS.
__global__ __launch_bounds__(64) void k_trtri64(const double* __restrict__ L, long ld, int b0, int nbk,
                                                double* __restrict__ Linv, const int* __restrict__ info) {
  __shared__ double Lc[TB][TB + 1];  // Lc[col][row]
  __shared__ double Y[TB][TB + 1];   // Y[col][row]
  if (*info != 0) return;
  const int c = threadIdx.x;
  for (int r = 0; r < TB; ++r)
    Lc[c][r] = (r < nbk && c < nbk && r >= c) ? L[(long)(b0 + r) + (long)(b0 + c) * ld] : 0.0;
  __syncthreads();
  for (int r = 0; r < TB; ++r) {
    double y = 0.0;
    if (c < nbk && r < nbk && r >= c) {
      double acc = (r == c) ? 1.0 : 0.0;
      for (int l = c; l < r; ++l) acc -= Lc[l][r] * Y[c][l];
      y = acc / Lc[r][r];
    }
    Y[c][r] = y;
  }
  for (int r = 0; r < TB; ++r) Linv[r + (long)c * TB] = Y[c][r];
}

// For every lower tile pair (R, C), R >= C, of an nrows x nrows matrix:
//  mode 0: lower <- T1 - T2^T  (T1 = tile (R,C), T2 = tile (C,R)); diagonal 0;
//          with `full` the upper triangle receives the negated transpose.
//  mode 1: upper <- -lower^T (completion of a skew matrix from its lower part)
__global__ __launch_bounds__(256) void k_skew_pairs(double* __restrict__ W, long ld, int nrows,
                                                    int mode, int full) {
  __shared__ double t1[TB][TB + 1];
  __shared__ double t2[TB][TB + 1];
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

__global__ __launch_bounds__(256) void k_fill(int m, int n, double* __restrict__ dst, long ldd,
                                              double v, int upper_only) {
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= m) return;
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    if (c >= n) break;
    if (upper_only && r >= c) continue;
    dst[r + c * ldd] = v;
  }
}

dim3 grid2d(long m, long n) { return dim3((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64)); }

}  // namespace

int launch_build_M(hipStream_t s, int n, const double* A, long lda, const double* B, long ldb,
                   double* M, long ldm) {
  const long N = 2L * n;
  k_build_M<<<grid2d(N, N), 256, 0, s>>>(n, A, lda, B, ldb, M, ldm);
  BSE_LAUNCHED();
  return 0;
}

int copy_matrix(hipStream_t s, int m, int n, const double* src, long lds, double* dst, long ldd) {
  if (m <= 0 || n <= 0) return 0;
  k_copy<<<grid2d(m, n), 256, 0, s>>>(m, n, src, lds, dst, ldd);
  BSE_LAUNCHED();
  return 0;
}

int zero_upper(hipStream_t s, int N, double* A, long lda) {
  if (N <= 0) return 0;
  k_fill<<<grid2d(N, N), 256, 0, s>>>(N, N, A, lda, 0.0, 1);
  BSE_LAUNCHED();
  return 0;
}

int trtri_diag64(hipStream_t s, const double* L, long ld, int b0, int nbk, double* Linv, const int* info_dev) {
  k_trtri64<<<1, 64, 0, s>>>(L, ld, b0, nbk, Linv, info_dev);
  BSE_LAUNCHED();
  return 0;
}

int potrf_f64(hipStream_t s, int N, double* M, long ld, int* info_dev, double* linv, bool reset_info) {
  if (reset_info) {
    k_set_int<<<1, 64, 0, s>>>(info_dev, 0);
    BSE_LAUNCHED();
  }
  for (int k0 = 0; k0 < N; k0 += TB) {
    const int nbk = (N - k0 < TB) ? N - k0 : TB;
    k_potf2<<<1, 256, 0, s>>>(M, ld, N, k0, info_dev);
    BSE_LAUNCHED();
    const int rest = N - k0 - nbk;
    if (rest > 0) {
      double* a21 = M + (k0 + nbk) + (long)k0 * ld;
      // A21 <- A21 L_kk^{-T}; in place is safe: one column tile of output
      k_trtri64<<<1, 64, 0, s>>>(M, ld, k0, nbk, linv, info_dev);
      BSE_LAUNCHED();
      BSE_TRY(gemm_f64(s, false, true, rest, nbk, nbk, 1.0, a21, ld, linv, TB, 0.0, a21, ld, 0, 0, 0));
      double* a22 = M + (k0 + nbk) + (long)(k0 + nbk) * ld;
      BSE_TRY(gemm_f64(s, false, true, rest, rest, nbk, -1.0, a21, ld, a21, ld, 1.0, a22, ld, 1, 0, 0));
    }
  }
  return 0;
}

int form_W(hipStream_t s, int N, const double* L, long ldl, double* W, long ldw, bool full) {
  const int n = N / 2;
  const double* L11 = L;
  const double* L21 = L + n;
  const double* L22 = L + n + (long)n * ldl;
  // C = L11^T L21 into W11, then W11 = C - C^T
  BSE_TRY(gemm_f64(s, true, false, n, n, n, 1.0, L11, ldl, L21, ldl, 0.0, W, ldw, 0, 1, 0));
  const long nt = (n + TB - 1) / TB;
  k_skew_pairs<<<(unsigned)(nt * (nt + 1) / 2), 256, 0, s>>>(W, ldw, n, 0, full ? 1 : 0);
  BSE_LAUNCHED();
  // W21 = -L22^T L11
  BSE_TRY(gemm_f64(s, true, false, n, n, n, -1.0, L22, ldl, L11, ldl, 0.0, W + n, ldw, 0, 1, 1));
  // W22 = 0
  k_fill<<<grid2d(n, n), 256, 0, s>>>(n, n, W + n + (long)n * ldw, ldw, 0.0, 0);
  BSE_LAUNCHED();
  if (full) {
    const long Nt = (N + TB - 1) / TB;
    k_skew_pairs<<<(unsigned)(Nt * (Nt + 1) / 2), 256, 0, s>>>(W, ldw, N, 1, 1);
    BSE_LAUNCHED();
  }
  return 0;
}

}  // namespace bse
