// Back-transformation to the eigenvectors of H (Algorithm 1 step 5 as
// organised by Algorithm 3 steps 3-6, remarks 3 and 4).
//
//   x_j = S Q L U D v_j / sqrt(lambda_j)
//
// evaluated right to left:
//   * D v_j (D = diag(i^k)) is a real vector in its even rows (real part,
//     sign (-1)^(k/2)) and in its odd rows (imaginary part, sign
//     (-1)^((k-1)/2)); the real and imaginary parts of all n vectors are kept
//     side by side as one real N x N matrix Z = [Re | Im], so that U and L
//     are applied with real products only (remark 4's real/imaginary split).
//   * U = H_0 ... H_{N-3} is applied from the left in blocks of reflectors,
//     last block first, each block as I - V T V^T (compact WY, T from the
//     forward column-wise recurrence of LAPACK's larft).
//   * L is applied by a triangular MFMA product.
//   * Q = (1/sqrt 2)[I -iI; I iI] and S = diag(I, -I) only combine rows, so
//     they are folded with the 1/sqrt(lambda) scaling into the kernel that
//     writes the interleaved complex output (remark 3: O(n^2) work).
#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

__global__ __launch_bounds__(256) void k_scatter_DV(int N, const double* __restrict__ Vt, double* __restrict__ Z,
                                                    long ldz) {
  __shared__ double t[64][65];
  const int n = N / 2;
  const int k0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int jj = idx & 63, kk = idx >> 6;
    const int j = j0 + jj, k = k0 + kk;
    t[kk][jj] = (j < n && k < N) ? Vt[(long)j + (long)k * n] : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int kk = idx & 63, jj = idx >> 6;
    const int j = j0 + jj, k = k0 + kk;
    if (j >= n || k >= N) continue;
    const double v = t[kk][jj];
    const double sgn = ((k >> 1) & 1) ? -1.0 : 1.0;
    const bool even = (k & 1) == 0;
    Z[(long)k + (long)j * ldz] = even ? sgn * v : 0.0;
    Z[(long)k + (long)(n + j) * ldz] = even ? 0.0 : sgn * v;
  }
}

// Explicit reflector block: Vb[r, l] for rows r in [j0+1, N):
//   0 above row j0+l+1, 1 at row j0+l+1, W[r, j0+l] below.
__global__ __launch_bounds__(256) void k_extract_V(const double* __restrict__ W, long ldw, int N, int j0,
                                                   int nbk, double* __restrict__ Vb, long ldv) {
  const long r = (long)j0 + 1 + (long)blockIdx.x * 64 + (threadIdx.x & 63);
  if (r >= N) return;
  for (int l = threadIdx.x >> 6; l < nbk; l += 4) {
    const long diag = (long)j0 + l + 1;
    double v;
    if (r < diag) v = 0.0;
    else if (r == diag) v = 1.0;
    else v = W[r + (long)(j0 + l) * ldw];
    Vb[r + (long)l * ldv] = v;
  }
}

// T (upper, nbk x nbk, ld nbq) with H_{j0} ... H_{j0+nbk-1} = I - V T V^T,
// from S = V^T V:  T[l,l] = tau_l,  T[0:l, l] = -tau_l T[0:l,0:l] S[0:l, l].
__global__ __launch_bounds__(64) void k_larft(const double* __restrict__ S, int nbq, int nbk,
                                              const double* __restrict__ tau, int j0, double* __restrict__ T) {
  __shared__ double Ts[64][65];   // Ts[col][row]
  __shared__ double u[64];
  const int i = threadIdx.x;
  for (int c = 0; c < 64; ++c) Ts[c][i] = 0.0;
  __syncthreads();
  for (int l = 0; l < nbk; ++l) {
    const double tl = tau[j0 + l];
    if (i < l) u[i] = -tl * S[i + (long)l * nbq];
    __syncthreads();
    if (i < l) {
      double acc = 0.0;
      for (int m = i; m < l; ++m) acc += Ts[m][i] * u[m];
      Ts[l][i] = acc;
    }
    if (i == l) Ts[l][l] = tl;
    __syncthreads();
  }
  for (int c = 0; c < nbk; ++c)
    if (i < nbk) T[i + (long)c * nbq] = Ts[c][i];
}

__global__ __launch_bounds__(256) void k_finish_X(int n, const double* __restrict__ G, long ldg,
                                                  const double* __restrict__ lam, double* __restrict__ X,
                                                  long ldx) {
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= n) return;
  for (int q = 0; q < 16; ++q) {
    const long j = c0 + q;
    if (j >= n) break;
    const double g1r = G[r + j * ldg], g1i = G[r + (n + j) * ldg];
    const double g2r = G[n + r + j * ldg], g2i = G[n + r + (n + j) * ldg];
    const double c = 1.0 / sqrt(2.0 * lam[j]);
    double* x1 = X + 2 * (r + j * ldx);
    double* x2 = X + 2 * (n + r + j * ldx);
    x1[0] = (g1r + g2i) * c;
    x1[1] = (g1i - g2r) * c;
    x2[0] = (g2i - g1r) * c;
    x2[1] = -(g1i + g2r) * c;
  }
}

// One workgroup per column: canonical phase (largest modulus, lowest index on
// ties, made real positive), then the weights of eq. absp with y = S x.
__global__ __launch_bounds__(256) void k_phase_weights(int n, double* __restrict__ X, long ldx,
                                                       const double* __restrict__ dr,
                                                       const double* __restrict__ dl, double* __restrict__ w) {
  __shared__ double sval[4];
  __shared__ int sidx[4];
  __shared__ double red[4];
  __shared__ double ph[2];
  const int j = blockIdx.x;
  const int N = 2 * n;
  double* x = X + 2 * (long)j * ldx;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int r = threadIdx.x; r < N; r += 256) {
    const double m = hypot(x[2 * r], x[2 * r + 1]);
    if (m > best) {
      best = m;
      bi = r;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sval[wv] = best;
    sidx[wv] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sval[0];
    int ix = sidx[0];
    for (int k = 1; k < 4; ++k)
      if (sval[k] > b || (sval[k] == b && sidx[k] < ix)) {
        b = sval[k];
        ix = sidx[k];
      }
    const double pr = x[2 * ix], pi = x[2 * ix + 1];
    const double m = hypot(pr, pi);
    ph[0] = (m > 0.0) ? pr / m : 1.0;
    ph[1] = (m > 0.0) ? -pi / m : 0.0;
  }
  __syncthreads();
  const double cr = ph[0], ci = ph[1];
  double ar = 0.0, ai = 0.0, br = 0.0, bim = 0.0, den = 0.0;
  for (int r = threadIdx.x; r < N; r += 256) {
    const double xr0 = x[2 * r], xi0 = x[2 * r + 1];
    const double xr = xr0 * cr - xi0 * ci;
    const double xi = xr0 * ci + xi0 * cr;
    x[2 * r] = xr;
    x[2 * r + 1] = xi;
    if (dr != nullptr) {
      const double sg = (r < n) ? 1.0 : -1.0;
      // conj(dr) * x
      const double drr = dr[2 * r], dri = dr[2 * r + 1];
      ar += drr * xr + dri * xi;
      ai += drr * xi - dri * xr;
      // conj(y) * dl with y = S x
      const double dlr = dl[2 * r], dli = dl[2 * r + 1];
      br += sg * (xr * dlr + xi * dli);
      bim += sg * (xr * dli - xi * dlr);
      den += sg * (xr * xr + xi * xi);
    }
  }
  if (dr == nullptr) return;
  ar = block_sum(ar, red);
  ai = block_sum(ai, red);
  br = block_sum(br, red);
  bim = block_sum(bim, red);
  den = block_sum(den, red);
  if (threadIdx.x == 0) {
    const double nr = ar * br - ai * bim, ni = ar * bim + ai * br;
    w[2 * j] = nr / den;
    w[2 * j + 1] = ni / den;
  }
}

}  // namespace

size_t backtr_work_bytes(long N, long ld, int nbq) {
  (void)N;
  return ((size_t)ld * nbq + 2 * (size_t)nbq * nbq + 2 * (size_t)nbq * ld) * sizeof(double) + 5 * 256;
}

int backtr_bind_work(void* base, long N, long ld, int nbq, BacktrWork* w) {
  (void)N;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += round_up((long)bytes, 256);
    return q;
  };
  w->Vb = reinterpret_cast<double*>(take((size_t)ld * nbq * sizeof(double)));
  w->S = reinterpret_cast<double*>(take((size_t)nbq * nbq * sizeof(double)));
  w->T = reinterpret_cast<double*>(take((size_t)nbq * nbq * sizeof(double)));
  w->W1 = reinterpret_cast<double*>(take((size_t)nbq * ld * sizeof(double)));
  w->W2 = reinterpret_cast<double*>(take((size_t)nbq * ld * sizeof(double)));
  w->nbq = nbq;
  return 0;
}

int scatter_DV(hipStream_t s, int N, const double* Vt, double* Z, long ldz) {
  const int n = N / 2;
  dim3 g((unsigned)((N + 63) / 64), (unsigned)((n + 63) / 64));
  k_scatter_DV<<<g, 256, 0, s>>>(N, Vt, Z, ldz);
  BSE_LAUNCHED();
  return 0;
}

int apply_U(hipStream_t s, int N, const double* W, long ldw, const double* tau, double* Z, long ldz,
            int ncols, const BacktrWork& w) {
  const int nrefl = N - 2;  // H_0 .. H_{N-3}; H_{N-2} is the identity
  if (nrefl <= 0) return 0;
  const int nbq = w.nbq;
  const int nblocks = (nrefl + nbq - 1) / nbq;
  for (int q = nblocks - 1; q >= 0; --q) {
    const int j0 = q * nbq;
    const int nbk = (nrefl - j0 < nbq) ? nrefl - j0 : nbq;
    const int m = N - j0 - 1;
    double* Vb = w.Vb + (j0 + 1);
    double* Zs = Z + (j0 + 1);
    k_extract_V<<<(unsigned)((m + 63) / 64), 256, 0, s>>>(W, ldw, N, j0, nbk, w.Vb, ldw);
    BSE_LAUNCHED();
    BSE_TRY(gemm_f64(s, true, false, nbk, nbk, m, 1.0, Vb, ldw, Vb, ldw, 0.0, w.S, nbq, 0, 0, 0));
    k_larft<<<1, 64, 0, s>>>(w.S, nbq, nbk, tau, j0, w.T);
    BSE_LAUNCHED();
    BSE_TRY(gemm_f64(s, true, false, nbk, ncols, m, 1.0, Vb, ldw, Zs, ldz, 0.0, w.W1, nbq, 0, 0, 0));
    BSE_TRY(gemm_f64(s, false, false, nbk, ncols, nbk, 1.0, w.T, nbq, w.W1, nbq, 0.0, w.W2, nbq, 0, 0, 0));
    BSE_TRY(gemm_f64(s, false, false, m, ncols, nbk, -1.0, Vb, ldw, w.W2, nbq, 1.0, Zs, ldz, 0, 0, 0));
  }
  return 0;
}

int finish_X(hipStream_t s, int n, const double* G, long ldg, const double* lam, double* X, long ldx) {
  dim3 g((unsigned)((n + 63) / 64), (unsigned)((n + 63) / 64));
  k_finish_X<<<g, 256, 0, s>>>(n, G, ldg, lam, X, ldx);
  BSE_LAUNCHED();
  return 0;
}

int phase_and_weights(hipStream_t s, int n, double* X, long ldx, const double* dr, const double* dl,
                      double* w) {
  k_phase_weights<<<(unsigned)n, 256, 0, s>>>(n, X, ldx, dr, dl, w);
  BSE_LAUNCHED();
  return 0;
}

}  // namespace bse
