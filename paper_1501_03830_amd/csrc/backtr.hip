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
//   * U = H_0 ... H_{N-3} is applied from the left in blocks of 256
//     reflectors, last block first, each block as I - V T V^T (compact WY);
//     T is applied by a triangular solve with its inverse
//     diag(1/tau) + strict_upper(V^T V) (trsm.hip), never formed.
//   * L is applied by a triangular MFMA product.
//   * Q = (1/sqrt 2)[I -iI; I iI] and S = diag(I, -I) only combine rows, so
//     they are folded with the 1/sqrt(lambda) scaling into the kernel that
//     writes the interleaved complex output (remark 3: O(n^2) work).
#include <vector>

#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int NBQ = APPLYU_RB;  // reflectors per block

__global__ __launch_bounds__(256) void k_scatter_DV(const Prob* __restrict__ probs) {
  __shared__ double t[64][65];
  const Prob& P = probs[blockIdx.z];
  const int N = P.N, n = P.n;
  const int k0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (k0 >= N || j0 >= n) return;  // uniform
  const BSE_GLOBAL double* __restrict__ Vt = gbl(P.Vt);
  BSE_GLOBAL double* __restrict__ Z = gbl(P.Z);
  // the mixed-precision path keeps this basis in FP32 until the refinement
  const bool f32 = P.prec == BSE_PREC_FP32_REFINE;
  BSE_GLOBAL float* __restrict__ Z32 = gbl(P.Z32);
  const long ldz = P.ld;
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
    const double re = even ? sgn * v : 0.0, im = even ? 0.0 : sgn * v;
    if (f32) {
      Z32[(long)k + (long)j * ldz] = (float)re;
      Z32[(long)k + (long)(n + j) * ldz] = (float)im;
    } else {
      Z[(long)k + (long)j * ldz] = re;
      Z[(long)k + (long)(n + j) * ldz] = im;
    }
  }
}

// Explicit reflector block q: Vb[r, l] for rows r in [j0+o, N), j0 = 256 q,
// o = refl_off(P) (1 after the one-stage reduction, the band width after the
// two-stage one, whose first stage stores reflector k below the band):
//   0 above row j0+l+o, 1 at row j0+l+o, W[r, j0+l] below (and its FP32 copy
//   Vb32 in the mixed-precision path, whose products with the FP32 basis run
//   on the FP32 matrix cores).
__global__ __launch_bounds__(256) void k_extract_V(const Prob* __restrict__ probs, int q) {
  const Prob& P = probs[blockIdx.z];
  const int N = P.N;
  const int o = refl_off(P);
  const int nrefl = N - 1 - o;
  const int j0 = q * NBQ;
  if (j0 >= nrefl) return;  // uniform
  const int nbk = min(NBQ, nrefl - j0);
  const BSE_GLOBAL double* __restrict__ W = gbl(P.W);
  const BSE_GLOBAL float* __restrict__ W32 = gbl(P.W32);
  const bool f32 = P.prec == BSE_PREC_FP32_REFINE;   // reflectors stored in FP32
  BSE_GLOBAL double* __restrict__ Vb = gbl(P.Vb);
  BSE_GLOBAL float* __restrict__ Vb32 = gbl(P.Vb32);
  const long ldw = P.ld, ldv = P.ld;
  const long r = (long)j0 + o + (long)blockIdx.x * 64 + (threadIdx.x & 63);
  if (r >= N) return;
  for (int l = threadIdx.x >> 6; l < nbk; l += 4) {
    const long diag = (long)j0 + l + o;
    double v;
    if (r < diag) v = 0.0;
    else if (r == diag) v = 1.0;
    else v = f32 ? (double)W32[r + (long)(j0 + l) * ldw] : W[r + (long)(j0 + l) * ldw];
    Vb[r + (long)l * ldv] = v;
    if (f32) Vb32[r + (long)l * ldv] = (float)v;
  }
}

// X = S Q G Lambda^{-1/2} from G = L U D V_+ = [Re | Im] held in P.W
__global__ __launch_bounds__(256) void k_finish_X(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  const int n = P.n;
  const BSE_GLOBAL double* __restrict__ G = gbl(P.W);
  const long ldg = P.ld;
  const BSE_GLOBAL double* __restrict__ lam = gbl(P.lambda);
  const BSE_GLOBAL int* __restrict__ perm = gbl(P.perm);   // null: identity order
  BSE_GLOBAL double* __restrict__ X = gbl(P.X);
  const long ldx = P.ldx;
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= n) return;
  for (int q = 0; q < 16; ++q) {
    const long j = c0 + q;
    if (j >= n) break;
    const long js = perm ? (long)perm[j] : j;   // eigenpair written to column j
    const double g1r = G[r + js * ldg], g1i = G[r + (n + js) * ldg];
    const double g2r = G[n + r + js * ldg], g2i = G[n + r + (n + js) * ldg];
    const double c = 1.0 / sqrt(2.0 * lam[j]);
    auto x1 = X + 2 * (r + j * ldx);
    auto x2 = X + 2 * (n + r + j * ldx);
    x1[0] = (g1r + g2i) * c;
    x1[1] = (g1i - g2r) * c;
    x2[0] = (g2i - g1r) * c;
    x2[1] = -(g1i + g2r) * c;
  }
}

// One workgroup per column: canonical phase (largest modulus, lowest index on
// ties, made real positive), then the weights of eq. absp with y = S x.
__global__ __launch_bounds__(256) void k_phase_weights(const Prob* __restrict__ probs) {
  __shared__ double sval[4];
  __shared__ int sidx[4];
  __shared__ double red[4];
  __shared__ double ph[2];
  const Prob& P = probs[blockIdx.z];
  const int n = P.n;
  const int j = blockIdx.x;
  if (j >= n) return;  // uniform
  const long ldx = P.ldx;
  BSE_GLOBAL double* __restrict__ X = gbl(P.X);
  const bool weights = (P.flags & BSE_WANT_WEIGHTS) != 0 && P.dr != nullptr && P.w != nullptr;
  const BSE_GLOBAL double* __restrict__ dr = gbl(weights ? P.dr : nullptr);
  const BSE_GLOBAL double* __restrict__ dl = gbl(weights ? (P.dl ? P.dl : P.dr) : nullptr);
  BSE_GLOBAL double* __restrict__ w = gbl(P.w);
  const int N = 2 * n;
  auto x = X + 2 * (long)j * ldx;
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
    if (ix < 0 || ix >= N) ix = 0;  // no finite maximum (NaN input): keep index 0
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

// Real problems (FLAG_REAL_IN, eq. H-real).  The eigenvectors of a real H
// are real up to a phase, so after the canonical phase every column is real
// to rounding, except inside a group of equal eigenvalues whose computed
// basis is a complex combination of real eigenvectors.  k_real_flags marks
// the columns whose imaginary part exceeds 1e-8 of their norm.
__global__ __launch_bounds__(256) void k_real_flags(const Prob* __restrict__ probs) {
  __shared__ double red[4];
  const Prob& P = probs[blockIdx.z];
  const int n = P.n, N = P.N;
  const int j = blockIdx.x;
  if (j >= n) return;   // uniform
  const BSE_GLOBAL double* __restrict__ x = gbl(P.X) + 2 * (long)j * P.ldx;
  double im = 0.0, tot = 0.0;
  for (int r = threadIdx.x; r < N; r += 256) {
    const double a = x[2 * r], b = x[2 * r + 1];
    im += b * b;
    tot += a * a + b * b;
  }
  im = block_sum(im, red);
  tot = block_sum(tot, red);
  if (threadIdx.x == 0) gbl(P.cid)[j] = (im > 1e-16 * tot) ? 1 : 0;
}

// One workgroup per group of equal eigenvalues (first column g0, c columns):
// the real and imaginary parts of its columns span its real eigenspace.
// Modified Gram-Schmidt, twice, in the inner product <p, q> = p1^T q1 -
// p2^T q2 of Theorem 3's normalisation (positive on the eigenvectors of the
// positive eigenvalues) over the candidates Re x_g0, Im x_g0, Re x_g0+1, ...
// keeps each candidate with at least half its norm left, until c are kept;
// they replace the group's columns with zero imaginary parts.  Work space:
// the same columns of P.W (free once X is written).
__global__ __launch_bounds__(256) void k_realify(const Prob* __restrict__ probs, const int* __restrict__ groups,
                                                 int ngroups) {
  __shared__ double red[4];
  const Prob& P = probs[0];
  const int g = blockIdx.x;
  if (g >= ngroups) return;
  const int g0 = groups[2 * g], c = groups[2 * g + 1];
  const long N = P.N, n = P.n, ld = P.ld, ldx = P.ldx;
  BSE_GLOBAL double* __restrict__ X = gbl(P.X);
  BSE_GLOBAL double* __restrict__ T = gbl(P.W);
  int kept = 0;
  for (int cand = 0; cand < 2 * c && kept < c; ++cand) {
    const long col = g0 + cand / 2;
    const int part = cand & 1;
    BSE_GLOBAL double* t = T + (long)(g0 + kept) * ld;
    double nn = 0.0;
    for (long r = threadIdx.x; r < N; r += 256) {
      const double v = X[2 * (r + col * ldx) + part];
      t[r] = v;
      nn += (r < n ? 1.0 : -1.0) * v * v;
    }
    const double orig = block_sum(nn, red);
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < kept; ++q) {
        const BSE_GLOBAL double* u = T + (long)(g0 + q) * ld;
        double d = 0.0;
        for (long r = threadIdx.x; r < N; r += 256) d += (r < n ? 1.0 : -1.0) * u[r] * t[r];
        d = block_sum(d, red);
        for (long r = threadIdx.x; r < N; r += 256) t[r] -= d * u[r];
        __syncthreads();
      }
    }
    nn = 0.0;
    for (long r = threadIdx.x; r < N; r += 256) nn += (r < n ? 1.0 : -1.0) * t[r] * t[r];
    const double res = block_sum(nn, red);
    if (orig > 0.0 && res > 0.0 && res >= 0.25 * orig) {
      const double f = 1.0 / sqrt(res);
      for (long r = threadIdx.x; r < N; r += 256) t[r] *= f;
      __syncthreads();
      ++kept;
    }
  }
  if (kept < c) {
    if (threadIdx.x == 0) gbl(P.info)[1] = 1;   // no real basis found
    return;
  }
  for (int q = 0; q < c; ++q) {
    const BSE_GLOBAL double* u = T + (long)(g0 + q) * ld;
    for (long r = threadIdx.x; r < N; r += 256) {
      X[2 * (r + (long)(g0 + q) * ldx)] = u[r];
      X[2 * (r + (long)(g0 + q) * ldx) + 1] = 0.0;
    }
  }
}

// the real parts of X into the caller's real 2n x n output
__global__ __launch_bounds__(256) void k_real_copy(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  const long N = P.N, n = P.n;
  const long r = (long)blockIdx.x * 256 + threadIdx.x;
  const long j = blockIdx.y;
  if (r >= N || j >= n) return;
  gbl(P.Xr)[r + j * P.ldxr] = gbl(P.X)[2 * (r + j * P.ldx)];
}

// strictly lower triangle of W into its FP32 copy (the part the reduction
// reads)
__global__ __launch_bounds__(256) void k_to_f32(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  const long N = P.N;
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= N) return;
  const BSE_GLOBAL double* __restrict__ W = gbl(P.W);
  BSE_GLOBAL float* __restrict__ W32 = gbl(P.W32);
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    if (c >= N || c >= r) break;
    W32[r + c * P.ld] = (float)W[r + c * P.ld];
  }
}

}  // namespace

int to_f32_batched(hipStream_t s, const Batch& b) {
  if (b.count <= 0) return 0;
  const long N0 = b.maxN();
  BSE_LAUNCH(k_to_f32, dim3((unsigned)((N0 + 63) / 64), (unsigned)((N0 + 63) / 64), (unsigned)b.count), 256, 0, s, b.dev);
  return 0;
}

size_t backtr_work_bytes(long N, long ld) {
  (void)N;
  return ((size_t)ld * NBQ + (size_t)NBQ * NBQ + 2 * (size_t)NBQ * ld) * sizeof(double) +
         2 * (size_t)NBQ * ld * sizeof(float) + 6 * 256;
}

void backtr_bind_work(char* base, long N, long ld, Prob* P) {
  (void)N;
  char* p = base;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += round_up((long)bytes, 256);
    return q;
  };
  P->Vb = reinterpret_cast<double*>(take((size_t)ld * NBQ * sizeof(double)));
  P->S = reinterpret_cast<double*>(take((size_t)NBQ * NBQ * sizeof(double)));
  P->W1 = reinterpret_cast<double*>(take((size_t)NBQ * ld * sizeof(double)));
  P->W2 = reinterpret_cast<double*>(take((size_t)NBQ * ld * sizeof(double)));
  P->Vb32 = reinterpret_cast<float*>(take((size_t)ld * NBQ * sizeof(float)));
  P->W2f = reinterpret_cast<float*>(take((size_t)NBQ * ld * sizeof(float)));
}

int apply_UD_batched(hipStream_t s, const Batch& b) {
  if (b.count <= 0) return 0;
  const int N0 = b.maxN(), n0 = b.maxn();
  // Z = [Re(D V_+) | Im(D V_+)]
  BSE_LAUNCH(k_scatter_DV, dim3((unsigned)((N0 + 63) / 64), (unsigned)((n0 + 63) / 64), (unsigned)b.count), 256, 0, s, b.dev);
  // after the two-stage reduction (a batch of one): Z <- Q2 Z for the
  // chase's reflectors, then the band reduction's below as U
  const int o = refl_off(b.host[0]);
  if (o > 1) BSE_TRY(sbr_q2_apply(s, b));
  // Z <- U Z with U = H_0 ... H_{N-2-o}, last block of reflectors first (the
  // one-stage H_{N-2} is the identity)
  const int nrefl0 = N0 - 1 - o;
  if (nrefl0 <= 0) return 0;
  const int nblocks0 = (nrefl0 + NBQ - 1) / NBQ;
  for (int q = nblocks0 - 1; q >= 0; --q) {
    const int j0 = q * NBQ;
    const int nact = b.active_N_above(j0 + 1 + o);   // N - 1 - o > j0
    const int m0 = N0 - j0 - o;
    BSE_LAUNCH(k_extract_V, dim3((unsigned)((m0 + 63) / 64), 1, (unsigned)nact), 256, 0, s, b.dev, q);
    BSE_TRY(gemm_batched(s, b, nact, GOP_APPLYU_S, q));
    BSE_TRY(gemm_batched(s, b, nact, GOP_APPLYU_W1, q));
    for (int h = NBQ / 64 - 1; h >= 0; --h) {
      if (h < NBQ / 64 - 1) BSE_TRY(gemm_batched(s, b, nact, GOP_APPLYU_WB, APPLYU_SUB * q + h));
      BSE_TRY(wy_solve_batched(s, b, nact, q, h));
    }
    BSE_TRY(gemm_batched(s, b, nact, GOP_APPLYU_Z, q));
  }
  return 0;
}

int real_output_single(hipStream_t s, const Batch& b) {
  if (b.count != 1) return set_error(BSE_EUNSUPPORTED, "real problems are solved one at a time");
  const Prob& P = b.host[0];
  const int n = P.n, N = P.N;
  BSE_LAUNCH(k_real_flags, dim3((unsigned)n, 1, 1), 256, 0, s, b.dev);
  std::vector<int> flag(n);
  std::vector<double> lam(n);
  BSE_HIP(hipMemcpyAsync(flag.data(), P.cid, n * sizeof(int), hipMemcpyDeviceToHost, s));
  BSE_HIP(hipMemcpyAsync(lam.data(), P.lambda, n * sizeof(double), hipMemcpyDeviceToHost, s));
  BSE_HIP(hipStreamSynchronize(s));
  // groups: runs of eigenvalues closer than 1e-8 lambda_max (consecutive)
  // that hold a flagged column
  std::vector<int> groups;
  const double tol = 1e-8 * (n > 0 ? lam[n - 1] : 0.0);
  for (int j = 0; j < n;) {
    int e = j + 1;
    while (e < n && lam[e] - lam[e - 1] <= tol) ++e;
    bool any = false;
    for (int k = j; k < e; ++k) any = any || flag[k] != 0;
    if (any) {
      groups.push_back(j);
      groups.push_back(e - j);
    }
    j = e;
  }
  if (!groups.empty()) {
    // the group list goes to the inverse-iteration factors' space (free here)
    int* dgroups = reinterpret_cast<int*>(P.inv);
    BSE_HIP(hipMemcpyAsync(dgroups, groups.data(), groups.size() * sizeof(int), hipMemcpyHostToDevice, s));
    const int ng = (int)groups.size() / 2;
    BSE_LAUNCH(k_realify, dim3((unsigned)ng), 256, 0, s, b.dev, dgroups, ng);
    // canonical sign and the weights of the new columns
    BSE_LAUNCH(k_phase_weights, dim3((unsigned)n, 1, 1), 256, 0, s, b.dev);
    BSE_HIP(hipStreamSynchronize(s));   // the group list is host memory
  }
  BSE_LAUNCH(k_real_copy, dim3((unsigned)((N + 255) / 256), (unsigned)n, 1), 256, 0, s, b.dev);
  return 0;
}

int finish_batched(hipStream_t s, const Batch& b) {
  if (b.count <= 0) return 0;
  const int n0 = b.maxn();
  BSE_LAUNCH(k_finish_X, dim3((unsigned)((n0 + 63) / 64), (unsigned)((n0 + 63) / 64), (unsigned)b.count), 256, 0, s, b.dev);
  BSE_LAUNCH(k_phase_weights, dim3((unsigned)n0, 1, (unsigned)b.count), 256, 0, s, b.dev);
  return 0;
}

}  // namespace bse
