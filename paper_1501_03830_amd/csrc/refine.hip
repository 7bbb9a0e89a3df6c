// FP64 refinement of the eigenpairs produced by the mixed-precision path.
//
// Not in the paper: this is an iterative refinement in the style of Ogita and
// Aishima (symmetric eigendecomposition refinement, 2018), carried over to
// the real Schur form of the skew-symmetric W = L^T J L.  If W z = i lambda z
// with z = a + i b, then W a = -lambda b and W b = lambda a, and the columns
// Ub = sqrt(2) [a_1 .. a_n | b_1 .. b_n] satisfy
//     Ub^T Ub = I,   Ub^T W Ub = Sigma = [0 Lambda; -Lambda 0].
// Given an approximate Ub (from the FP32 reduction), one sweep computes in
// FP64, with W = L^T J L from the FP64 Cholesky factor of Algorithm 1 step 2,
//     Y = L Ub,  S = Ub^T W Ub = Y^T J Y = C - C^T (C = Y[0:n]^T Y[n:N]),
//     G = Ub^T Ub,  R = I - G,
// (two products of N^3 flops each for S: L is triangular and C has depth n),
// the refined lambda_k of each pair from its 2 x 2 blocks,
//     lambda_k = s_k / sqrt(det G_kk),  s_k = -S[n+k, k],
// and the correction Ub <- Ub + Ub F, F = R/2 + E with E skew.  E is zero on
// the 2 x 2 diagonal blocks (the phase of z_k is free) and, for k != l,
// solves the first-order Sylvester equation
//     sigma_k E_kl - E_kl sigma_l = -S_kl - (R_kl sigma_l + sigma_k R_kl)/2,
// sigma_k = lambda_k [0 1; -1 0], which has the closed form used below.  For
// lambda_k = lambda_l (a degenerate eigenvalue) the equation is singular
// only along the E that commute with [0 1; -1 0] (rotations inside the
// eigenspace, which are free); the anti-commuting part, which pairs the real
// and imaginary parts, is still determined and is applied (minimum-norm
// solution) for pairs closer than DEGEN relative.
//
// Pairs closer than the FP32 reduction can resolve arrive mixed by large
// angles, and the first-order solution for them exceeds GCAP.  As in Ogita
// and Aishima's treatment of clustered eigenvalues, runs of consecutive pairs
// closer than CGAP relative form clusters (at most REF_CMAX pairs), and a
// cluster with such a block is rotated exactly: with the cluster's 2c x 2c
// blocks G_c = R R^T and S_c of the sweep, K = R^{-1} S_c R^{-T} is skew and
// its real Schur basis Q (pairs a, b with K a = -mu b, K b = mu a) gives the
// cluster's columns of the new basis as Ub_c R^{-T} Q.  Q comes from Jacobi
// on K^T K (eigenvalues mu^2, each twice) followed by Gram-Schmidt that builds
// each pair from one vector a and b = -K a / mu.  The cluster's block of F
// becomes R^{-T} Q - I and the first-order corrections of its columns from
// outside the cluster are carried along (F[l, c] <- F[l, c] R^{-T} Q).  A
// block outside any cluster whose solution exceeds GCAP is left to the
// orthogonalisation part and counted.  The error of Ub falls quadratically; a
// problem stops after the sweep whose largest correction is below STOP_TOL
// with no block left out, then its eigenvalues are taken from the refined
// basis (error of order STOP_TOL^4 relative) and sorted.  A problem still
// short of that after MAX_SWEEPS reports INFO_NOCONV.  Each problem converges
// on its own: kernels skip problems that finished in an earlier sweep.  The
// final eigenvalues use the same identity on the product L Ub that the
// output needs (k_ref_final, after L is applied).
#include <cmath>
#include <cstring>

#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int MAX_SWEEPS = 6;
constexpr double GCAP = 0.25;
constexpr double DEGEN = 1e-10;
// Pairs closer than this (relative) may arrive mixed by angles the
// first-order correction cannot undo: the FP32 basis mixes a pair of
// relative gap g by about 1e-8 / g (measured: largest first correction
// ~1e-3 at gaps near 1e-5 on the n = 8192 workload), i.e. beyond GCAP below
// g ~ 4e-8; 1e-6 leaves a factor of 25.
constexpr double CGAP = 1e-6;
// A sweep whose largest correction entry is e leaves an eigenvalue error of
// about 3.5e-5 e^4 relative (measured on clustered s_a = 0.3 spectra,
// e = 6e-3 .. 6e-2); e <= 1e-2 keeps it near 4e-13, far below 1e-10.
constexpr double STOP_TOL = 1e-2;

// skip problems whose refinement finished before sweep `sweep`
__device__ inline bool finished_before(const Prob& P, int sweep) {
  const int st = *gbl(P.refstate);
  return st != 0 && st <= sweep;
}

__device__ inline double* basis(const Prob& P, int sweep) { return (sweep & 1) ? P.R4 : P.Z; }

// Z <- f Z32 over the N x N block: the basis of sweep 0, from the FP32
// basis the back-transformation left in R4
__global__ __launch_bounds__(256) void k_ref_scale(const Prob* __restrict__ probs, double f) {
  const Prob& P = probs[blockIdx.z];
  const long N = P.N;
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= N) return;
  BSE_GLOBAL double* __restrict__ Z = gbl(P.Z);
  const BSE_GLOBAL float* __restrict__ Z32 = gbl(P.Z32);
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    if (c >= N) break;
    Z[r + c * P.ld] = f * (double)Z32[r + c * P.ld];
  }
}

__global__ void k_ref_reset(const Prob* __restrict__ probs) {
  if (threadIdx.x == 0) *gbl(probs[blockIdx.z].refstate) = 0;
}

// lambda_k of each pair from the 2 x 2 diagonal blocks of S (R2) and G (R3)
__global__ __launch_bounds__(64) void k_ref_lambda(const Prob* __restrict__ probs, int sweep) {
  const Prob& P = probs[blockIdx.z];
  const int n = P.n;
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= n || finished_before(P, sweep)) return;
  const long ld = P.ld;
  const BSE_GLOBAL double* __restrict__ S = gbl(P.R2);
  const BSE_GLOBAL double* __restrict__ G = gbl(P.R3);
  const double s = -S[(n + k) + (long)k * ld];
  const double gaa = G[k + (long)k * ld], gbb = G[(n + k) + (long)(n + k) * ld];
  const double gab = G[(n + k) + (long)k * ld];
  gbl(P.shift)[k] = s / sqrt(gaa * gbb - gab * gab);
}

// S = Ub^T W Ub = C - C^T (lower triangle, in place in R2) from
// C = Y[0:n]^T Y[n:N], Y = L Ub: workgroup (I, J), I >= J, of 64 x 64 tiles
// stages the partner tile (J, I) in LDS, both tiles read along their columns,
// and writes the lower tile (I, J).  Upper tiles are only read, so the
// workgroups do not overlap.
__global__ __launch_bounds__(256) void k_ref_skew(const Prob* __restrict__ probs, int sweep) {
  __shared__ double t[64][65];
  const Prob& P = probs[blockIdx.z];
  if (finished_before(P, sweep)) return;   // uniform
  const long N = P.N, ld = P.ld;
  const int I = blockIdx.x, J = blockIdx.y;
  const long r0 = (long)I * 64, c0 = (long)J * 64;
  if (J > I || r0 >= N) return;   // uniform
  BSE_GLOBAL double* __restrict__ C = gbl(P.R2);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // t[i][j] = C[c0 + j, r0 + i], the partner of C[r0 + i, c0 + j]
  for (int i = wv; i < 64; i += 4) {
    const long col = r0 + i, row = c0 + lane;
    t[i][lane] = (col < N && row < N) ? C[row + col * ld] : 0.0;
  }
  __syncthreads();
  const long row = r0 + lane;
  if (row >= N) return;
  for (int j = wv; j < 64; j += 4) {
    const long col = c0 + j;
    if (col > row || col >= N) continue;
    BSE_GLOBAL double* e = C + row + col * ld;
    *e = *e - t[lane][j];
  }
}

// entry (i, j) of the full matrices from their stored lower triangles
__device__ inline double skew_at(const BSE_GLOBAL double* S, long ld, long i, long j) {
  return (i >= j) ? S[i + j * ld] : -S[j + i * ld];
}
__device__ inline double sym_at(const BSE_GLOBAL double* G, long ld, long i, long j) {
  return (i >= j) ? G[i + j * ld] : G[j + i * ld];
}

// F and a copy of Ub, both rounded to FP32, into R1 (Y = L Ub is no longer
// needed): the basis update Ub + Ub F takes its correction product in FP32,
// which perturbs Ub by about 1e-7 of the correction (far below the error the
// sweep leaves).  Also per-tile maxima of the correction and the number of
// clamped blocks.
//
// One workgroup per 32 x 32 block of pairs (k, l): it produces the four
// output tiles at rows {k, n+k} and columns {l, n+l}, so each 2 x 2 block of
// S and G is read once (by output element it was read four times), and every
// global access is coalesced: the eight source tiles (S and G, four
// quadrants) are staged in LDS, lower-triangle entries with lanes along the
// stored rows and mirrored ones with lanes along the stored columns.
constexpr int RFB = 32;   // pairs per block side
__global__ __launch_bounds__(256) void k_ref_F(const Prob* __restrict__ probs, int sweep) {
  __shared__ double tS[4][RFB][RFB + 1];   // [quadrant][l][k]
  __shared__ double tG[4][RFB][RFB + 1];
  __shared__ double red[2][4];
  __shared__ int cst[2][RFB];              // cluster starts of the k and l pairs
  const Prob& P = probs[blockIdx.z];
  const long n = P.n, ld = P.ld;
  const long nblk = (n + RFB - 1) / RFB;
  if ((long)blockIdx.x >= nblk || (long)blockIdx.y >= nblk) return;   // uniform
  if (finished_before(P, sweep)) return;
  const BSE_GLOBAL double* __restrict__ S = gbl(P.R2);
  const BSE_GLOBAL double* __restrict__ G = gbl(P.R3);
  const BSE_CONST double* __restrict__ lam = ro(P.shift);
  BSE_GLOBAL float* __restrict__ F32 = gbl(reinterpret_cast<float*>(P.R1));
  BSE_GLOBAL float* __restrict__ U32 = F32 + ld * ld;
  const BSE_GLOBAL double* __restrict__ Ub = gbl(basis(P, sweep));
  const long k0 = (long)blockIdx.x * RFB, l0 = (long)blockIdx.y * RFB;
  const int tid = threadIdx.x;
  if (tid < 2 * RFB) {
    const long q = (tid < RFB ? k0 : l0 - RFB) + tid;
    cst[tid / RFB][tid % RFB] = (q < n) ? gbl(P.clstart)[q] : -1 - tid;
  }
  // quadrant q = 2 qr + qc holds (row k + n qr, column l + n qc); S is
  // skew and G symmetric, both stored as their lower triangles
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long orow = (q >> 1) ? n : 0, ocol = (q & 1) ? n : 0;
    // lower entries, lanes along the stored rows (k)
    for (int idx = tid; idx < RFB * RFB; idx += 256) {
      const int kk = idx % RFB, ll = idx / RFB;
      const long k = k0 + kk, l = l0 + ll;
      const long gr = k + orow, gc = l + ocol;
      if (k < n && l < n && gr >= gc) {
        tS[q][ll][kk] = S[gr + gc * ld];
        tG[q][ll][kk] = G[gr + gc * ld];
      } else if (k >= n || l >= n) {
        tS[q][ll][kk] = 0.0;
        tG[q][ll][kk] = 0.0;
      }
    }
    // mirrored entries, lanes along the stored rows (l)
    for (int idx = tid; idx < RFB * RFB; idx += 256) {
      const int ll = idx % RFB, kk = idx / RFB;
      const long k = k0 + kk, l = l0 + ll;
      const long gr = k + orow, gc = l + ocol;
      if (k < n && l < n && gr < gc) {
        tS[q][ll][kk] = -S[gc + gr * ld];
        tG[q][ll][kk] = G[gc + gr * ld];
      }
    }
  }
  __syncthreads();
  const int kk = tid % RFB, lg = tid / RFB;   // 8 groups of 4 columns
  const long k = k0 + kk;
  double cmax = 0.0, nclamp = 0.0;
  if (k < n) {
    const double lk = lam[k];
    for (int u = 0; u < RFB / 8; ++u) {
      const int ll = lg * (RFB / 8) + u;
      const long l = l0 + ll;
      if (l >= n) break;
      const double R11 = -tG[0][ll][kk], R12 = -tG[1][ll][kk];
      const double R21 = -tG[2][ll][kk], R22 = -tG[3][ll][kk];
      double e11 = 0.0, e12 = 0.0, e21 = 0.0, e22 = 0.0;
      if (k != l) {
        const double ll_ = lam[l];
        const double S11 = tS[0][ll][kk], S12 = tS[1][ll][kk];
        const double S21 = tS[2][ll][kk], S22 = tS[3][ll][kk];
        // C = -S_kl - (R_kl sigma_l + sigma_k R_kl) / 2
        const double c11 = -S11 - 0.5 * (-R12 * ll_ + lk * R21);
        const double c12 = -S12 - 0.5 * (R11 * ll_ + lk * R22);
        const double c21 = -S21 - 0.5 * (-R22 * ll_ - lk * R11);
        const double c22 = -S22 - 0.5 * (R21 * ll_ - lk * R12);
        if (fabs(lk - ll_) <= DEGEN * fmax(lk, ll_)) {
          // degenerate pair: g22 - g11 and g12 + g21 are fixed, the rest is free
          const double lm = 0.5 * (lk + ll_);
          const double d = (c12 + c21) / (4.0 * lm), h = (c11 - c22) / (4.0 * lm);
          e11 = -d;
          e12 = h;
          e21 = h;
          e22 = d;
        } else {
          const double det = lk * lk - ll_ * ll_;
          const double f11 = (c12 * ll_ - lk * c21) / det;
          const double f22 = (-ll_ * c21 + lk * c12) / det;
          const double f12 = (-ll_ * c11 - lk * c22) / det;
          const double f21 = (ll_ * c22 + lk * c11) / det;
          const double emax = fmax(fmax(fabs(f11), fabs(f12)), fmax(fabs(f21), fabs(f22)));
          if (emax <= GCAP) {   // NaN or a close pair: orthogonalise only
            e11 = f11;
            e12 = f12;
            e21 = f21;
            e22 = f22;
          } else if (cst[0][kk] == cst[1][ll]) {
            // inside a cluster: the exact rotation of the cluster replaces
            // this block (k_ref_rr)
            gbl(P.clflag)[cst[0][kk]] = 1;
          } else {
            nclamp += 4.0;   // one per output entry of the block
          }
        }
      }
      // F = R/2 + E at (k, l), (k, n+l), (n+k, l), (n+k, n+l); R = I - G
      const double dg = (k == l) ? 1.0 : 0.0;
      const double f11 = 0.5 * (dg + R11) + e11, f12 = 0.5 * R12 + e12;
      const double f21 = 0.5 * R21 + e21, f22 = 0.5 * (dg + R22) + e22;
      if (k != l) cmax = fmax(cmax, fmax(fabs(f11), fabs(f22)));
      cmax = fmax(cmax, fmax(fabs(f12), fabs(f21)));
      const long o11 = k + l * ld, o12 = k + (n + l) * ld, o21 = (n + k) + l * ld, o22 = (n + k) + (n + l) * ld;
      F32[o11] = (float)f11;
      F32[o12] = (float)f12;
      F32[o21] = (float)f21;
      F32[o22] = (float)f22;
      U32[o11] = (float)Ub[o11];
      U32[o12] = (float)Ub[o12];
      U32[o21] = (float)Ub[o21];
      U32[o22] = (float)Ub[o22];
    }
  }
  // workgroup maxima / sums
  for (int off = 32; off >= 1; off >>= 1) {
    cmax = fmax(cmax, __shfl_xor(cmax, off, 64));
    nclamp += __shfl_xor(nclamp, off, 64);
  }
  const int w = tid >> 6;
  if ((tid & 63) == 0) {
    red[0][w] = cmax;
    red[1][w] = nclamp;
  }
  __syncthreads();
  if (tid == 0) {
    double m = 0.0, cl = 0.0;
    for (int i = 0; i < 4; ++i) {
      m = fmax(m, red[0][i]);
      cl += red[1][i];
    }
    // one slot per block, as many blocks as 64 x 64 tiles of the N x N matrix
    const long t = (long)blockIdx.x + (long)blockIdx.y * nblk;
    BSE_GLOBAL double* __restrict__ part = gbl(P.refmax);
    part[2 * t] = m;
    part[2 * t + 1] = cl;
  }
}

// Clusters of the sweep: runs of consecutive pairs whose eigenvalue
// estimates differ by at most CGAP relative, cut into pieces of REF_CMAX
// pairs.  clstart[k] = first pair of k's cluster; the cluster flags and
// maxima are cleared.  One workgroup per problem: each thread takes a chunk
// of pairs, and the last run start before every chunk comes from a scan.
__device__ inline bool cluster_break(const BSE_GLOBAL double* lam, int k) {
  if (k == 0) return true;
  const double a = lam[k], b = lam[k - 1];
  return !(fabs(a - b) <= CGAP * fmax(a, b));
}

__global__ __launch_bounds__(1024) void k_ref_clusters(const Prob* __restrict__ probs, int sweep) {
  __shared__ int last[1024];
  const Prob& P = probs[blockIdx.z];
  if (finished_before(P, sweep)) return;
  const int n = P.n;
  const BSE_GLOBAL double* __restrict__ lam = gbl(P.shift);
  const int T = blockDim.x;
  const int chunk = (n + T - 1) / T;
  const int b = threadIdx.x * chunk, e = min(n, b + chunk);
  int lb = -1;
  for (int k = b; k < e; ++k)
    if (cluster_break(lam, k)) lb = k;
  last[threadIdx.x] = lb;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < T; ++t) {
      const int v = last[t];
      last[t] = run;
      if (v >= 0) run = v;
    }
  }
  __syncthreads();
  int r = last[threadIdx.x];
  BSE_GLOBAL int* __restrict__ cs = gbl(P.clstart);
  for (int k = b; k < e; ++k) {
    if (cluster_break(lam, k)) r = k;
    cs[k] = r + ((k - r) / REF_CMAX) * REF_CMAX;
    gbl(P.clflag)[k] = 0;
    gbl(P.clmax)[k] = 0.0;
  }
}

// Pairs (basis columns k and n + k) of the cluster that starts at pair k0
// with c pairs, as indices 0..2c-1 of its block.
__device__ inline long cluster_col(int i, int c, long k0, long n) { return i < c ? k0 + i : n + k0 + (i - c); }

__device__ inline int cluster_size(const BSE_GLOBAL int* cs, int k0, int n) {
  int c = 1;
  while (k0 + c < n && c < REF_CMAX && cs[k0 + c] == k0) ++c;
  return c;
}

// Exact rotation of one flagged cluster (one wavefront per cluster start):
// T = R^{-T} Q as described at the top of this file, into the cluster's
// block of F (T - I, FP32) and its slot of clT (FP64), with max |T - I| in
// clmax.  If G_c is not numerically positive definite or Q cannot be
// completed, nothing is written except a large clmax (the sweep counts as
// not converged).
constexpr int RM = 2 * REF_CMAX;
__global__ __launch_bounds__(64) void k_ref_rr(const Prob* __restrict__ probs, int sweep) {
  __shared__ double Km[RM][RM + 1];
  __shared__ double Mm[RM][RM + 1];
  __shared__ double Vm[RM][RM + 1];
  __shared__ double Rm[RM][RM + 1];
  __shared__ double Qm[RM][RM + 1];
  __shared__ double vec[RM];
  __shared__ int ord[RM];
  const Prob& P = probs[blockIdx.z];
  const int n = P.n;
  const int k0 = blockIdx.x;
  if (k0 >= n || finished_before(P, sweep)) return;
  const BSE_GLOBAL int* __restrict__ cs = gbl(P.clstart);
  if (cs[k0] != k0 || gbl(P.clflag)[k0] == 0) return;
  const int c = cluster_size(cs, k0, n);
  const int m = 2 * c;
  const long ld = P.ld;
  const int lane = threadIdx.x;
  const BSE_GLOBAL double* __restrict__ S = gbl(P.R2);
  const BSE_GLOBAL double* __restrict__ G = gbl(P.R3);
  for (int idx = lane; idx < m * m; idx += 64) {
    const int i = idx % m, j = idx / m;
    const long gi = cluster_col(i, c, k0, n), gj = cluster_col(j, c, k0, n);
    Km[i][j] = skew_at(S, ld, gi, gj);
    Rm[i][j] = sym_at(G, ld, gi, gj);
  }
  __syncthreads();
  // G_c = R R^T, lower, column by column
  bool ok = true;
  for (int j = 0; j < m; ++j) {
    const double djj = Rm[j][j];
    ok = ok && (djj > 0.0);
    const double d = sqrt(fmax(djj, 1e-300));
    __syncthreads();
    if (lane == j) Rm[j][j] = d;
    if (lane > j && lane < m) Rm[lane][j] /= d;
    __syncthreads();
    for (int idx = lane; idx < m * m; idx += 64) {
      const int i = idx % m, l = idx / m;
      if (l > j && i >= l) Rm[i][l] -= Rm[i][j] * Rm[l][j];
    }
    __syncthreads();
  }
  // X = R^{-1} S_c (lane = column), then K = X R^{-T} (lane = row)
  if (lane < m) {
    for (int i = 0; i < m; ++i) {
      double x = Km[i][lane];
      for (int l = 0; l < i; ++l) x -= Rm[i][l] * Mm[l][lane];
      Mm[i][lane] = x / Rm[i][i];
    }
  }
  __syncthreads();
  if (lane < m) {
    for (int j = 0; j < m; ++j) {
      double y = Mm[lane][j];
      for (int l = 0; l < j; ++l) y -= Rm[j][l] * Vm[lane][l];
      Vm[lane][j] = y / Rm[j][j];
    }
  }
  __syncthreads();
  for (int idx = lane; idx < m * m; idx += 64) {
    const int i = idx % m, j = idx / m;
    Km[i][j] = 0.5 * (Vm[i][j] - Vm[j][i]);
  }
  __syncthreads();
  // K^T K and V = I
  for (int idx = lane; idx < m * m; idx += 64) {
    const int i = idx % m, j = idx / m;
    double t = 0.0;
    for (int l = 0; l < m; ++l) t += Km[l][i] * Km[l][j];
    Mm[i][j] = t;
    Vm[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // cyclic Jacobi on K^T K
  for (int sw = 0; sw < 30; ++sw) {
    double off = 0.0, dia = 0.0;
    for (int idx = lane; idx < m * m; idx += 64) {
      const int i = idx % m, j = idx / m;
      if (i == j) dia = fmax(dia, fabs(Mm[i][j]));
      else off = fmax(off, fabs(Mm[i][j]));
    }
    for (int o = 32; o >= 1; o >>= 1) {
      off = fmax(off, __shfl_xor(off, o, 64));
      dia = fmax(dia, __shfl_xor(dia, o, 64));
    }
    if (off <= 1e-15 * dia) break;
    for (int p = 0; p < m - 1; ++p) {
      for (int q = p + 1; q < m; ++q) {
        const double apq = Mm[p][q];
        if (apq == 0.0) continue;
        const double theta = (Mm[q][q] - Mm[p][p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cr = 1.0 / sqrt(t * t + 1.0), sr = t * cr;
        __syncthreads();
        if (lane < m) {
          const double mp = Mm[lane][p], mq = Mm[lane][q];
          Mm[lane][p] = cr * mp - sr * mq;
          Mm[lane][q] = sr * mp + cr * mq;
          const double vp = Vm[lane][p], vq = Vm[lane][q];
          Vm[lane][p] = cr * vp - sr * vq;
          Vm[lane][q] = sr * vp + cr * vq;
        }
        __syncthreads();
        if (lane < m) {
          const double mp = Mm[p][lane], mq = Mm[q][lane];
          Mm[p][lane] = cr * mp - sr * mq;
          Mm[q][lane] = sr * mp + cr * mq;
        }
        __syncthreads();
        if (lane == 0) {
          Mm[p][q] = 0.0;
          Mm[q][p] = 0.0;
        }
        __syncthreads();
      }
    }
  }
  // eigenvectors of K^T K by increasing eigenvalue
  if (lane < m) {
    const double d = Mm[lane][lane];
    int rank = 0;
    for (int j = 0; j < m; ++j) rank += (Mm[j][j] < d) || (Mm[j][j] == d && j < lane);
    ord[rank] = lane;
  }
  __syncthreads();
  // pairs (a, b = -K a / mu), each orthogonal to the pairs before it
  int np = 0;
  for (int r = 0; r < m && np < c; ++r) {
    const int col = ord[r];
    double v = (lane < m) ? Vm[lane][col] : 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < np; ++j) {
        const double qa = (lane < m) ? Qm[lane][j] : 0.0;
        v -= wave_sum(qa * v) * qa;
        const double qb = (lane < m) ? Qm[lane][c + j] : 0.0;
        v -= wave_sum(qb * v) * qb;
      }
    }
    const double nv = sqrt(wave_sum(v * v));
    if (nv < 0.5) continue;
    v /= nv;
    if (lane < m) vec[lane] = v;
    __syncthreads();
    double ka = 0.0;
    if (lane < m)
      for (int j = 0; j < m; ++j) ka += Km[lane][j] * vec[j];
    __syncthreads();
    double bv = -ka;
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < np; ++j) {
        const double qa = (lane < m) ? Qm[lane][j] : 0.0;
        bv -= wave_sum(qa * bv) * qa;
        const double qb = (lane < m) ? Qm[lane][c + j] : 0.0;
        bv -= wave_sum(qb * bv) * qb;
      }
      bv -= wave_sum(v * bv) * v;
    }
    const double nb = sqrt(wave_sum(bv * bv));
    if (!(nb > 0.0)) continue;
    bv /= nb;
    if (lane < m) {
      Qm[lane][np] = v;
      Qm[lane][c + np] = bv;
    }
    __syncthreads();
    ++np;
  }
  ok = ok && (np == c);
  if (!ok) {
    if (lane == 0) gbl(P.clmax)[k0] = 1e300;
    return;
  }
  // T = R^{-T} Q (lane = column), into Km
  if (lane < m) {
    for (int i = m - 1; i >= 0; --i) {
      double t = Qm[i][lane];
      for (int l = i + 1; l < m; ++l) t -= Rm[l][i] * Km[l][lane];
      Km[i][lane] = t / Rm[i][i];
    }
  }
  __syncthreads();
  BSE_GLOBAL float* __restrict__ F32 = gbl(reinterpret_cast<float*>(P.R1));
  BSE_GLOBAL double* __restrict__ Tg = gbl(P.clT) + (long)k0 * REF_CMAX4;
  double mx = 0.0;
  for (int idx = lane; idx < m * m; idx += 64) {
    const int i = idx % m, j = idx / m;
    const double t = Km[i][j], f = t - ((i == j) ? 1.0 : 0.0);
    F32[cluster_col(i, c, k0, n) + cluster_col(j, c, k0, n) * ld] = (float)f;
    Tg[i + j * m] = t;
    mx = fmax(mx, fabs(f));
  }
  for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) gbl(P.clmax)[k0] = mx;
}

// The first-order corrections of a rotated cluster's columns from outside
// the cluster follow the rotation: F[l, c] <- F[l, c] T for every row l
// outside the cluster (one workgroup per cluster start).
__global__ __launch_bounds__(256) void k_ref_rr_rows(const Prob* __restrict__ probs, int sweep) {
  __shared__ double Ts[RM * RM];
  const Prob& P = probs[blockIdx.z];
  const int n = P.n;
  const int k0 = blockIdx.x;
  if (k0 >= n || finished_before(P, sweep)) return;
  const BSE_GLOBAL int* __restrict__ cs = gbl(P.clstart);
  if (cs[k0] != k0 || gbl(P.clflag)[k0] == 0) return;
  if (!(gbl(P.clmax)[k0] < 1e300)) return;   // no rotation was made
  const int c = cluster_size(cs, k0, n);
  const int m = 2 * c;
  const long ld = P.ld, N = P.N;
  const BSE_GLOBAL double* __restrict__ Tg = gbl(P.clT) + (long)k0 * REF_CMAX4;
  for (int idx = threadIdx.x; idx < m * m; idx += 256) Ts[idx] = Tg[idx];
  __syncthreads();
  BSE_GLOBAL float* __restrict__ F32 = gbl(reinterpret_cast<float*>(P.R1));
  for (long l = threadIdx.x; l < N; l += 256) {
    const bool inside = (l >= k0 && l < k0 + c) || (l >= n + k0 && l < n + k0 + c);
    if (inside) continue;
    double f[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) f[i] = (i < m) ? (double)F32[l + cluster_col(i, c, k0, n) * ld] : 0.0;
#pragma unroll
    for (int j = 0; j < RM; ++j) {
      if (j >= m) break;
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < RM; ++i) t += f[i] * Ts[i + j * m];
      F32[l + cluster_col(j, c, k0, n) * ld] = (float)t;
    }
  }
}

// reduce the tile maxima; decide whether this problem is done after `sweep`
__global__ __launch_bounds__(256) void k_ref_decide(const Prob* __restrict__ probs, int sweep) {
  __shared__ double red[2][4];
  const Prob& P = probs[blockIdx.z];
  if (finished_before(P, sweep)) return;
  const long ntile = (P.N + 63) / 64;
  const long nt2 = ntile * ntile;
  const BSE_GLOBAL double* __restrict__ part = gbl(P.refmax);
  double m = 0.0, cl = 0.0;
  for (long t = threadIdx.x; t < nt2; t += 256) {
    m = fmax(m, part[2 * t]);
    cl += part[2 * t + 1];
  }
  // exact cluster rotations of this sweep (zero where none was made)
  for (long k = threadIdx.x; k < P.n; k += 256) m = fmax(m, gbl(P.clmax)[k]);
  for (int off = 32; off >= 1; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off, 64));
    cl += __shfl_xor(cl, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = m;
    red[1][w] = cl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0, cc = 0.0;
    for (int i = 0; i < 4; ++i) {
      mm = fmax(mm, red[0][i]);
      cc += red[1][i];
    }
    gbl(P.refout)[0] = mm;
    gbl(P.refout)[1] = cc;
    const bool converged = (mm < STOP_TOL) && (cc == 0.0);
    if (converged || sweep == MAX_SWEEPS - 1) *gbl(P.refstate) = sweep + 1;
    if (!converged && sweep == MAX_SWEEPS - 1 && gbl(P.info)[1] == 0) gbl(P.info)[1] = INFO_NOCONV;
  }
}

// lambda_k = -b_k^T W a_k / sqrt(det [a_k b_k]^T [a_k b_k]) for the final
// basis pair [a_k b_k] = sqrt(2) [Z_k Z_{n+k}], taken after L is applied
// (G = L Z in P.W): with W = L^T J L, b^T W a = (L b)^T J (L a), so
//   b_k^T W a_k = 2 sum_{i<n} (G[i, n+k] G[n+i, k] - G[n+i, n+k] G[i, k])
// and the factors of 2 cancel against those of the Gram determinant.  This
// spares a product with W of n columns; G is the FP64 product the output
// needs anyway.  One workgroup per pair.
__global__ __launch_bounds__(256) void k_ref_final(const Prob* __restrict__ probs) {
  __shared__ double red[4][4];
  const Prob& P = probs[blockIdx.z];
  const long n = P.n, N = P.N, ld = P.ld;
  const long k = blockIdx.x;
  if (k >= n) return;   // uniform
  const BSE_GLOBAL double* __restrict__ Z = gbl(P.Z);
  const BSE_GLOBAL double* __restrict__ G = gbl(P.W);
  const BSE_GLOBAL double* za = Z + k * ld;
  const BSE_GLOBAL double* zb = Z + (n + k) * ld;
  const BSE_GLOBAL double* ga = G + k * ld;
  const BSE_GLOBAL double* gb = G + (n + k) * ld;
  double s = 0.0, gaa = 0.0, gbb = 0.0, gab = 0.0;
  for (long r = threadIdx.x; r < n; r += 256) s += gb[r] * ga[n + r] - gb[n + r] * ga[r];
  for (long r = threadIdx.x; r < N; r += 256) {
    const double a = za[r], b = zb[r];
    gaa += a * a;
    gbb += b * b;
    gab += a * b;
  }
  s = block_sum(s, red[0]);
  gaa = block_sum(gaa, red[1]);
  gbb = block_sum(gbb, red[2]);
  gab = block_sum(gab, red[3]);
  if (threadIdx.x == 0) gbl(P.shift)[k] = -s / sqrt(gaa * gbb - gab * gab);
}

// ascending order: rank of each eigenvalue by counting (ties by index)
__global__ __launch_bounds__(256) void k_ref_sort(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  const int n = P.n;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const BSE_CONST double* __restrict__ lam = ro(P.shift);
  const double x = lam[k];
  int rank = 0;
  for (int m = 0; m < n; ++m) {
    const double y = lam[m];
    rank += (y < x) || (y == x && m < k);
  }
  gbl(P.perm)[rank] = k;
  gbl(P.lambda)[rank] = x;
}

// final basis / sqrt(2) into Z
__global__ __launch_bounds__(256) void k_ref_out(const Prob* __restrict__ probs) {
  const Prob& P = probs[blockIdx.z];
  const long N = P.N;
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= N) return;
  const BSE_GLOBAL double* __restrict__ U = gbl(basis(P, *gbl(P.refstate)));
  BSE_GLOBAL double* __restrict__ Z = gbl(P.Z);
  const double f = 0.70710678118654752440;   // 1/sqrt(2)
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    if (c >= N) break;
    Z[r + c * P.ld] = f * U[r + c * P.ld];
  }
}

dim3 grid_NN(const Batch& b) {
  const long N0 = b.maxN();
  return dim3((unsigned)((N0 + 63) / 64), (unsigned)((N0 + 63) / 64), (unsigned)b.count);
}

}  // namespace

int refine_batched(hipStream_t s, const Batch& b, const RefineIO& io, RefineStats* st) {
  if (b.count <= 0) return 0;
  const int n0 = b.maxn();
  BSE_LAUNCH(k_ref_reset, dim3(1, 1, (unsigned)b.count), 64, 0, s, b.dev);
  BSE_LAUNCH(k_ref_scale, grid_NN(b), 256, 0, s, b.dev, 1.41421356237309504880);
  int sweeps = 0;
  for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
    // S = Ub^T W Ub through Y = L Ub (W = L^T J L): 2 N^3 flops where the
    // product with W and then with Ub^T took 2.5 N^3
    BSE_TRY(gemm_batched(s, b, b.count, GOP_REF_Y, sweep));
    BSE_TRY(gemm_batched(s, b, b.count, GOP_REF_C, sweep));
    {
      const unsigned nt = (unsigned)((b.maxN() + 63) / 64);
      BSE_LAUNCH(k_ref_skew, dim3(nt, nt, (unsigned)b.count), 256, 0, s, b.dev, sweep);
    }
    BSE_TRY(gemm_batched(s, b, b.count, GOP_REF_G, sweep));
    BSE_LAUNCH(k_ref_lambda, dim3((unsigned)((n0 + 63) / 64), 1, (unsigned)b.count), 64, 0, s, b.dev, sweep);
    BSE_LAUNCH(k_ref_clusters, dim3(1, 1, (unsigned)b.count), 1024, 0, s, b.dev, sweep);
    BSE_LAUNCH(k_ref_F, grid_NN(b), 256, 0, s, b.dev, sweep);
    BSE_LAUNCH(k_ref_rr, dim3((unsigned)n0, 1, (unsigned)b.count), 64, 0, s, b.dev, sweep);
    BSE_LAUNCH(k_ref_rr_rows, dim3((unsigned)n0, 1, (unsigned)b.count), 256, 0, s, b.dev, sweep);
    BSE_LAUNCH(k_ref_decide, dim3(1, 1, (unsigned)b.count), 256, 0, s, b.dev, sweep);
    BSE_TRY(gemm_batched(s, b, b.count, GOP_REF_U, sweep));
    sweeps = sweep + 1;
    // every problem's state and largest correction, to decide on the host
    BSE_HIP(hipMemcpyAsync(io.hstate, io.dstate, io.nslots * sizeof(int), hipMemcpyDeviceToHost, s));
    BSE_HIP(hipMemcpyAsync(io.hout, io.dout, io.nslots * 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    BSE_HIP(hipStreamSynchronize(s));
    bool all_done = true;
    double worst = 0.0;
    for (int i = 0; i < b.count; ++i) {
      const long slot = b.host[i].refstate - io.dstate;
      const int state = io.hstate[slot];
      if (state == 0) all_done = false;
      if (state == 0 || state == sweep + 1) worst = fmax(worst, io.hout[2 * slot]);
    }
    if (st) {
      st->last_correction = worst;
      if (sweep == 0) st->first_correction = worst;
    }
    if (all_done) break;
  }
  if (st) st->sweeps = sweeps;
  // the final basis / sqrt(2) to Z, where L is applied to it; the eigenvalues
  // follow from that product (refine_final_batched)
  BSE_LAUNCH(k_ref_out, grid_NN(b), 256, 0, s, b.dev);
  return 0;
}

int refine_final_batched(hipStream_t s, const Batch& b) {
  if (b.count <= 0) return 0;
  const int n0 = b.maxn();
  BSE_LAUNCH(k_ref_final, dim3((unsigned)n0, 1, (unsigned)b.count), 256, 0, s, b.dev);
  BSE_LAUNCH(k_ref_sort, dim3((unsigned)((n0 + 255) / 256), 1, (unsigned)b.count), 256, 0, s, b.dev);
  return 0;
}

}  // namespace bse
