// Solves with one 64 x 64 triangular block, one thread per right-hand side.
//
// Three places of the chain apply the inverse of a small triangular block to
// many vectors:
//   * the Cholesky panel (Algorithm 1 step 2): A21 <- A21 L_kk^{-T}, i.e.
//     L_kk x = a for every row a of A21;
//   * the forward substitution of the cluster Gram-Schmidt (Algorithm 3
//     step 2): L_bb X = B for the 64 rows of V_+^T at block b;
//   * the compact-WY application of the reflectors (Algorithm 3 step 3):
//     W2 = T W1 with I - V T V^T = H_j0 ... H_j0+127, one 64-row diagonal
//     block of T^{-1} at a time.  For reflectors
//     H = I - tau v v^T the factor built by LAPACK's larft recurrence is the
//     inverse of diag(1/tau) + strict_upper(V^T V), so W2 solves
//     (diag(1/tau) + strict_upper(V^T V)) W2 = W1 and T is never formed.
// Each thread keeps its vector in registers and runs the substitution in
// axpy form (once x_l is final it is removed from the remaining rows), so
// the updates of one step are independent instructions.  The triangular
// block is the same for every lane and is staged in LDS, where every lane
// reads the same address (a broadcast).  The lower-triangular solves run one
// wavefront per workgroup, which spreads a panel of 16384 rows over 256
// compute units; the block is read from LDS with its diagonal replaced by
// the reciprocal (the scalar cache, read step by step, left every wave
// waiting on cache misses, ~70 us per 16384-row panel).
#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int NB = 64;
#define BSE_LDS __attribute__((address_space(3)))

// Stage the lower-triangular block at Lp (column-major, ld) of order 64
// (FULL) or nbk < 64 into Ls[col][row], the diagonal replaced by its
// reciprocal; entries outside the nbk x nbk block are zero.  Run by a
// 64-lane workgroup, lane = row; ends with a barrier.
template <bool FULL>
__device__ inline void stage_lower64(const BSE_GLOBAL double* Lp, long ld, int nbk, BSE_LDS double (*Ls)[NB]) {
  const int t = threadIdx.x;
#pragma unroll 16
  for (int l = 0; l < NB; ++l)
    Ls[l][t] = (FULL || (l < nbk && t < nbk)) ? Lp[t + (long)l * ld] : 0.0;
  __syncthreads();
  if (FULL || t < nbk) Ls[t][t] = 1.0 / Ls[t][t];
  __syncthreads();
}

// x <- L^{-1} x with L staged by stage_lower64.  The reads of each step are
// taken in groups of 16 rows with a scheduling barrier after each group: left
// free, the compiler hoists the whole triangle's reads and spills.
template <bool FULL, int L0, int L1>
__device__ __attribute__((always_inline)) inline void lower_solve_steps(const BSE_LDS double (*Ls)[NB], int nbk,
                                                                        double (&x)[NB]) {
#pragma unroll
  for (int l = L0; l < L1; ++l) {
    if (FULL || l < nbk) {
      x[l] *= Ls[l][l];
#pragma unroll
      for (int r = l + 1; r < NB; ++r) {
        if (FULL || r < nbk) x[r] -= Ls[l][r] * x[l];
        if (((r - l) & 15) == 0) __builtin_amdgcn_sched_barrier(0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}
// (four loops of 16 steps: one loop of 64 is past the compiler's limit for
// a full unroll, and x must stay in registers)
template <bool FULL>
__device__ __attribute__((always_inline)) inline void lower_solve64(const BSE_LDS double (*Ls)[NB], int nbk,
                                                                    double (&x)[NB]) {
  lower_solve_steps<FULL, 0, 16>(Ls, nbk, x);
  lower_solve_steps<FULL, 16, 32>(Ls, nbk, x);
  lower_solve_steps<FULL, 32, 48>(Ls, nbk, x);
  lower_solve_steps<FULL, 48, 64>(Ls, nbk, x);
}

// x <- U^{-1} x, U upper, Us[col][row], with the reciprocal of U's diagonal
// stored on the diagonal of Us
__device__ inline void upper_solve64(const double (*Us)[NB + 1], double (&x)[NB]) {
#pragma unroll
  for (int l = NB - 1; l >= 0; --l) {
    x[l] *= Us[l][l];
#pragma unroll
    for (int r = 0; r < l; ++r) x[r] -= Us[l][r] * x[l];
  }
}

// Cholesky panel: rows k0+nbk .. Nm-1 of the panel columns k0 .. k0+nbk-1
// of matrix sel (0: M, 1: the Gram matrix) <- themselves times L_kk^{-T}.
// One wavefront of 64 rows per workgroup.
template <bool FULL>
__global__ __launch_bounds__(NB) void k_trsm_rows(const Prob* __restrict__ probs, int sel, int k0) {
  __shared__ double Ls[NB][NB];
  const Prob& P = probs[blockIdx.z];
  double* Mp;
  long ld;
  int Nm;
  if (sel == 0) {
    Mp = P.L;
    ld = P.ld;
    Nm = P.N;
  } else {
    Mp = P.inv;
    ld = P.n;
    Nm = P.n;
  }
  if (k0 >= Nm || gbl(P.info)[sel] != 0) return;   // uniform
  if (sel == 1 && *gbl(P.reorth) == 0) return;     // uniform: no Gram-Schmidt
  const int nbk = min(NB, Nm - k0);
  if (FULL != (nbk == NB)) return;                  // uniform: the other variant
  const int first = k0 + nbk;
  if (first + (long)blockIdx.x * NB >= Nm) return;   // uniform: past this problem's rows
  // the diagonal block is not written by this launch (only the rows below)
  BSE_GLOBAL double* __restrict__ M = gbl(Mp);
  stage_lower64<FULL>(M + (long)k0 + (long)k0 * ld, ld, nbk, (BSE_LDS double(*)[NB])Ls);
  const long r = first + (long)blockIdx.x * NB + threadIdx.x;
  if (r >= Nm) return;
  double x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = (FULL || c < nbk) ? M[r + (long)(k0 + c) * ld] : 0.0;
  lower_solve64<FULL>((const BSE_LDS double(*)[NB])Ls, nbk, x);
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (FULL || c < nbk) M[r + (long)(k0 + c) * ld] = x[c];
}

// Gram-Schmidt forward substitution, diagonal block b0: rows b0 .. b0+63 of
// V_+^T (n x N, ld n) <- L_bb^{-1} times themselves, one column per thread,
// one wavefront per workgroup.
template <bool FULL>
__global__ __launch_bounds__(NB) void k_trsm_cols(const Prob* __restrict__ probs, int b0) {
  __shared__ double Ls[NB][NB];
  const Prob& P = probs[blockIdx.z];
  const int n = P.n, N = P.N;
  if (b0 >= n || gbl(P.info)[1] != 0) return;   // uniform
  if (*gbl(P.reorth) == 0) return;              // uniform: no Gram-Schmidt
  const int nbk = min(NB, n - b0);
  if (FULL != (nbk == NB)) return;              // uniform: the other variant
  if ((long)blockIdx.x * NB >= N) return;       // uniform: past this problem's columns
  // Gram factor, read-only here
  stage_lower64<FULL>(gbl(P.inv) + (long)b0 + (long)b0 * n, n, nbk, (BSE_LDS double(*)[NB])Ls);
  const long j = (long)blockIdx.x * NB + threadIdx.x;
  if (j >= N) return;
  BSE_GLOBAL double* __restrict__ v = gbl(P.Vt) + b0 + j * n;
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = (FULL || i < nbk) ? v[i] : 0.0;
  lower_solve64<FULL>((const BSE_LDS double(*)[NB])Ls, nbk, x);
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (FULL || i < nbk) v[i] = x[i];
}

// Compact-WY factor of reflector block q (RB = APPLYU_RB reflectors):
// T^{-1} = diag(1/tau) + strict_upper(S), S = V^T V, is block upper
// triangular in 64 x 64 blocks, so W2 = T W1 is a block back substitution:
// for h = RB/64 - 1 .. 0, rows h of W1 minus S[h, h+1:] W2[h+1:] (a GEMM,
// skipped for the last h), then the solve with the diagonal block (this
// kernel).  A
// reflector with tau = 0 is the identity: its row of W2 is zero (its
// right-hand side is set to zero and its row and column of the block are
// left out).
constexpr int RB = APPLYU_RB;
__global__ __launch_bounds__(256) void k_wy_solve(const Prob* __restrict__ probs, int q, int h) {
  __shared__ double Us[NB][NB + 1];
  __shared__ int zero[NB];
  const Prob& P = probs[blockIdx.z];
  const int N = P.N;
  const int nrefl = N - 1 - refl_off(P);
  const int jb = q * RB;
  if (jb >= nrefl) return;   // uniform
  if ((long)blockIdx.x * blockDim.x >= N) return;   // uniform
  const int nbk = min(RB, nrefl - jb);
  const int off = NB * h;    // first reflector of this half inside the block
  if (off >= nbk) return;    // uniform: the block has no second half
  const int nsub = min(NB, nbk - off);
  const int j0 = jb + off;
  const BSE_CONST double* __restrict__ S = ro(P.S);
  const BSE_CONST double* __restrict__ tau = ro(P.tau);
  if (threadIdx.x < NB) {
    const int i = threadIdx.x;
    zero[i] = (i >= nsub) || (tau[j0 + i] == 0.0);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int r = idx & 63, c = idx >> 6;
    double v;
    if (r == c) v = zero[r] ? 1.0 : tau[j0 + r];   // the reciprocal of T^{-1}'s diagonal 1/tau
    else if (r < c && !zero[r] && !zero[c]) v = S[(off + r) + (long)(off + c) * RB];
    else v = 0.0;
    Us[c][r] = v;
  }
  __syncthreads();
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const BSE_GLOBAL double* __restrict__ w1 = gbl(P.W1) + off + j * RB;
  BSE_GLOBAL double* __restrict__ w2 = gbl(P.W2) + off + j * RB;
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = zero[i] ? 0.0 : w1[i];
  upper_solve64(Us, x);
#pragma unroll
  for (int i = 0; i < NB; ++i) w2[i] = x[i];
  if (P.prec == BSE_PREC_FP32_REFINE) {   // operand of the FP32 update of Z
    BSE_GLOBAL float* __restrict__ w2f = gbl(P.W2f) + off + j * RB;
#pragma unroll
    for (int i = 0; i < NB; ++i) w2f[i] = (float)x[i];
  }
}

}  // namespace

int trsm_rows_batched(hipStream_t s, const Batch& b, int nact, int sel, int k0) {
  if (nact <= 0) return 0;
  const long rows = (long)(sel == 0 ? b.host[0].N : b.host[0].n) - k0 - NB;
  if (rows <= 0) return 0;
  const dim3 g((unsigned)((rows + NB - 1) / NB), 1, (unsigned)nact);
  BSE_LAUNCH(k_trsm_rows<true>, g, NB, 0, s, b.dev, sel, k0);
  BSE_LAUNCH(k_trsm_rows<false>, g, NB, 0, s, b.dev, sel, k0);
  return 0;
}

int trsm_cols_batched(hipStream_t s, const Batch& b, int nact, int b0) {
  if (nact <= 0) return 0;
  const long N0 = b.maxN();
  const dim3 g((unsigned)((N0 + NB - 1) / NB), 1, (unsigned)nact);
  BSE_LAUNCH(k_trsm_cols<true>, g, NB, 0, s, b.dev, b0);
  BSE_LAUNCH(k_trsm_cols<false>, g, NB, 0, s, b.dev, b0);
  return 0;
}

int wy_solve_batched(hipStream_t s, const Batch& b, int nact, int q, int h) {
  if (nact <= 0) return 0;
  const long N0 = b.maxN();
  BSE_LAUNCH(k_wy_solve, dim3((unsigned)((N0 + 255) / 256), 1, (unsigned)nact), 256, 0, s, b.dev, q, h);
  return 0;
}

}  // namespace bse
