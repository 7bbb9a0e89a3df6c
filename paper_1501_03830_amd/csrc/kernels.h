// Host-side launchers of the gfx950 kernels.  Every launcher returns 0 or a
// BSE_* error code and enqueues work on the given stream only.
//
// Launchers work on a Batch: problems sorted by decreasing order N and
// described by Prob records that live in device memory.  A launch serves
// every problem that still has work at that step -- always a prefix of the
// sorted batch -- with the problem number in blockIdx.z; workgroups beyond
// their own problem's extent exit at once.  A single solve is a batch of one.
#pragma once

#include "common.h"

namespace bse {

// ---------------------------------------------------------------- batches
struct Batch {
  int count = 0;
  const Prob* host = nullptr;  // host mirror, sorted by decreasing N
  const Prob* dev = nullptr;   // device copy
  // device scratch of SKTRD_NB rows of 2 (count + 1) ints: the workgroup
  // prefixes of one panel's launches, which let a batch's reduction kernels
  // run without empty workgroups
  int* wgpre = nullptr;
  int maxN() const { return count ? host[0].N : 0; }
  int maxn() const { return count ? host[0].n : 0; }
  // number of problems (a prefix) whose N exceeds x
  int active_N_above(long x) const {
    int k = 0;
    while (k < count && host[k].N > x) ++k;
    return k;
  }
};

// ---------------------------------------------------------------- gemm.hip
struct GemmParams {
  int M, N, K;
  const double* A;
  long lda;
  const double* B;
  long ldb;
  double* C;
  long ldc;
  double alpha, beta;
  int c_uplo, a_tri, b_tri;
  int ta, tb;
  int tiles_m, tiles_n;
  long ntiles;
  int splits, kchunk;
  double* part;  // split-K partial products [splits][M x N], ld M
  float* Cf;     // C in FP32 (when non-null C is unused), ld ldc
  // FP32 products (f32 != 0): operands Af, Bf in FP32 (A, B unused), FP32
  // matrix cores, C = alpha A B + beta Cin (Cin FP64, C when null) or Cf
  int f32;
  const float* Af;
  const float* Bf;
  const double* Cin;
  // Band of the reorthogonalisation's Gram matrix (band_lam non-null): C row
  // r belongs to eigenvalue band_r0 + r; a tile whose rows' first eigenvalue
  // exceeds the last eigenvalue of its columns (band_c0 + column, or the
  // fixed index band_cfix >= 0 for products whose K runs over eigenvalues)
  // by more than REORTH_BAND * band_scal[1] holds only zeros and is skipped.
  const double* band_lam;
  const double* band_scal;
  int band_r0, band_c0, band_cfix, band_n;
};

// Eigenvalue pairs farther apart than this fraction of ||T_s||_1 are left
// out of the reorthogonalisation: inverse iteration leaves such vectors
// orthogonal to about eps / (5 REORTH_BAND) already (measured: 4.6e-15 at
// this distance on the benchmark kernel and on the Clement matrix), and the
// Gram matrix with those entries dropped has a Cholesky factor without fill
// outside the band.
constexpr double REORTH_BAND = 0.01;

// Reflectors per block of the back-transformation with U (four 64-row
// sub-blocks of the compact-WY factor).
constexpr int APPLYU_RB = 256;
constexpr int APPLYU_SUB = APPLYU_RB / 64;   // 64-row sub-blocks per reflector block

// Columns per panel of the skew tridiagonalisation (the batch header keeps
// the workgroup prefixes of a whole panel).
constexpr int SKTRD_NB = 64;

// Columns per panel of the blocked Cholesky factorisations: the panel is
// factored in 64-column sub-panels, and the trailing update after it is one
// product with K = CHOL_PANEL.
constexpr int CHOL_PANEL = 256;

// The products of the chain, as functions of (problem, step).
enum GemmOp {
  GOP_NONE = 0,
  GOP_POTRF_SYRK,  // Cholesky of M: trailing update after the panel at `step`
  GOP_GRAM_SYRK,   // Cholesky of the Gram matrix: trailing update
  GOP_POTRF_PANEL, // Cholesky of M: sub-panel h of the panel at k0 (step = k0 + h)
  GOP_GRAM_PANEL,  // Cholesky of the Gram matrix: the same
  GOP_FORMW_C,     // L11^T L21
  GOP_FORMW_21,    // -L22^T L11
  GOP_SKTRD_R2K,   // skew rank-2k update after the panel starting at column `step`
  GOP_GRAM,        // Gram matrix of the inverse-iteration vectors
  GOP_GRAM_UPD,    // forward substitution: rows below the 128-row block at `step`
  GOP_GRAM_UPD_PANEL,  // forward substitution: second half of the block at `step`
  GOP_APPLYU_S,    // V^T V of reflector block `step`
  GOP_APPLYU_W1,   // V^T Z
  GOP_APPLYU_WB,   // block solve with T^{-1}: sub-block h -= S_h,>h (later rows); step APPLYU_SUB q + h
  GOP_APPLYU_Z,    // Z -= V (T V^T Z)
  GOP_APPLY_L,     // G = L Z
  GOP_REF_Y,       // refinement: Y = L Ub (basis Ub of sweep `step`; L lower triangular)
  GOP_REF_C,       // refinement: C = Y[0:n]^T Y[n:N], so that Ub^T W Ub = C - C^T
  GOP_REF_G,       // refinement: G = Ub^T Ub (lower)
  GOP_REF_U,       // refinement: next basis = Ub + Ub F (the product in FP32)
  // two-stage reduction, panel at column `step` (rows r0 = step + SBR_B ..):
  GOP_SBR_X,       // X = L22 Vp (L22 the strict lower part of the trailing block)
  GOP_SBR_XT,      // X -= L22^T Vp
  GOP_SBR_S,       // S = Vp^T Vp
  GOP_SBR_Y,       // Y = X T
  GOP_SBR_Z,       // Z = Vp^T Y
  GOP_SBR_S2,      // S2 = T^T Z
  GOP_SBR_YY,      // Y <- Y - (1/2) Vp S2
  GOP_SBR_R2K,     // W22 += [Vp Y][Y -Vp]^T (full block)
};

// Refinement products, which read the problem's refinement state (the sweep
// it converged in) to skip finished problems; no other product reads it.
__host__ __device__ constexpr bool is_refine_op(int op) { return op >= GOP_REF_Y && op <= GOP_REF_U; }

// Bandwidth of the two-stage reduction's band (the panel width of its first
// stage).
constexpr int SBR_B = 64;
// Row offset of the reflectors the block back-transformation applies:
// reflector k acts on rows k + off .. N-1 (and N - 1 - off of them are
// stored), off = 1 after the one-stage reduction, SBR_B for the band
// reduction of the two-stage one.
__host__ __device__ inline int refl_off(const Prob& P) { return P.uoff > 1 ? P.uoff : 1; }
__host__ __device__ GemmParams gemm_params(int op, const Prob& P, int step);
// Product `op` at `step` for the first nact problems of the batch.
int gemm_batched(hipStream_t s, const Batch& b, int nact, int op, int step);

// ---------------------------------------------------------------- chol.hip
// M into P.L (ld P.ld) from the lower triangles of A and B
int build_M_batched(hipStream_t s, const Batch& b);
// Blocked Cholesky of the lower triangle.  sel 0: M (order N, in P.L, ld
// P.ld); sel 1: the Gram matrix (order n, in P.inv, ld n).  The first failing
// leading minor goes to P.info[sel] (0 = success); with reset_info false a
// failure recorded earlier is kept.
int potrf_batched(hipStream_t s, const Batch& b, int sel, bool reset_info);
// W = L^T J L into P.W: lower triangle and the W22 = 0 block; `full` also
// fills the strict upper triangle with -W^T.
int form_W_batched(hipStream_t s, const Batch& b, bool full);
// plain copies for the stage entry points
int copy_matrix(hipStream_t s, int m, int n, const double* src, long lds, double* dst, long ldd);
int zero_upper(hipStream_t s, int N, double* A, long lda);

// ---------------------------------------------------------------- trsm.hip
// Cholesky panel of matrix sel (0: M, 1: Gram): rows below the diagonal block
// at k0 <- themselves times L_kk^{-T} (first nact problems)
int trsm_rows_batched(hipStream_t s, const Batch& b, int nact, int sel, int k0);
// rows b0 .. b0+63 of V_+^T <- L_bb^{-1} times themselves (Gram factor)
int trsm_cols_batched(hipStream_t s, const Batch& b, int nact, int b0);
// Rows 64h .. 64h+63 of P.W2 <- solve with the diagonal block h of
// T^{-1} = diag(1/tau) + strict_upper(V^T V) of reflector block q
// (APPLYU_RB reflectors, S = V^T V in P.S); the right-hand side is the same
// rows of P.W1
int wy_solve_batched(hipStream_t s, const Batch& b, int nact, int q, int h);

// ---------------------------------------------------------------- sktrd.hip
size_t sktrd_work_bytes(long N, long ld);
void sktrd_bind_work(char* base, long N, long ld, Prob* P);
// Optional per-launch timing of the skew matvec (event pairs from a pool).
struct KernelTimer {
  hipEvent_t* ev = nullptr;
  int cap = 0;    // number of events in the pool
  int used = 0;   // events recorded so far (pairs)
  double bytes = 0.0;
};
// W = U T U^T in place: alpha (N-1), tau (N-1), reflectors below the
// subdiagonal of P.W.
int sktrd_batched(hipStream_t s, const Batch& b, KernelTimer* timer);
// Tile table of the skew matvec (2 x 9 ints: thresholds t0..t3 and tile
// counts v0..v4, FP64 then FP32): read, replace (host copy, validated), and
// copy to the current device.
int tile_table_get(int* tab);
int tile_table_set(const int* tab);
int tile_table_upload();

// ---------------------------------------------------------------- sbr.hip
// Two-stage skew tridiagonalisation of P.W (strict lower triangle, zero
// upper triangle) for a batch of one: dense to band of width SBR_B (panel
// Householder QR, MFMA two-sided updates), then band to tridiagonal by bulge
// chasing (one persistent launch).  alpha as sktrd_batched.  `work` holds
// the chase's progress words and error flags (device, N + 4 + 128 ints).
// With `vectors` both stages' reflectors are kept for sbr_q2_apply and the
// block back-transformation: the band reduction's below the band in P.W (as
// the one-stage ones, at row offset SBR_B), the chase's in P.W's upper
// triangle (reflector (s, t) in row s, from column s + 1 + SBR_B t on).
int sbr_single(hipStream_t s, const Batch& b, int* work, bool vectors);
// Z <- Q2 Z for the chase's reflectors (Q2 their product in the order they
// were made), on P.Z (N x N, ld); uses P.inv for the compact-WY factors.
int sbr_q2_apply(hipStream_t s, const Batch& b);
// bytes of P.inv that sbr_q2_apply needs for an order-N problem
size_t sbr_q2_T_bytes(long N);

// ---------------------------------------------------------------- stein.hip
// positive eigenvalues of tridiag(alpha, 0, alpha) into P.lambda
int bisect_batched(hipStream_t s, const Batch& b);
// eigenvectors by inverse iteration into P.Vt (n x N, ld n)
int invit_batched(hipStream_t s, const Batch& b);
// Gram-Schmidt inside clusters; failures go to P.info[1].  The FP64 path
// groups eigenvalues closer than 1e-3 ||T_s||_1 and always runs it.  The
// mixed path, whose refinement orthogonalises the basis anyway, only needs it
// for near-degenerate clusters (closer than 1e-10 ||T_s||_1): a problem
// without one skips it.  dflags (device, per slot, P.reorth points into it)
// and hflags (pinned host) carry that decision.
int reorth_batched(hipStream_t s, const Batch& b, const int* dflags, int* hflags, int nslots);
int transpose_to(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst, long ldd);

// ---------------------------------------------------------------- backtr.hip
size_t backtr_work_bytes(long N, long ld);
void backtr_bind_work(char* base, long N, long ld, Prob* P);
// P.Z = U D V_+ as [Re | Im]
int apply_UD_batched(hipStream_t s, const Batch& b);
// P.X from G = L Z (in P.W, made by GOP_APPLY_L), canonical phase and the
// weights
int finish_batched(hipStream_t s, const Batch& b);
// Real problems (a batch of one with FLAG_REAL_IN): after finish_batched,
// makes every column of X real (a real basis inside groups of equal
// eigenvalues, then the canonical sign and the weights again) and writes
// the real parts to P.Xr.  Synchronises the stream.
int real_output_single(hipStream_t s, const Batch& b);
// lower triangle of P.W into P.W32 (mixed-precision path)
int to_f32_batched(hipStream_t s, const Batch& b);

// ---------------------------------------------------------------- refine.hip
// Refinement of the eigenpairs against the FP64 W (mixed-precision path).
// Reads the basis from P.Z, leaves refined eigenvectors in P.Z, eigenvalues
// ascending in P.lambda and the output order in P.perm.  The batch header's
// per-slot state words and correction maxima (device) are copied to pinned
// host arrays after each sweep to decide whether to go on.
struct RefineIO {
  const int* dstate;      // device, nslots (P.refstate points into it)
  const double* dout;     // device, 2 per slot (P.refout points into it)
  int* hstate;            // pinned host copies
  double* hout;
  int nslots;
};
struct RefineStats {
  int sweeps = 0;
  double first_correction = 0.0;
  double last_correction = 0.0;
};
int refine_batched(hipStream_t s, const Batch& b, const RefineIO& io, RefineStats* st);
// The refined eigenvalues, from the final basis in Z and G = L Z in P.W (after
// L is applied), sorted (P.lambda, P.perm).
int refine_final_batched(hipStream_t s, const Batch& b);

}  // namespace bse
