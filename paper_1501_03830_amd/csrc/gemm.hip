// FP64 matrix multiply on the gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
//   C = alpha * op(A) * op(B) + beta * C      (column-major)
//
// Used for every dense contraction of the chain: the Cholesky trailing
// update, W = L^T J L, the skew rank-2k update of the tridiagonalisation,
// the block-reflector applications, the products with L and the Gram
// matrices of the reorthogonalisation.  Options:
//   c_uplo  0: full C;  1: lower triangle incl. diagonal;  2: strictly lower;
//           3: lower triangle incl. diagonal of a tall C (all tiles visited)
//           (only tiles touching the requested triangle are launched)
//   a_tri   the stored A is lower triangular: the K loop skips its zeros
//   b_tri   the stored B is lower triangular
//
// Batched form: the operands of every product in the chain are a function of
// the problem (Prob) and a step index (panel, block ...), so a launch passes
// an operation code and the step; each workgroup derives its problem's
// parameters itself (gemm_params) and the launch covers all problems of a
// batch (blockIdx.z).  Workgroups beyond a problem's own tile count exit.
//
// Tiling: a 256-thread workgroup (4 wavefronts in a 2 x 2 arrangement) owns a
// 64 x 64 C tile (each wave 2 x 2 MFMA blocks of 16 x 16); K steps of 16 are
// staged through LDS with a register prefetch of the next slab.  The epilogue
// goes through LDS so that C is read and written a whole column (64
// consecutive doubles) per instruction.  Products with few output tiles and a
// long K (V^T Z in the reflector application) are split along K into the
// problem's scratch buffer and summed by a second kernel.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "driver.h"

namespace bse {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;
constexpr int F32_TILE = 128;   // tile edge of the FP32 products

}  // namespace

// Parameters of product `op` at `step` for problem P (host and device).
__host__ __device__ GemmParams gemm_params(int op, const Prob& P, int step) {
  GemmParams g{};
  g.alpha = 1.0;
  g.beta = 0.0;
  const long ld = P.ld;
  const int NB = 64;
  switch (op) {
    case GOP_POTRF_PANEL:
    case GOP_GRAM_PANEL: {
      // sub-panel h >= 1 of the panel at k0 (step = k0 + h), brought up to
      // date with the sub-panels before it in the same panel (left-looking):
      // A[kh:, kh:kh+64] -= A[kh:, k0:kh] A[kh:kh+64, k0:kh]^T with
      // kh = k0 + 64 h (lower triangle of the diagonal block, all of the
      // rows below it)
      const bool gram = (op == GOP_GRAM_PANEL);
      double* Mx = gram ? P.inv : P.L;
      const int Nm = gram ? P.n : P.N;
      const long ldm = gram ? (long)P.n : ld;
      const int h = step & (NB - 1);
      const int k0 = step - h;
      const int kh = k0 + NB * h;
      const int rest = Nm - kh;
      if (h <= 0 || rest <= 0) break;
      double* a21 = Mx + kh + (long)k0 * ldm;
      g.ta = 0; g.tb = 1; g.M = rest; g.N = rest < NB ? rest : NB; g.K = NB * h; g.alpha = -1.0; g.beta = 1.0;
      g.A = a21; g.lda = ldm; g.B = a21; g.ldb = ldm;
      g.C = Mx + kh + (long)kh * ldm; g.ldc = ldm; g.c_uplo = 3;
      if (gram) {
        g.band_lam = P.lambda; g.band_scal = P.scal; g.band_r0 = g.band_c0 = kh; g.band_cfix = -1; g.band_n = P.n;
      }
      break;
    }
    case GOP_POTRF_SYRK:
    case GOP_GRAM_SYRK: {
      // trailing update after the CHOL_PANEL-column panel at `step` (the
      // panel itself is solved by k_potf2, trsm_rows_batched and the
      // sub-panel products): A22 -= A21 A21^T, lower triangle
      const bool gram = (op == GOP_GRAM_SYRK);
      double* Mx = gram ? P.inv : P.L;
      const int Nm = gram ? P.n : P.N;
      const long ldm = gram ? (long)P.n : ld;
      const int k0 = step;
      const int nbk = (Nm - k0 < CHOL_PANEL) ? Nm - k0 : CHOL_PANEL;
      const int rest = Nm - k0 - nbk;
      if (nbk <= 0 || rest <= 0) break;  // M = N = 0: nothing to do
      double* a21 = Mx + (k0 + nbk) + (long)k0 * ldm;
      g.ta = 0; g.tb = 1; g.M = rest; g.N = rest; g.K = nbk; g.alpha = -1.0; g.beta = 1.0;
      g.A = a21; g.lda = ldm; g.B = a21; g.ldb = ldm;
      g.C = Mx + (k0 + nbk) + (long)(k0 + nbk) * ldm; g.ldc = ldm; g.c_uplo = 1;
      if (gram) {
        g.band_lam = P.lambda; g.band_scal = P.scal; g.band_r0 = g.band_c0 = k0 + nbk; g.band_cfix = -1; g.band_n = P.n;
      }
      break;
    }
    case GOP_FORMW_C:   // W11 <- L11^T L21
      g.ta = 1; g.tb = 0; g.M = P.n; g.N = P.n; g.K = P.n;
      g.A = P.L; g.lda = ld; g.B = P.L + P.n; g.ldb = ld; g.C = P.W; g.ldc = ld; g.a_tri = 1;
      break;
    case GOP_FORMW_21:  // W21 <- -L22^T L11
      g.ta = 1; g.tb = 0; g.M = P.n; g.N = P.n; g.K = P.n; g.alpha = -1.0;
      g.A = P.L + P.n + (long)P.n * ld; g.lda = ld; g.B = P.L; g.ldb = ld; g.C = P.W + P.n; g.ldc = ld;
      g.a_tri = 1; g.b_tri = 1;
      break;
    case GOP_SKTRD_R2K: {  // trailing W += [v p ...][p -v ...]^T after the panel at `step`
      const int k0 = step;
      if (k0 > P.N - 2) break;
      const int nbp = (P.N - 1 - k0 < NB) ? P.N - 1 - k0 : NB;
      const int e = k0 + nbp;
      const int m2 = P.N - e;
      if (m2 < 2 || e > P.N - 2) break;
      g.ta = 0; g.tb = 1; g.M = m2; g.N = m2; g.K = 2 * nbp; g.beta = 1.0;
      g.A = P.Y1 + e; g.lda = ld; g.B = P.Y2 + e; g.ldb = ld; g.C = P.W + e + (long)e * ld; g.ldc = ld;
      g.c_uplo = 2;
      if (P.prec == BSE_PREC_FP32_REFINE) {
        // W held in FP32: the product on the FP32 matrix cores from FP32
        // copies of the panel vectors (k_y_to_f32), accumulated in FP32
        g.C = nullptr;
        g.Cf = P.W32 + e + (long)e * ld;
        g.f32 = 1;
        g.A = nullptr;
        g.B = nullptr;
        g.Af = P.Y1f + e;
        g.Bf = P.Y2f + e;
      }
      break;
    }
    case GOP_GRAM:  // G <- Vt Vt^T (lower)
      g.ta = 0; g.tb = 1; g.M = P.n; g.N = P.n; g.K = P.N;
      g.A = P.Vt; g.lda = P.n; g.B = P.Vt; g.ldb = P.n; g.C = P.inv; g.ldc = P.n; g.c_uplo = 1;
      g.band_lam = P.lambda; g.band_scal = P.scal; g.band_r0 = g.band_c0 = 0; g.band_cfix = -1; g.band_n = P.n;
      break;
    case GOP_GRAM_UPD_PANEL: {  // rows b0+64..b0+127 -= L[.., b0:b0+64] (rows b0..b0+63)
      const int b0 = step;
      const int rest = P.n - b0 - NB;
      if (rest <= 0) break;
      g.ta = 0; g.tb = 0; g.M = rest < NB ? rest : NB; g.N = P.N; g.K = NB; g.alpha = -1.0; g.beta = 1.0;
      g.A = P.inv + (b0 + NB) + (long)b0 * P.n; g.lda = P.n; g.B = P.Vt + b0; g.ldb = P.n;
      g.C = P.Vt + b0 + NB; g.ldc = P.n;
      g.band_lam = P.lambda; g.band_scal = P.scal; g.band_r0 = b0 + NB; g.band_cfix = b0 + NB - 1; g.band_n = P.n;
      break;
    }
    case GOP_GRAM_UPD: {  // rows below the 128-row block -= L21 (rows of the block)
      const int b0 = step;
      if (b0 >= P.n) break;
      const int nbk = (P.n - b0 < 2 * NB) ? P.n - b0 : 2 * NB;
      const int rest = P.n - b0 - nbk;
      if (rest <= 0) break;
      g.ta = 0; g.tb = 0; g.M = rest; g.N = P.N; g.K = nbk; g.alpha = -1.0; g.beta = 1.0;
      g.A = P.inv + (b0 + nbk) + (long)b0 * P.n; g.lda = P.n; g.B = P.Vt + b0; g.ldb = P.n;
      g.C = P.Vt + b0 + nbk; g.ldc = P.n;
      g.band_lam = P.lambda; g.band_scal = P.scal; g.band_r0 = b0 + nbk; g.band_cfix = b0 + nbk - 1; g.band_n = P.n;
      break;
    }
    case GOP_APPLYU_S:
    case GOP_APPLYU_W1:
    case GOP_APPLYU_WB:
    case GOP_APPLYU_Z: {
      // reflector block q of RB (H_j0 .. H_j0+nbk-1, j0 = RB q); the block
      // solve's products carry their sub-block h in step = APPLYU_SUB q + h
      constexpr int RB = APPLYU_RB;
      const int q = (op == GOP_APPLYU_WB) ? step / APPLYU_SUB : step;
      const int h = (op == GOP_APPLYU_WB) ? step % APPLYU_SUB : 0;
      const int o = refl_off(P);   // reflector k acts on rows k + o ..
      const int nrefl = P.N - 1 - o;
      const int j0 = q * RB;
      if (nrefl <= 0 || j0 >= nrefl) break;
      const int nbk = (nrefl - j0 < RB) ? nrefl - j0 : RB;
      const int m = P.N - j0 - o;
      const double* Vb = P.Vb + (j0 + o);
      double* Zs = P.Z + (j0 + o);
      if (op == GOP_APPLYU_S) {         // S = V^T V
        g.ta = 1; g.tb = 0; g.M = nbk; g.N = nbk; g.K = m;
        g.A = Vb; g.lda = ld; g.B = Vb; g.ldb = ld; g.C = P.S; g.ldc = RB;
      } else if (op == GOP_APPLYU_W1) {  // W1 = V^T Z
        g.ta = 1; g.tb = 0; g.M = nbk; g.N = P.N; g.K = m;
        g.A = Vb; g.lda = ld; g.B = Zs; g.ldb = ld; g.C = P.W1; g.ldc = RB;
        if (P.prec == BSE_PREC_FP32_REFINE) {   // FP32 basis, FP32 matrix cores
          g.f32 = 1; g.Af = P.Vb32 + (j0 + o); g.Bf = P.Z32 + (j0 + o);
        }
      } else if (op == GOP_APPLYU_WB) {  // W1[h] -= S[h, h+1:] W2[h+1:] (64-row sub-blocks)
        const int r0 = NB * h, c0 = NB * (h + 1);
        if (c0 >= nbk) break;
        g.ta = 0; g.tb = 0; g.M = NB; g.N = P.N; g.K = nbk - c0; g.alpha = -1.0; g.beta = 1.0;
        g.A = P.S + r0 + (long)c0 * RB; g.lda = RB; g.B = P.W2 + c0; g.ldb = RB; g.C = P.W1 + r0; g.ldc = RB;
      } else {                           // Z -= V W2
        g.ta = 0; g.tb = 0; g.M = m; g.N = P.N; g.K = nbk; g.alpha = -1.0; g.beta = 1.0;
        g.A = Vb; g.lda = ld; g.B = P.W2; g.ldb = RB; g.C = Zs; g.ldc = ld;
        if (P.prec == BSE_PREC_FP32_REFINE) {
          g.f32 = 1; g.Af = P.Vb32 + (j0 + o); g.Bf = P.W2f; g.C = nullptr; g.Cf = P.Z32 + (j0 + o);
        }
      }
      break;
    }
    case GOP_APPLY_L:  // G = L Z into the W buffer
      g.ta = 0; g.tb = 0; g.M = P.N; g.N = P.N; g.K = P.N;
      g.A = P.L; g.lda = ld; g.B = P.Z; g.ldb = ld; g.C = P.W; g.ldc = ld; g.a_tri = 1;
      break;
    case GOP_REF_Y:
    case GOP_REF_C:
    case GOP_REF_G:
    case GOP_REF_U: {
      // the basis of sweep `step` alternates between Z (even) and R4 (odd)
      double* Ub = (step & 1) ? P.R4 : P.Z;
      double* Un = (step & 1) ? P.Z : P.R4;
      g.M = P.N; g.N = P.N; g.K = P.N;
      if (op == GOP_REF_Y) {
        // Y = L Ub (L lower triangular: the K loop skips its zero upper part)
        g.ta = 0; g.tb = 0; g.A = P.L; g.lda = ld; g.B = Ub; g.ldb = ld; g.C = P.R1; g.ldc = ld; g.a_tri = 1;
      } else if (op == GOP_REF_C) {
        // C = Y[0:n]^T Y[n:N] (full): with W = L^T J L, Ub^T W Ub = Y^T J Y = C - C^T
        g.K = P.n;
        g.ta = 1; g.tb = 0; g.A = P.R1; g.lda = ld; g.B = P.R1 + P.n; g.ldb = ld; g.C = P.R2; g.ldc = ld;
      } else if (op == GOP_REF_G) {  // Ub^T Ub, lower triangle
        g.ta = 1; g.tb = 0; g.A = Ub; g.lda = ld; g.B = Ub; g.ldb = ld; g.C = P.R3; g.ldc = ld; g.c_uplo = 1;
      } else {
        // Un = Ub + Ub F: the correction product in FP32 (F and a rounded
        // copy of Ub in R1, see the refinement), the sum in FP64
        const float* F32 = reinterpret_cast<const float*>(P.R1);
        g.f32 = 1; g.ta = 0; g.tb = 0;
        g.Af = F32 + ld * ld; g.lda = ld; g.Bf = F32; g.ldb = ld;
        g.C = Un; g.Cin = Ub; g.ldc = ld; g.beta = 1.0;
      }
      break;
    }
    case GOP_SBR_X:
    case GOP_SBR_XT:
    case GOP_SBR_S:
    case GOP_SBR_Y:
    case GOP_SBR_Z:
    case GOP_SBR_S2:
    case GOP_SBR_YY:
    case GOP_SBR_R2K: {
      // panel of the two-stage reduction at column k0 = step: reflectors of
      // rows r0 = k0 + SBR_B .. N-1, explicit in Vp (P.Vb, ld), T and the
      // small products in P.S (64 x 64 blocks at 0: S, 4096: T, 8192: Z,
      // 12288: S2), X in P.W1 and Y in P.W2 (both ld x 64)
      const int k0 = step;
      const int r0 = k0 + SBR_B;
      const int m = P.N - r0;
      if (m < 2) break;
      const int nr = (m - 1 < SBR_B) ? m - 1 : SBR_B;   // reflectors in the panel
      const int B2 = SBR_B * SBR_B;
      double* Tm = P.S + B2;
      double* Zm = P.S + 2 * B2;
      double* S2 = P.S + 3 * B2;
      double* W22 = P.W + r0 + (long)r0 * ld;
      switch (op) {
        case GOP_SBR_X:    // L22 V (zero upper triangle: triangular A)
          g.ta = 0; g.tb = 0; g.M = m; g.N = nr; g.K = m; g.a_tri = 1;
          g.A = W22; g.lda = ld; g.B = P.Vb; g.ldb = ld; g.C = P.W1; g.ldc = ld;
          break;
        case GOP_SBR_XT:   // - L22^T V
          g.ta = 1; g.tb = 0; g.M = m; g.N = nr; g.K = m; g.a_tri = 1; g.alpha = -1.0; g.beta = 1.0;
          g.A = W22; g.lda = ld; g.B = P.Vb; g.ldb = ld; g.C = P.W1; g.ldc = ld;
          break;
        case GOP_SBR_S:
          g.ta = 1; g.tb = 0; g.M = nr; g.N = nr; g.K = m;
          g.A = P.Vb; g.lda = ld; g.B = P.Vb; g.ldb = ld; g.C = P.S; g.ldc = SBR_B;
          break;
        case GOP_SBR_Y:
          g.ta = 0; g.tb = 0; g.M = m; g.N = nr; g.K = nr;
          g.A = P.W1; g.lda = ld; g.B = Tm; g.ldb = SBR_B; g.C = P.W2; g.ldc = ld;
          break;
        case GOP_SBR_Z:
          g.ta = 1; g.tb = 0; g.M = nr; g.N = nr; g.K = m;
          g.A = P.Vb; g.lda = ld; g.B = P.W2; g.ldb = ld; g.C = Zm; g.ldc = SBR_B;
          break;
        case GOP_SBR_S2:
          g.ta = 1; g.tb = 0; g.M = nr; g.N = nr; g.K = nr;
          g.A = Tm; g.lda = SBR_B; g.B = Zm; g.ldb = SBR_B; g.C = S2; g.ldc = SBR_B;
          break;
        case GOP_SBR_YY:
          g.ta = 0; g.tb = 0; g.M = m; g.N = nr; g.K = nr; g.alpha = -0.5; g.beta = 1.0;
          g.A = P.Vb; g.lda = ld; g.B = S2; g.ldb = SBR_B; g.C = P.W2; g.ldc = ld;
          break;
        default:   // GOP_SBR_R2K, strict lower triangle
          g.ta = 0; g.tb = 1; g.M = m; g.N = m; g.K = 2 * nr; g.beta = 1.0;
          g.A = P.Y1; g.lda = ld; g.B = P.Y2; g.ldb = ld; g.C = W22; g.ldc = ld; g.c_uplo = 2;
          break;
      }
      break;
    }
    default:
      break;
  }
  // tiles and split-K: few output tiles and a long K are split along K into
  // the problem's scratch buffer
  const int tbm = g.f32 ? F32_TILE : BM, tbn = g.f32 ? F32_TILE : BN;
  g.tiles_m = (g.M + tbm - 1) / tbm;
  g.tiles_n = (g.N + tbn - 1) / tbn;
  g.ntiles = (g.M <= 0 || g.N <= 0) ? 0
             : ((g.c_uplo == 1 || g.c_uplo == 2) ? (long)g.tiles_m * (g.tiles_m + 1) / 2 : (long)g.tiles_m * g.tiles_n);
  g.splits = 1;
  g.kchunk = g.K;
  g.part = nullptr;
  if (g.ntiles > 0 && g.ntiles < 1024 && g.K >= 2048 && P.gscr != nullptr) {
    long splits = (2048 + g.ntiles - 1) / g.ntiles;
    if (splits > 16) splits = 16;
    const long maxk = g.K / 512;
    if (splits > maxk) splits = maxk;
    while (splits > 1 && (size_t)splits * g.M * g.N * sizeof(double) > P.gscr_bytes) --splits;
    if (splits > 1) {
      g.splits = (int)splits;
      g.kchunk = (int)(((g.K + splits - 1) / splits + BK - 1) / BK * BK);
      g.part = P.gscr;
    }
  }
  return g;
}

namespace {

// Workgroups are dealt to the 8 XCDs round-robin in dispatch order, and each
// XCD has its own L2.  xcd_remap turns the dispatch index into an index in
// which every XCD owns one contiguous range, so tiles that share A or B
// panels run on the same XCD.
__device__ inline long xcd_remap(long wg, long total) {
  constexpr long NX = 8;
  const long q = total / NX, r = total % NX;
  const long x = wg % NX, local = wg / NX;
  return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// Tile (tm, tn) of a full tile grid in bands of GROUP tile rows, column by
// column inside a band: consecutive tiles share their B panel, and a band's
// A panels stay in L2 while it is swept.
__device__ inline void grouped_tile(long t, int tiles_m, int tiles_n, int& tm, int& tn) {
  constexpr int GROUP = 8;
  const long per_band = (long)GROUP * tiles_n;
  const int band = (int)(t / per_band);
  const int first = band * GROUP;
  const int rows = min(GROUP, tiles_m - first);
  const long in_band = t - (long)band * per_band;
  tm = first + (int)(in_band % rows);
  tn = (int)(in_band / rows);
}

// Tile (R, C), R >= C, of the lower triangle of an nt x nt tile grid, in
// bands of GROUP tile rows: a band holds the columns 0 .. its last row,
// column by column with the band's rows fastest, so consecutive tiles share
// their B panel and a band's A panels stay in L2 while it is swept (row by
// row, every tile row re-read all B panels of its columns).
__device__ inline void grouped_lower_tile(long t, int nt, int& R, int& C) {
  constexpr int GROUP = 8;
  int r0 = 0;
  long before = 0;
  for (;;) {   // at most nt / GROUP bands
    const int g = min(GROUP, nt - r0);
    const long cnt = (long)g * r0 + (long)g * (g + 1) / 2;
    if (t < before + cnt || r0 + g >= nt) break;
    before += cnt;
    r0 += GROUP;
  }
  const int g = min(GROUP, nt - r0);
  long o = t - before;
  if (o < (long)g * r0) {
    C = (int)(o / g);
    R = r0 + (int)(o % g);
    return;
  }
  o -= (long)g * r0;
  int c = 0;
  while (o >= g - c) {
    o -= g - c;
    ++c;
  }
  C = r0 + c;
  R = r0 + c + (int)o;
}

template <bool TA, bool TB, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const Prob* __restrict__ probs, int op, int step,
                                                       GemmParams single) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int AS = BK * (BM + PAD), BS = BK * (BN + PAD);
  constexpr int SMEM = 2 * (AS + BS);
  // the epilogue goes through the same LDS, EC columns at a time
  constexpr int EC0 = SMEM / (BM + 1);
  constexpr int EC = EC0 >= BN ? BN : (EC0 >= 64 ? 64 : 32);
  static_assert(EC * (BM + 1) <= SMEM, "epilogue chunk does not fit");
  __shared__ double smem[SMEM];

  int stp = step;
  if (probs && is_refine_op(op)) {
    // refinement products: skip problems that finished in an earlier sweep;
    // step < 0 means the problem's own final sweep
    const int st = *gbl(probs[blockIdx.z].refstate);
    if (step >= 0 && st != 0 && st <= step) return;
    if (step < 0) stp = st;
  }
  if (probs && (op == GOP_GRAM || op == GOP_GRAM_SYRK || op == GOP_GRAM_PANEL || op == GOP_GRAM_UPD ||
                 op == GOP_GRAM_UPD_PANEL) && *gbl(probs[blockIdx.z].reorth) == 0)
    return;   // no cluster Gram-Schmidt for this problem
  const GemmParams p = probs ? gemm_params(op, probs[blockIdx.z], stp) : single;
  const BSE_GLOBAL double* __restrict__ Ag = gbl(p.A);
  const BSE_GLOBAL double* __restrict__ Bg = gbl(p.B);
  // tiles of this configuration (the host sized the grid for it)
  const int tiles_m = (p.M + BM - 1) / BM, tiles_n = (p.N + BN - 1) / BN;
  const long ntiles = (p.M <= 0 || p.N <= 0) ? 0
                      : ((p.c_uplo == 1 || p.c_uplo == 2) ? (long)tiles_m * (tiles_m + 1) / 2 : (long)tiles_m * tiles_n);
  // With a triangular operand the tiles' K ranges differ.  A triangular A
  // makes K depend on the tile row only: tiles go column by column (rows
  // fastest) and every XCD takes a contiguous range, i.e. whole columns with
  // all their K lengths, and the B panel of a column stays on one XCD.  With
  // a triangular B, K depends on the column, and a contiguous range per XCD
  // would give one XCD all the long tiles, so those products keep the
  // dispatch order (long and short tiles interleaved over the XCDs).
  // The remap covers this problem's own tiles (a batch's grid is sized for
  // its largest problem, and a remap over the whole grid would put all of a
  // small problem's tiles on the first XCDs).
  const bool tri = p.a_tri || p.b_tri;
  const long total = ntiles * p.splits;
  if ((long)blockIdx.x >= total) return;  // uniform: beyond this problem's tiles
  long tile = p.b_tri ? (long)blockIdx.x : xcd_remap(blockIdx.x, total);
  int slice = 0;
  if (p.splits > 1) {
    slice = (int)(tile % p.splits);
    tile /= p.splits;
  }
  int tm, tn;
  if (p.c_uplo == 1 || p.c_uplo == 2) {
    grouped_lower_tile(tile, tiles_m, tm, tn);
  } else if (tri) {
    tm = (int)(tile % tiles_m);
    tn = (int)(tile / tiles_m);
  } else {
    grouped_tile(tile, tiles_m, tiles_n, tm, tn);
  }
  const int i0 = tm * BM, j0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  if (p.band_lam && p.splits == 1) {
    // a tile of the reorthogonalisation's products outside the band is zero
    // and stays zero (uniform)
    const BSE_GLOBAL double* __restrict__ lam = gbl(p.band_lam);
    const int rlo = p.band_r0 + i0;
    const int chi = p.band_cfix >= 0 ? p.band_cfix : min(p.band_c0 + j0 + BN - 1, p.band_n - 1);
    if (rlo < p.band_n && lam[rlo] - lam[chi] > REORTH_BAND * gbl(p.band_scal)[1]) return;
  }

  // K range that can hold non-zero products for this tile
  int kbeg = 0, kend = p.K;
  if (p.a_tri) {
    if (!TA) kend = min(kend, i0 + BM);
    else kbeg = max(kbeg, i0);
  }
  if (p.b_tri) {
    if (!TB) kbeg = max(kbeg, j0);
    else kend = min(kend, j0 + BN);
  }
  kbeg = (kbeg / BK) * BK;
  if (p.splits > 1) {
    const int s0 = slice * p.kchunk;
    kbeg = max(kbeg, s0);
    kend = min(kend, s0 + p.kchunk);
  }

  d4_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};

  // global -> register staging: each thread moves EA (EB) consecutive
  // elements along the contiguous direction of the stored operand
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  double ra[EA], rb[EB];
  auto load_a = [&](int k0) {
    if (!TA) {
      constexpr int TPC = BM / EA;
      const int kk = tid / TPC, ii = (tid % TPC) * EA;
      const int k = k0 + kk;
#pragma unroll
      for (int q = 0; q < EA; ++q) {
        const int i = i0 + ii + q;
        ra[q] = (i < p.M && k < kend) ? Ag[(long)i + (long)k * p.lda] : 0.0;
      }
    } else {
      constexpr int TPC = BK / EA;
      const int ii = tid / TPC, kk = (tid % TPC) * EA;
      const int i = i0 + ii;
#pragma unroll
      for (int q = 0; q < EA; ++q) {
        const int k = k0 + kk + q;
        ra[q] = (i < p.M && k < kend) ? Ag[(long)k + (long)i * p.lda] : 0.0;
      }
    }
  };
  auto store_a = [&](int buf) {
    double* s = smem + buf * AS;
    if (!TA) {
      constexpr int TPC = BM / EA;
      const int kk = tid / TPC, ii = (tid % TPC) * EA;
#pragma unroll
      for (int q = 0; q < EA; ++q) s[kk * (BM + PAD) + ii + q] = ra[q];
    } else {
      constexpr int TPC = BK / EA;
      const int ii = tid / TPC, kk = (tid % TPC) * EA;
#pragma unroll
      for (int q = 0; q < EA; ++q) s[(kk + q) * (BM + PAD) + ii] = ra[q];
    }
  };
  auto load_b = [&](int k0) {
    if (!TB) {
      constexpr int TPC = BK / EB;
      const int jj = tid / TPC, kk = (tid % TPC) * EB;
      const int j = j0 + jj;
#pragma unroll
      for (int q = 0; q < EB; ++q) {
        const int k = k0 + kk + q;
        rb[q] = (j < p.N && k < kend) ? Bg[(long)k + (long)j * p.ldb] : 0.0;
      }
    } else {
      constexpr int TPC = BN / EB;
      const int kk = tid / TPC, jj = (tid % TPC) * EB;
      const int k = k0 + kk;
#pragma unroll
      for (int q = 0; q < EB; ++q) {
        const int j = j0 + jj + q;
        rb[q] = (j < p.N && k < kend) ? Bg[(long)j + (long)k * p.ldb] : 0.0;
      }
    }
  };
  auto store_b = [&](int buf) {
    double* s = smem + 2 * AS + buf * BS;
    if (!TB) {
      constexpr int TPC = BK / EB;
      const int jj = tid / TPC, kk = (tid % TPC) * EB;
#pragma unroll
      for (int q = 0; q < EB; ++q) s[(kk + q) * (BN + PAD) + jj] = rb[q];
    } else {
      constexpr int TPC = BN / EB;
      const int kk = tid / TPC, jj = (tid % TPC) * EB;
#pragma unroll
      for (int q = 0; q < EB; ++q) s[kk * (BN + PAD) + jj + q] = rb[q];
    }
  };

  int buf = 0;
  if (kbeg < kend) {
    load_a(kbeg);
    load_b(kbeg);
    store_a(0);
    store_b(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      load_a(k0 + BK);
      load_b(k0 + BK);
    }
    const double* a_s = smem + buf * AS;
    const double* b_s = smem + 2 * AS + buf * BS;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[FM], bf[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) af[a] = a_s[kr * (BM + PAD) + wr * WM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < FN; ++b) bf[b] = b_s[kr * (BN + PAD) + wc * WN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (more) {
      store_a(buf ^ 1);
      store_b(buf ^ 1);
    }
    __syncthreads();
    buf ^= 1;
  }

  // Epilogue through LDS, EC columns at a time.  In a 16 x 16 f64 block the
  // entry (i, j) lives in lane 16 (i mod 4) + j, accumulator element i / 4.
  // The old C values of 8 elements per thread are loaded before any of them
  // is stored: the compiler cannot move a load of C above a store to C, so
  // the element loop made one round trip per element (a few percent of the
  // K = 128 updates).  Batches of 8 keep the register count, and so the
  // occupancy, of the main loop.
  double* Cs = smem;  // Cs[(c - c0) * (BM + 1) + r]
  const bool split = p.splits > 1;
  const bool read_c = !split && p.beta != 0.0;
  constexpr int PER = 8, NBAT = EC * BM / (256 * PER);
  static_assert(NBAT * 256 * PER == EC * BM, "epilogue chunk is not a whole number of batches");
#pragma unroll
  for (int c0 = 0; c0 < BN; c0 += EC) {
    __syncthreads();
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int cl = wc * WN + b * 16 + (lane & 15);
        if (cl < c0 || cl >= c0 + EC) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rl = wr * WM + a * 16 + (lane >> 4) + 4 * v;
          Cs[(cl - c0) * (BM + 1) + rl] = acc[a][b][v];
        }
      }
    __syncthreads();
    if (p.Cf && !split) {
      // FP32 C (the rank-2k update of the FP32 copy of W): the chunk's old
      // values in one batch, kept in FP32 (as many registers as 8 doubles)
      constexpr int PF = 2 * PER, NBF = EC * BM / (256 * PF);
      static_assert(NBF * 256 * PF == EC * BM, "epilogue chunk is not a whole number of batches");
#pragma unroll
      for (int h = 0; h < NBF; ++h) {
        bool ok[PF];
        float cold[PF];
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int idx = tid + 256 * (h * PF + u);
          const int rl = idx % BM, cl = c0 + idx / BM;
          const int row = i0 + rl, col = j0 + cl;
          ok[u] = row < p.M && col < p.N && !((p.c_uplo == 1 || p.c_uplo == 3) && row < col) &&
                  !(p.c_uplo == 2 && row <= col);
          cold[u] = 0.0f;
          if (ok[u] && read_c) cold[u] = gbl(p.Cf)[(long)row + (long)col * p.ldc];
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          if (!ok[u]) continue;
          const int idx = tid + 256 * (h * PF + u);
          const int rl = idx % BM, cl = c0 + idx / BM;
          const int row = i0 + rl, col = j0 + cl;
          const double out = p.alpha * Cs[(cl - c0) * (BM + 1) + rl];
          const double res = read_c ? out + p.beta * (double)cold[u] : out;
          gbl(p.Cf)[(long)row + (long)col * p.ldc] = (float)res;
        }
      }
      continue;
    }
#pragma unroll
    for (int h = 0; h < NBAT; ++h) {
      bool ok[PER];
      double cold[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + 256 * (h * PER + u);
        const int rl = idx % BM, cl = c0 + idx / BM;
        const int row = i0 + rl, col = j0 + cl;
        ok[u] = row < p.M && col < p.N && !((p.c_uplo == 1 || p.c_uplo == 3) && row < col) &&
                !(p.c_uplo == 2 && row <= col);
        cold[u] = 0.0;
        if (ok[u] && read_c) {
          const long o = (long)row + (long)col * p.ldc;
          cold[u] = p.Cf ? (double)gbl(p.Cf)[o] : gbl(p.C)[o];
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        if (!ok[u]) continue;
        const int idx = tid + 256 * (h * PER + u);
        const int rl = idx % BM, cl = c0 + idx / BM;
        const int row = i0 + rl, col = j0 + cl;
        const double val = Cs[(cl - c0) * (BM + 1) + rl];
        const double out = p.alpha * val;
        const double res = read_c ? out + p.beta * cold[u] : out;
        const long o = (long)row + (long)col * p.ldc;
        if (split) gbl(p.part)[(long)slice * p.M * p.N + (long)row + (long)col * p.M] = val;
        else if (p.Cf) gbl(p.Cf)[o] = (float)res;
        else gbl(p.C)[o] = res;
      }
    }
  }
}

typedef float f4_t __attribute__((ext_vector_type(4)));

// FP32 products on the FP32 matrix cores: 128 x 128 tiles, K steps of 16,
// four waves of 64 x 64 outputs, each 4 x 4 blocks of v_mfma_f32_16x16x4f32.
// (FP32 operands are half the bytes of FP64 ones at over twice the matrix
// rate, so a tile needs four times the FP64 tile's reuse to stay off the
// memory bound.)  In a 16 x 16 f32 block the entry (i, j) lives in lane
// j + 16 (i / 4), accumulator element i mod 4; the f64 instruction
// interleaves the rows the other way.  Full outputs, or the lower
// (c_uplo 1) or strictly lower (c_uplo 2) triangle of a square one in
// triangular tile order; B transposed or not.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const Prob* __restrict__ probs, int op, int step,
                                                       GemmParams single) {
  constexpr int TBM = F32_TILE, TBN = F32_TILE, TBK = 16;
  // row pitch of 144 floats: the four K rows read by one MFMA operand fetch
  // fall 16 banks apart
  constexpr int LA = TBM + 16, LB = TBN + 16;
  constexpr int AS = TBK * LA, BS = TBK * LB;
  constexpr int WM = 64, WN = 64, FM = 4, FN = 4;
  constexpr int EC = 64;   // epilogue columns per pass through LDS
  static_assert(EC * (TBM + 1) <= 2 * (AS + BS), "epilogue chunk does not fit");
  __shared__ float smem[2 * (AS + BS)];
  int stp = step;
  if (probs && is_refine_op(op)) {
    const int st = *gbl(probs[blockIdx.z].refstate);
    if (step >= 0 && st != 0 && st <= step) return;
    if (step < 0) stp = st;
  }
  const GemmParams p = probs ? gemm_params(op, probs[blockIdx.z], stp) : single;
  const BSE_GLOBAL float* __restrict__ Ag = gbl(p.Af);
  const BSE_GLOBAL float* __restrict__ Bg = gbl(p.Bf);
  const int tiles_m = (p.M + TBM - 1) / TBM, tiles_n = (p.N + TBN - 1) / TBN;
  const bool tri_c = p.c_uplo == 1 || p.c_uplo == 2;
  const long ntiles = (p.M <= 0 || p.N <= 0) ? 0 : (tri_c ? (long)tiles_m * (tiles_m + 1) / 2 : (long)tiles_m * tiles_n);
  // remap over this problem's own tiles (see the FP64 kernel)
  const long total = ntiles * p.splits;
  if ((long)blockIdx.x >= total) return;  // uniform: beyond this problem's tiles
  long tile = xcd_remap(blockIdx.x, total);
  int slice = 0;
  if (p.splits > 1) {
    slice = (int)(tile % p.splits);
    tile /= p.splits;
  }
  int tm, tn;
  if (tri_c) grouped_lower_tile(tile, tiles_m, tm, tn);
  else grouped_tile(tile, tiles_m, tiles_n, tm, tn);
  const int i0 = tm * TBM, j0 = tn * TBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  // output entries kept: all, the lower triangle, or the strictly lower one
  auto in_c = [&](int row, int col) {
    return row < p.M && col < p.N && (p.c_uplo != 1 || row >= col) && (p.c_uplo != 2 || row > col);
  };
  int kbeg = 0, kend = p.K;
  if (p.splits > 1) {
    const int s0 = slice * p.kchunk;
    kbeg = max(kbeg, s0);
    kend = min(kend, s0 + p.kchunk);
  }

  f4_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};

  // staging: 8 elements of A and 8 of B per thread and K step, the lanes of
  // each load running along the operand's contiguous direction
  constexpr int E = TBM * TBK / 256;
  float ra[E], rb[E];
  auto load_a = [&](int k0) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      int i, k;
      if (!TA) {
        i = i0 + (tid & 127);
        k = k0 + (tid >> 7) + 2 * q;
      } else {
        k = k0 + (tid & 15);
        i = i0 + (tid >> 4) + 16 * q;
      }
      ra[q] = (i < p.M && k < kend) ? (TA ? Ag[(long)k + (long)i * p.lda] : Ag[(long)i + (long)k * p.lda]) : 0.0f;
    }
  };
  auto store_a = [&](int buf) {
    float* sa = smem + buf * AS;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      if (!TA) sa[((tid >> 7) + 2 * q) * LA + (tid & 127)] = ra[q];
      else sa[(tid & 15) * LA + (tid >> 4) + 16 * q] = ra[q];
    }
  };
  auto load_b = [&](int k0) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      int j, k;
      if (!TB) {
        k = k0 + (tid & 15);
        j = j0 + (tid >> 4) + 16 * q;
      } else {   // B stored N x K: the lanes run along j
        j = j0 + (tid & 127);
        k = k0 + (tid >> 7) + 2 * q;
      }
      rb[q] = (j < p.N && k < kend) ? (TB ? Bg[(long)j + (long)k * p.ldb] : Bg[(long)k + (long)j * p.ldb]) : 0.0f;
    }
  };
  auto store_b = [&](int buf) {
    float* sb = smem + 2 * AS + buf * BS;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      if (!TB) sb[(tid & 15) * LB + (tid >> 4) + 16 * q] = rb[q];
      else sb[((tid >> 7) + 2 * q) * LB + (tid & 127)] = rb[q];
    }
  };

  int buf = 0;
  if (kbeg < kend) {
    load_a(kbeg);
    load_b(kbeg);
    store_a(0);
    store_b(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += TBK) {
    const bool more = k0 + TBK < kend;
    if (more) {
      load_a(k0 + TBK);
      load_b(k0 + TBK);
    }
    const float* a_s = smem + buf * AS;
    const float* b_s = smem + 2 * AS + buf * BS;
#pragma unroll
    for (int ks = 0; ks < TBK; ks += 4) {
      const int kr = ks + (lane >> 4);
      float af[FM], bf[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) af[a] = a_s[kr * LA + wr * WM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < FN; ++b) bf[b] = b_s[kr * LB + wc * WN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (more) {
      store_a(buf ^ 1);
      store_b(buf ^ 1);
    }
    __syncthreads();
    buf ^= 1;
  }

  // epilogue through LDS, EC columns (the two waves with wc = pass) at a time:
  // Cs[(c - c0) * (TBM + 1) + r]
  float* Cs = smem;
  const bool split = p.splits > 1;
#pragma unroll
  for (int pass = 0; pass < TBN / EC; ++pass) {
    if (pass > 0) __syncthreads();
    if (wc == pass) {
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          const int cl = b * 16 + (lane & 15);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rl = wr * WM + a * 16 + 4 * (lane >> 4) + v;
            Cs[cl * (TBM + 1) + rl] = acc[a][b][v];
          }
        }
    }
    __syncthreads();
    if (p.Cf && !split) {
      // FP32 C (the basis update of the mixed back-transformation): 8 old
      // values per batch, kept in FP32 (8 registers, as the 4 doubles below)
      constexpr int PF = 8, NBF = EC * TBM / (256 * PF);
      static_assert(NBF * 256 * PF == EC * TBM, "epilogue pass is not a whole number of batches");
      const bool read_cf = p.beta != 0.0;
#pragma unroll
      for (int h = 0; h < NBF; ++h) {
        bool ok[PF];
        float cold[PF];
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int idx = tid + 256 * (h * PF + u);
          const int rl = idx % TBM, cl = idx / TBM;
          const int row = i0 + rl, col = j0 + pass * EC + cl;
          ok[u] = in_c(row, col);
          cold[u] = 0.0f;
          if (ok[u] && read_cf) cold[u] = gbl(p.Cf)[(long)row + (long)col * p.ldc];
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          if (!ok[u]) continue;
          const int idx = tid + 256 * (h * PF + u);
          const int rl = idx % TBM, cl = idx / TBM;
          const int row = i0 + rl, col = j0 + pass * EC + cl;
          const double out = p.alpha * (double)Cs[cl * (TBM + 1) + rl];
          const double res = read_cf ? out + p.beta * (double)cold[u] : out;
          gbl(p.Cf)[(long)row + (long)col * p.ldc] = (float)res;
        }
      }
      continue;
    }
    // the old C values of 4 elements per thread are loaded before any of
    // them is stored (one round trip per element otherwise; 4 keeps the
    // main loop's occupancy)
    constexpr int PER = 4, NB16 = EC * TBM / (256 * PER);
    static_assert(NB16 * 256 * PER == EC * TBM, "epilogue pass is not a whole number of batches");
    const bool read_c = !split && p.beta != 0.0;
#pragma unroll
    for (int h = 0; h < NB16; ++h) {
      bool ok[PER];
      double cold[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + 256 * (h * PER + u);
        const int rl = idx % TBM, cl = idx / TBM;
        const int row = i0 + rl, col = j0 + pass * EC + cl;
        ok[u] = in_c(row, col);
        cold[u] = 0.0;
        if (ok[u] && read_c) {
          const long o = (long)row + (long)col * p.ldc;
          cold[u] = p.Cf ? (double)gbl(p.Cf)[o] : (p.Cin ? gbl(p.Cin)[o] : gbl(p.C)[o]);
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        if (!ok[u]) continue;
        const int idx = tid + 256 * (h * PER + u);
        const int rl = idx % TBM, cl = idx / TBM;
        const int row = i0 + rl, col = j0 + pass * EC + cl;
        const double val = (double)Cs[cl * (TBM + 1) + rl];
        const double out = p.alpha * val;
        const double res = read_c ? out + p.beta * cold[u] : out;
        const long o = (long)row + (long)col * p.ldc;
        if (split) gbl(p.part)[(long)slice * p.M * p.N + (long)row + (long)col * p.M] = val;
        else if (p.Cf) gbl(p.Cf)[o] = (float)res;
        else gbl(p.C)[o] = res;
      }
    }
  }
}

// C = alpha * sum_s part[s] + beta * C over the (uplo-restricted) M x N
__global__ __launch_bounds__(256) void k_splitk_reduce(const Prob* __restrict__ probs, int op, int step,
                                                       GemmParams single) {
  int stp = step;
  if (probs && is_refine_op(op)) {
    const int st = *gbl(probs[blockIdx.z].refstate);
    if (step >= 0 && st != 0 && st <= step) return;
    if (step < 0) stp = st;
  }
  if (probs && (op == GOP_GRAM || op == GOP_GRAM_SYRK || op == GOP_GRAM_PANEL || op == GOP_GRAM_UPD ||
                 op == GOP_GRAM_UPD_PANEL) && *gbl(probs[blockIdx.z].reorth) == 0)
    return;   // no cluster Gram-Schmidt for this problem
  const GemmParams p = probs ? gemm_params(op, probs[blockIdx.z], stp) : single;
  if (p.splits <= 1) return;
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= p.M) return;
  // The thread's 16 entries go through the partials split by split, with
  // the 16 loads of a split in flight together (the sum of each entry keeps
  // the order k = 0, 1, ...); the old C values are loaded first.  Columns
  // past N are read at column N - 1 (in bounds) and never stored.
  const BSE_GLOBAL double* part = gbl(p.part);
  const bool read_c = p.beta != 0.0;
  bool ok[16];
  double cold[16];   // old C (FP64 C)
  float coldf[16];   // old C (FP32 C), widened where it is used
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    ok[q] = c < p.N && !((p.c_uplo == 1 || p.c_uplo == 3) && r < c) && !(p.c_uplo == 2 && r <= c);
    cold[q] = 0.0;
    coldf[q] = 0.0f;
  }
  if (read_c) {   // uniform
    if (p.Cf) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (ok[q]) coldf[q] = gbl(p.Cf)[r + (c0 + q) * p.ldc];
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (ok[q]) cold[q] = gbl(p.C)[r + (c0 + q) * p.ldc];
    }
  }
  const long MN = (long)p.M * p.N;
  const long cmax = (long)p.N - 1;
  double sum[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) sum[q] = 0.0;
  for (int k = 0; k < p.splits; ++k) {
    const BSE_GLOBAL double* pk = part + (long)k * MN + r;
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = pk[min(c0 + q, cmax) * p.M];
#pragma unroll
    for (int q = 0; q < 16; ++q) sum[q] += v[q];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (!ok[q]) continue;
    const double out = p.alpha * sum[q];
    const double res = read_c ? out + p.beta * (p.Cf ? (double)coldf[q] : cold[q]) : out;
    const long o = r + (c0 + q) * p.ldc;
    if (p.Cf) gbl(p.Cf)[o] = (float)res;
    else gbl(p.C)[o] = res;
  }
}

// Tile configurations: 0 = 64 x 64 (BK 16), 1 = 128 x 128 (BK 16),
// 2 = 128 x 64 (BK 16, full outputs only: the triangular tile enumeration
// needs square tiles), 3 = 64 x 64 (BK 32).
constexpr int NCFG = 4;
constexpr int CFG_BM[NCFG] = {64, 128, 128, 64};
constexpr int CFG_BN[NCFG] = {64, 128, 64, 64};

template <bool TA, bool TB>
int launch_t(hipStream_t s, int cfg, dim3 grid, const Prob* probs, int op, int step, const GemmParams& single) {
  switch (cfg) {
    case 1: BSE_LAUNCH((gemm_f64_kernel<TA, TB, 128, 128, 16>), grid, 256, 0, s, probs, op, step, single); break;
    case 2: BSE_LAUNCH((gemm_f64_kernel<TA, TB, 128, 64, 16>), grid, 256, 0, s, probs, op, step, single); break;
    case 3: BSE_LAUNCH((gemm_f64_kernel<TA, TB, 64, 64, 32>), grid, 256, 0, s, probs, op, step, single); break;
    default: BSE_LAUNCH((gemm_f64_kernel<TA, TB, 64, 64, 16>), grid, 256, 0, s, probs, op, step, single); break;
  }
  return 0;
}

int launch(hipStream_t s, bool ta, bool tb, int cfg, dim3 grid, const Prob* probs, int op, int step,
           const GemmParams& single) {
  if (!ta && !tb) return launch_t<false, false>(s, cfg, grid, probs, op, step, single);
  if (!ta && tb) return launch_t<false, true>(s, cfg, grid, probs, op, step, single);
  if (ta && !tb) return launch_t<true, false>(s, cfg, grid, probs, op, step, single);
  return launch_t<true, true>(s, cfg, grid, probs, op, step, single);
}

// workgroups of a product with configuration cfg
long cfg_workgroups(const GemmParams& g, int cfg) {
  if (g.M <= 0 || g.N <= 0) return 0;
  const long tm = (g.M + CFG_BM[cfg] - 1) / CFG_BM[cfg], tn = (g.N + CFG_BN[cfg] - 1) / CFG_BN[cfg];
  return ((g.c_uplo == 1 || g.c_uplo == 2) ? tm * (tm + 1) / 2 : tm * tn) * g.splits;
}

}  // namespace

int gemm_batched(hipStream_t s, const Batch& b, int nact, int op, int step) {
  if (nact <= 0) return 0;
  long maxm = 0, maxn = 0, maxk = 0;
  bool any_split = false, any = false, f32 = false;
  int ta = -1, tb = -1;
  for (int i = 0; i < nact; ++i) {
    const GemmParams g = gemm_params(op, b.host[i], step);
    if (g.M <= 0 || g.N <= 0) continue;
    any = true;
    if (ta < 0) {
      ta = g.ta;
      tb = g.tb;
      f32 = g.f32 != 0;
    }
    if (g.splits > 1) any_split = true;
    maxm = std::max(maxm, (long)g.M);
    maxn = std::max(maxn, (long)g.N);
    maxk = std::max(maxk, (long)g.K);
  }
  if (!any) return 0;
  // 64 x 64 tiles throughout: on this device the 128-wide tiles (one or
  // two waves per SIMD) measured slower for every product of the chain
  const int cfg = 0;
  (void)maxk;
  long maxwg = 0;
  for (int i = 0; i < nact; ++i) maxwg = std::max(maxwg, cfg_workgroups(gemm_params(op, b.host[i], step), cfg));
  if (maxwg == 0) return 0;
  GemmParams dummy{};
  if (f32) {
    // 128 x 128 tiles (gemm_params counts them for FP32 products)
    long wg = 0;
    for (int i = 0; i < nact; ++i) {
      const GemmParams g = gemm_params(op, b.host[i], step);
      if (g.M > 0 && g.N > 0) wg = std::max(wg, g.ntiles * g.splits);
    }
    const dim3 grid((unsigned)wg, 1, (unsigned)nact);
    if (ta == 0 && tb == 0) BSE_LAUNCH((gemm_f32_kernel<false, false>), grid, 256, 0, s, b.dev, op, step, dummy);
    else if (ta == 0) BSE_LAUNCH((gemm_f32_kernel<false, true>), grid, 256, 0, s, b.dev, op, step, dummy);
    else if (tb == 0) BSE_LAUNCH((gemm_f32_kernel<true, false>), grid, 256, 0, s, b.dev, op, step, dummy);
    else BSE_LAUNCH((gemm_f32_kernel<true, true>), grid, 256, 0, s, b.dev, op, step, dummy);
  } else {
    BSE_TRY(launch(s, ta != 0, tb != 0, cfg, dim3((unsigned)maxwg, 1, (unsigned)nact), b.dev, op, step, dummy));
  }
  if (any_split) {
    BSE_LAUNCH(k_splitk_reduce, dim3((unsigned)((maxm + 63) / 64), (unsigned)((maxn + 63) / 64), (unsigned)nact), 256, 0, s, b.dev, op, step, dummy);
  }
  return 0;
}

}  // namespace bse
