// Blocked Householder tridiagonalisation of a real skew-symmetric matrix,
// W = U T U^T (Algorithm 3 step 1; Section 3.3, remark 1).
//
// Reflector k, H_k = I - tau_k v_k v_k^T, acts on rows/columns k+1..N-1 and
// zeroes W[k+2:, k].  For a skew S and p = tau S v one has v^T S v = 0, so
//     H S H = S + v p^T - p v^T
// (no extra rank-one correction as in the symmetric case).  Within a panel of
// nb columns the reflectors are accumulated as in LAPACK's latrd: the
// trailing matrix is not touched, the current one is
//     S~ = S + V P^T - P V^T,
// column i is brought up to date just before its reflector is built, and
//     p_i = tau_i (S v_i + V (P^T v_i) - P (V^T v_i)).
// After the panel, S <- S + V P^T - P V^T is one MFMA product
//     [v_0 p_0 v_1 p_1 ...] [p_0 -v_0 p_1 -v_1 ...]^T  (strictly lower part).
//
// Per column two kernels run:
//   sk_symv   the HBM-bound product S v over the strictly-lower triangle of
//             the trailing matrix, each element read once and used twice
//             (row sum for S v, column sum for -S^T v).  Workgroups stream
//             64-column strips; partial sums go to fixed slots and are summed
//             in a fixed order (deterministic).  Extra workgroups store v and
//             the partial dot products V^T v, P^T v.  Every workgroup first
//             builds the column's reflector (dlarfg convention) from the norm
//             partials left by the previous update, all in the same order, so
//             all of them hold the same tau and scale.
//   sk_update reduces the partials into p, applies the panel corrections,
//             brings the next column up to date and leaves one partial
//             squared norm of it per workgroup.
// W is held in FP64, or in FP32 for the mixed-precision path (the kernels are
// templates on its element type); sums, norms, v and p are always FP64.
//
// No workgroup waits for or signals another inside a launch: on this
// multi-XCD device a release fence per workgroup costs tens of nanoseconds
// each, serialised over the whole device.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int TS = 64;       // symv tile
constexpr int NBMAX = SKTRD_NB;   // panel width
constexpr int DUTY_BLK = 16; // row blocks per workgroup of the panel dot products
constexpr int TMAX = 16;     // row tiles per strip workgroup (upper bound)
constexpr int UPD_SMALL = 48;   // row blocks up to which the update uses 4 wavefronts

// Reflector of the first column of a panel (sk_start) and the subdiagonal
// entry of the column brought up to date by the last update.
struct Ctrl {
  double tau;
  double scale;
  double x0;
  double pad0;
};

__device__ inline void larfg(double x0, double xnorm, double& beta, double& tau, double& scale) {
  if (xnorm == 0.0) {
    beta = x0;
    tau = 0.0;
    scale = 0.0;
    return;
  }
  beta = -copysign(hypot(x0, xnorm), x0);
  tau = (beta - x0) / beta;
  scale = 1.0 / (x0 - beta);
}

// The matrix being reduced: P.W (FP64) or its FP32 copy P.W32.
template <class WT>
__device__ inline WT* wmat(const Prob& P);
template <>
__device__ inline double* wmat<double>(const Prob& P) {
  return P.W;
}
template <>
__device__ inline float* wmat<float>(const Prob& P) {
  return P.W32;
}

// Reflector of column j from the (already up to date) column itself.
template <class WT>
__global__ __launch_bounds__(256) void sk_start(const Prob* __restrict__ probs, int j) {
  __shared__ double red[4];
  const Prob& P = probs[blockIdx.z];
  const int N = P.N;
  if (j > N - 2) return;  // uniform
  const BSE_CONST WT* __restrict__ W = ro(wmat<WT>(P));
  const long ld = P.ld;
  BSE_GLOBAL Ctrl* __restrict__ ctrl = (BSE_GLOBAL Ctrl*)P.ctrl;
  double ss = 0.0;
  for (long r = j + 2 + threadIdx.x; r < N; r += 256) {
    const double v = W[r + (long)j * ld];
    ss += v * v;
  }
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) {
    const double x0 = W[(long)(j + 1) + (long)j * ld];
    double beta, t, sc;
    larfg(x0, sqrt(ss), beta, t, sc);
    ctrl->tau = t;
    ctrl->scale = sc;
    gbl(P.alpha)[j] = -beta;
    gbl(P.tau)[j] = t;
  }
}

// Row tiles per strip workgroup of the matvec for a trailing matrix of nblk
// row blocks.  Long strips amortise each workgroup's prologue (the reflector
// from the norm partials, the first loads) and its reductions; short ones
// keep enough workgroups in flight.  The count depends on the problem alone,
// so a problem's summation order -- and its result -- is the same whether it
// is solved alone or inside a batch.
//
// The counts come from a table of five size buckets per storage type:
// nblk >= t0 -> v0, >= t1 -> v1, >= t2 -> v2, >= t3 -> v3, else v4 (entries
// [t0 t1 t2 t3 v0 v1 v2 v3 v4], FP64 first).  The built-in table was measured
// inside the n = 8192 reduction and on a batch of 256 problems of order
// 128 .. 2048 (an isolated sweep without the prologue preferred about half
// these counts at mid sizes); FP32 tiles carry half the bytes, so their
// strips are longer from 80 row blocks up (16/12 beat the FP64 table by
// ~8 ms; 16 from 80 and 12 from 48 lost it again).  bse_set_tile_table
// replaces it (the autotuner's table); host and device copies are kept
// equal, since the host sizes the grids the device decodes.
constexpr int TILE_TAB = 9;
__constant__ int c_tiles[2][TILE_TAB] = {{224, 160, 80, 0, 16, 12, 8, 6, 6}, {160, 80, 0, 0, 16, 12, 6, 6, 6}};
static int h_tiles[2][TILE_TAB] = {{224, 160, 80, 0, 16, 12, 8, 6, 6}, {160, 80, 0, 0, 16, 12, 6, 6, 6}};

template <class WT>
__host__ __device__ inline int symv_tiles(int nblk) {
#if defined(__HIP_DEVICE_COMPILE__)
  const int* t = c_tiles[sizeof(WT) == 4 ? 1 : 0];
#else
  const int* t = h_tiles[sizeof(WT) == 4 ? 1 : 0];
#endif
  if (nblk >= t[0]) return t[4];
  if (nblk >= t[1]) return t[5];
  if (nblk >= t[2]) return t[6];
  if (nblk >= t[3]) return t[7];
  return t[8];
}

// One element of a matvec tile (NT: with the non-temporal hint), kept in
// its storage type until it is used (an FP32 tile in flight then takes half
// the registers).
template <bool NT, class Ptr>
__device__ inline auto tile_load(Ptr p) {
  if (NT) return __builtin_nontemporal_load(p);
  return *p;
}

// Strip workgroups of the matvec: strip Cl (Cl = 0 .. nblk-1) has
// ceil((nblk - Cl) / T) chunks of T row tiles.  strip_prefix(Cl) counts the
// chunks of the strips before Cl, from F(M) = sum_{m=1..M} ceil(m / T).
__host__ __device__ inline long chunk_sum(long M, long T) {
  const long q = M / T, r = M % T;
  return T * q * (q + 1) / 2 + r * (q + 1);
}
__host__ __device__ inline long strip_prefix(int Cl, int nblk, int T) {
  return chunk_sum(nblk, T) - chunk_sum(nblk - Cl, T);
}
// Duty workgroups per DUTY_BLK row blocks at panel column i: one per 16 of the
// 2i panel columns (at least one, which also stores v_i).
__host__ __device__ inline int duty_groups(int i) { return i > 0 ? (i + 7) / 8 : 1; }
// Workgroups of one problem's matvec launch at panel column i: the duty
// workgroups, then every (strip, chunk) of the trailing triangle, none empty.
__host__ __device__ inline long symv_workgroups(int nblk, int T, int i) {
  return (long)duty_groups(i) * ((nblk + DUTY_BLK - 1) / DUTY_BLK) + chunk_sum(nblk, T);
}

// Problem and workgroup index of this workgroup.  A single problem (or a
// launch sized per problem) has its problem in blockIdx.z; a batch launch puts
// all problems' workgroups back to back, problem p from wgpre[2p + which] on
// (the prefixes of the per-problem counts, written by k_plan at the start of
// the panel).
__device__ inline int locate_problem(const int* __restrict__ wgpre, int which, int nact, long& wid) {
  wid = blockIdx.x;
  if (wgpre == nullptr) return blockIdx.z;
  // count the problems whose first workgroup is at or before this one, 64
  // prefixes per vector load and ballot (one round trip for up to 64
  // problems, instead of a chain of dependent loads)
  const BSE_GLOBAL int* __restrict__ pre = gbl(wgpre);
  const int lane = threadIdx.x & 63;
  const long x = blockIdx.x;
  int cnt = 0;
  for (int base = 0; base < nact; base += 64) {
    const int q = base + lane;
    const bool le = q < nact && pre[2 * q + which] <= x;
    const int c = __popcll(__ballot(le));
    cnt += c;
    if (c < 64) break;
  }
  const int p = cnt - 1;
  wid = x - pre[2 * p + which];
  return p;
}

// Sums NV per-lane values (NV a power of two, at most 64) over the 64 lanes
// of a wavefront.  Each exchange hands half of the remaining values to the
// partner lane and keeps the other half, so it takes NV - 1 + log2(64 / NV)
// shuffles instead of 6 NV.  Lane L returns the total of value L / (64 / NV).
template <int NV>
__device__ inline double wave_sum_many(double (&v)[NV]) {
  const int lane = threadIdx.x & 63;
  int off = 32;
#pragma unroll
  for (int h = NV / 2; h >= 1; h >>= 1) {
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int q = 0; q < h; ++q) {
      const double snd = up ? v[q] : v[q + h];
      const double kp = up ? v[q + h] : v[q];
      v[q] = kp + __shfl_xor(snd, off, 64);
    }
    off >>= 1;
  }
  double r = v[0];
#pragma unroll
  for (; off >= 1; off >>= 1) r += __shfl_xor(r, off, 64);
  return r;
}

template <class Ptr>
__device__ inline double vval(Ptr W, long ld, int j, int s, int N, double scale, long r) {
  if (r == s) return 1.0;
  if (r > s && r < N) return scale * W[r + (long)j * ld];
  return 0.0;
}

// y = S v over the strictly lower triangle of the trailing matrix.
//
// The launch is one row of workgroups per problem (blockIdx.z), with no empty
// ones (a batch of small problems otherwise spends its time dispatching
// workgroups that only exit):
// blockIdx.x < nduty (dispatched first): workgroups (d, g) store v_i for row
//   blocks d*16 .. d*16+15 and their share (8 panel columns) of the panel dot
//   products V^T v, P^T v (summed by the update kernel).
// the rest: workgroup (Cl, k), in strip-major order, streams the 64-column
//   strip Cl over row tiles Cl + k*T .. Cl + k*T + T - 1.  Lane = row inside
//   a tile, wave w owns columns 16w..16w+15 of the strip, so every load
//   instruction reads 64 consecutive doubles of one column.  Row sums (S v)
//   of each tile go to Yrow[rl][Cl] (written once per workgroup); column
//   sums (-S^T v) accumulate in registers over the tiles and are reduced
//   across the wave once (wave_sum_many), into Ycol[Cl][k].
// NT: the tiles are read with the non-temporal hint.  A trailing triangle
// much larger than the device's last-level cache then streams faster (5.0 ->
// 5.5 TB/s at 16384 rows); one that nearly fits is read faster through it.
template <class WT, bool NT>
__global__ __launch_bounds__(256) void sk_symv(const Prob* __restrict__ probs, int j, int i,
                                               const int* __restrict__ wgpre, int nact) {
  __shared__ double rsum[TMAX][4][TS];   // per-wave row sums of every tile
  long wid;
  const Prob& P = probs[locate_problem(wgpre, 0, nact, wid)];
  const int N = P.N;
  if (j >= N - 2) return;  // uniform: this problem is already reduced
  const int s = j + 1;
  const int R0 = s / TS;
  const int nblk = (N - 1) / TS - R0 + 1;
  const int T = symv_tiles<WT>(nblk);
  const int nchunk = (nblk + T - 1) / T;
  const long ld = P.ld, ldy = P.ld;
  const int dstride = (int)(ld / TS);
  const BSE_CONST WT* __restrict__ W = ro(wmat<WT>(P));
  const BSE_CONST Ctrl* __restrict__ ctrl = (const BSE_CONST Ctrl*)P.ctrl;
  BSE_GLOBAL double* __restrict__ Y1 = gbl(P.Y1);
  BSE_GLOBAL double* __restrict__ Y2 = gbl(P.Y2);
  BSE_GLOBAL double* __restrict__ Yrow = gbl(P.Yrow);
  BSE_GLOBAL double* __restrict__ Ycol = gbl(P.Ycol);
  BSE_GLOBAL double* __restrict__ dotpart = gbl(P.dotpart);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // Scale 1 / (x0 - beta) of column j's reflector.  The first column of a
  // panel got it from sk_start.  Any other column was brought up to date by
  // the previous update, whose workgroups (one per row block from row j)
  // left partial squared norms of rows j+2.. and the subdiagonal entry x0;
  // every workgroup reduces them in the same fixed order, so all hold the
  // same tau and scale.  Branch-free, so that callers can issue their first
  // loads before it.
  auto column_scale = [&]() -> double {
    const BSE_CONST double* __restrict__ normpart = ro(P.normpart);
    const int nprev = (N - 1) / TS - j / TS + 1;
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = (lane + 64 * u < nprev) ? normpart[lane + 64 * u] : 0.0;
    double ss = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    for (int q = lane + 512; q < nprev; q += 64) ss += normpart[q];
    ss = wave_sum(ss);   // the same value in every lane
    double beta, tau, sc;
    larfg(ctrl->x0, sqrt(ss), beta, tau, sc);
    if (i > 0 && wid == 0 && threadIdx.x == 0) {   // the first duty workgroup
      gbl(P.alpha)[j] = -beta;
      gbl(P.tau)[j] = tau;
    }
    return uniform_double(i == 0 ? ctrl->scale : sc);
  };

  const int ngrp = duty_groups(i);
  const int nduty = ngrp * ((nblk + DUTY_BLK - 1) / DUTY_BLK);
  if (wid < nduty) {
    // duty workgroup (d, g) covers row blocks d*DUTY_BLK .. +DUTY_BLK-1 and the
    // panel columns 16g .. 16g+15 below 2i: group 0 stores v_i, every group
    // writes its partial dot products of those panel columns with v_i; the
    // update kernel adds the partials of each column (16 per 16384 rows).  Wave
    // w takes the 8 columns of half h = w & 1 and every second row block from
    // w >> 1, all of a block's loads issued at once: a wave waits on 8 blocks'
    // loads in turn (this bounds the launch's latency for short trailing
    // matrices).  The two waves of a half add in LDS.
    const int d = (int)wid / ngrp, g = (int)wid % ngrp;
    const int b1 = min(nblk, d * DUTY_BLK + DUTY_BLK);
    // wave-uniform column bases in scalar registers, a 32-bit row offset per
    // lane: the duty branch stays below the strips' register count
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    const int h = wvu & 1;
    const int lbase = 16 * g + 8 * h;
    const auto vcol = W + (long)j * ld;
    const auto ycol = Y1 + (long)lbase * ldy;
    const double scale = column_scale();
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int b = d * DUTY_BLK + (wvu >> 1); b < b1; b += 2) {
      // rows below (R0 + nblk) * 64 <= ld and the 2 * NBMAX panel columns are
      // allocated: every load is issued before the store of v
      const int r = (R0 + b) * TS + lane;
      const bool inrange = r >= s && r < N;
      const double x = vcol[r];
      double y[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double t = ycol[(long)q * ldy + r];
        y[q] = (lbase + q < 2 * i && inrange) ? t : 0.0;
      }
      const double v = (r == s) ? 1.0 : (inrange ? scale * x : 0.0);
      if (g == 0 && h == 0 && inrange) {
        Y1[r + (long)(2 * i) * ldy] = v;
        Y2[r + (long)(2 * i + 1) * ldy] = -v;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += y[q] * v;
    }
    if (i == 0) return;  // uniform
    // lane 8q ends with the wave's total of column lbase + q
    const double tot = wave_sum_many(acc);
    double* red = &rsum[0][0][0];
    if ((lane & 7) == 0) red[wv * 8 + (lane >> 3)] = tot;
    __syncthreads();
    if (wv < 2 && lane < 8 && lbase + lane < 2 * i)
      dotpart[(long)(lbase + lane) * dstride + d] = red[wv * 8 + lane] + red[(wv + 2) * 8 + lane];
    return;
  }

  // (strip, chunk) of this workgroup: the largest Cl with strip_prefix(Cl) <= w
  const long w = wid - nduty;
  if (w >= chunk_sum(nblk, T)) return;  // uniform: beyond this problem's workgroups
  int Cl = 0;
  {
    int hi = nblk - 1;
    while (Cl < hi) {
      const int mid = (Cl + hi + 1) >> 1;
      if (strip_prefix(mid, nblk, T) <= w) Cl = mid;
      else hi = mid - 1;
    }
  }
  const int k = (int)(w - strip_prefix(Cl, nblk, T));
  const int rl0 = Cl + k * T;
  const int rl1 = min(nblk, rl0 + T);
  const long C0 = (long)(R0 + Cl) * TS;
  // wave-uniform values live in scalar registers: the column base pointer and
  // v at the wave's 16 columns (keeps VGPR use, and so occupancy, low)
  const int wvu = __builtin_amdgcn_readfirstlane(wv);
  const long col0 = C0 + 16 * wvu;
  const auto vcol = W + (long)j * ld;   // column j holds x; v = scale * x below row s
  const auto colbase = W + col0 * ld;
  // The tile loop is a software pipeline: the loads of the next step are
  // issued before the current one is used, with no barrier, no global store
  // and no dependent load inside the loop (x at the tile's rows is fetched
  // with the tile).  Two register buffers take turns (the loop is unrolled
  // by two): copying a prefetch buffer into a working one made the wave wait
  // for the prefetched loads at the end of every step.  Tile values and x
  // stay in their storage type until used: converting an FP32 value on
  // arrival made the wave wait for that load, and with it for every load
  // issued before it.  The first step's loads and x at the strip's columns
  // are issued before the reflector is known.  A step is SP = 1 tile; the
  // array form (measured against a scalar rewrite of the same loop) compiles
  // to fewer waits.
  constexpr int SP = 1;   // tiles per step
  auto load_step = [&](int rl, WT(&t)[SP][16], WT(&x)[SP]) {
#pragma unroll
    for (int p = 0; p < SP; ++p) {
      if (p == 0 || rl + p < rl1) {
        const int off = (int)((long)(R0 + rl + p) * TS) + lane;   // 32-bit lane offset (rows < 2^28)
#pragma unroll
        for (int q = 0; q < 16; ++q) t[p][q] = tile_load<NT>(colbase + (long)q * ld + off);
        x[p] = vcol[off];
      }
    }
  };
  WT bufA[SP][16], bufB[SP][16];
  WT xA[SP], xB[SP], xc[16];
  load_step(rl0, bufA, xA);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const long c = col0 + q;
    xc[q] = vcol[c < N ? c : 0];
  }
  const double scale = column_scale();
  double vc[16];   // wave-uniform: moved to scalar registers
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const long c = col0 + q;
    vc[q] = uniform_double((c == s) ? 1.0 : ((c > s && c < N) ? scale * xc[q] : 0.0));
  }
  double cacc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) cacc[q] = 0.0;
  const bool strip_inside = C0 >= s;
  auto process_step = [&](int rl, WT(&a)[SP][16], const WT(&xr)[SP]) {
#pragma unroll
    for (int p = 0; p < SP; ++p) {
      if (p == 0 || rl + p < rl1) {
        const long rbase = (long)(R0 + rl + p) * TS;
        const long row = rbase + lane;
        const double vr = (row == s) ? 1.0 : ((row > s && row < N) ? scale * xr[p] : 0.0);
        const bool interior = (rl + p > Cl) && strip_inside && (rbase + TS <= N);
        if (!interior) {
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const long col = col0 + q;
            if (!(row > col && col >= s && row < N)) a[p][q] = 0.0;
          }
        }
        double racc = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          racc += a[p][q] * vc[q];
          cacc[q] += a[p][q] * vr;
        }
        rsum[rl + p - rl0][wv][lane] = racc;
      }
    }
  };
  for (int rl = rl0;;) {
    if (rl + SP < rl1) load_step(rl + SP, bufB, xB);
    process_step(rl, bufA, xA);
    rl += SP;
    if (rl >= rl1) break;
    if (rl + SP < rl1) load_step(rl + SP, bufA, xA);
    process_step(rl, bufB, xB);
    rl += SP;
    if (rl >= rl1) break;
  }
  // column sums over the 64 lanes: lane 4q ends with the total of column q
  const double csum = wave_sum_many(cacc);
  if ((lane & 3) == 0) Ycol[((long)Cl * nchunk + k) * TS + 16 * wv + (lane >> 2)] = -csum;
  __syncthreads();
  // Yrow is [row block][strip][64]: the update kernel of a row block reads
  // its b + 1 row parts contiguously
  for (int t = wv; t < rl1 - rl0; t += 4)
    Yrow[((long)(rl0 + t) * nblk + Cl) * TS + lane] =
        rsum[t][0][lane] + rsum[t][1][lane] + rsum[t][2][lane] + rsum[t][3][lane];
}

// FP32 copies of the panel's columns [v_l p_l] (Y1) and [p_l -v_l] (Y2),
// rows e = k0 + nbp .. N-1, for the rank-2k update of the FP32 W on the FP32
// matrix cores (mixed-precision problems only).  Grid: rows x 2 NBMAX
// columns x problems.
__global__ __launch_bounds__(256) void k_y_to_f32(const Prob* __restrict__ probs, int k0) {
  const Prob& P = probs[blockIdx.z];
  if (P.prec != BSE_PREC_FP32_REFINE) return;   // uniform
  const int N = P.N;
  if (k0 > N - 2) return;
  const int nbp = min(NBMAX, N - 1 - k0);
  const int e = k0 + nbp;
  if (N - e < 2 || e > N - 2) return;   // no update (as GOP_SKTRD_R2K)
  const int c = blockIdx.y;
  if (c >= 2 * nbp) return;
  const long r = e + (long)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  const long o = r + (long)c * P.ld;
  gbl(P.Y1f)[o] = (float)gbl(P.Y1)[o];
  gbl(P.Y2f)[o] = (float)gbl(P.Y2)[o];
}

// p_i = tau (S v + V c_P - P c_V) for the rows of block b, the in-place store
// of v_i, and the update of the next column with one partial squared norm of
// it per workgroup.  The UW wavefronts share the 64-row block: the partial
// sums of S v and the panel sums over l are split over them, so that every
// thread has only a few loads to wait for.
// UW wavefronts per workgroup: 16 while the row blocks have many partials to
// reduce, 4 for short trailing matrices (small problems of a batch, the end
// of a reduction), where the larger workgroups only cost occupancy.
template <class WT, int UW>
__global__ __launch_bounds__(64 * UW) void sk_update(const Prob* __restrict__ probs, int j, int i,
                                                     const int* __restrict__ wgpre, int nact) {
  __shared__ double cs[2 * NBMAX];
  __shared__ double ys_row[2 * NBMAX];   // Y1 row s (v_l[s], p_l[s])
  __shared__ double red[UW][TS];    // partial sums of S v
  __shared__ double red2[UW][TS];   // panel correction of p_i
  __shared__ double red3[UW][TS];   // panel correction of the next column
  __shared__ double red4[UW];
  long wid;
  const Prob& P = probs[locate_problem(wgpre, 1, nact, wid)];
  const int N = P.N;
  if (j >= N - 2) return;  // uniform
  const int s = j + 1;
  const int R0 = s / TS;
  const int nblk = (N - 1) / TS - R0 + 1;
  const int b = (int)wid;
  if (b >= nblk) return;  // uniform: beyond this problem's row blocks
  const int T = symv_tiles<WT>(nblk);
  const int nchunk = (nblk + T - 1) / T;
  const int k0 = j - i;   // first column of the panel
  const int nbp = min(NBMAX, N - 1 - k0);
  const long ld = P.ld, ldy = P.ld;
  const int dstride = (int)(ld / TS);
  BSE_GLOBAL WT* __restrict__ W = gbl(wmat<WT>(P));
  BSE_GLOBAL Ctrl* __restrict__ ctrl = (BSE_GLOBAL Ctrl*)P.ctrl;
  BSE_GLOBAL double* __restrict__ Y1 = gbl(P.Y1);
  BSE_GLOBAL double* __restrict__ Y2 = gbl(P.Y2);
  const BSE_CONST double* __restrict__ Yrow = ro(P.Yrow);
  const BSE_CONST double* __restrict__ Ycol = ro(P.Ycol);
  BSE_GLOBAL double* __restrict__ normpart = gbl(P.normpart);
  BSE_GLOBAL double* __restrict__ alpha = gbl(P.alpha);
  BSE_GLOBAL double* __restrict__ tau_arr = gbl(P.tau);
  const BSE_CONST double* __restrict__ dotpart = ro(P.dotpart);
  const int tid = threadIdx.x;
  const int t = tid & 63, part = tid >> 6;
  const double tau = tau_arr[j];   // written by sk_start or by this column's matvec
  if (tid < 2 * i) {
    // c[l] = sum of the symv duty workgroups' partial dot products
    const int nd = (nblk + DUTY_BLK - 1) / DUTY_BLK;   // 16 partials per 16384 rows
    double c = 0.0;
    for (int d0 = 0; d0 < nd; d0 += 16) {
      double pc[16];
#pragma unroll
      for (int dd = 0; dd < 16; ++dd) pc[dd] = (d0 + dd < nd) ? dotpart[(long)tid * dstride + d0 + dd] : 0.0;
#pragma unroll
      for (int dd = 0; dd < 16; ++dd) c += pc[dd];
    }
    cs[tid] = c;
    ys_row[tid] = Y1[s + (long)tid * ldy];
  }
  const long r = (long)(R0 + b) * TS + t;
  const bool inrange = r >= s && r < N;
  // this row's panel entries (v_l, p_l for l = part, part + UW, ...), v_i, and
  // W[r, s]: loaded once, before anything waits, and used by both
  // corrections below
  constexpr int NQ = NBMAX / UW;
  double yv[NQ], yp[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int l = part + UW * q;
    const bool use = inrange && l < i;
    yv[q] = use ? Y1[r + (long)(2 * l) * ldy] : 0.0;
    yp[q] = use ? Y1[r + (long)(2 * l + 1) * ldy] : 0.0;
  }
  const double vi = inrange ? Y1[r + (long)(2 * i) * ldy] : 0.0;
  const double wrs = (r >= s + 1 && r < N) ? (double)W[r + (long)s * ld] : 0.0;
  const bool next_col = (i + 1 < nbp) && (s <= N - 2);
  // partial sums of S v at row s (first row of block 0), needed by every
  // block for the next column: wave 1 starts loading them now
  double srow = 0.0;
  if (next_col && part == 1) {
    const long os = s - (long)R0 * TS;
    const int nch0 = (nblk + T - 1) / T;
    srow = (t == 0) ? Yrow[os] : 0.0;
    for (int c = t; c < nch0; c += 64) srow += Ycol[(long)c * TS + os];
  }
  {
    // partial sums of this row block: b+1 row parts (one per strip c <= b,
    // contiguous in Yrow[b][c][64]) and nch column parts (one per chunk of
    // strip b); loads are issued in batches of 8
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    const auto yr = Yrow + (long)b * nblk * TS + t;
    for (int c0 = part; c0 <= b; c0 += 8 * UW) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = c0 + UW * q;
        if (c <= b) acc[q] += yr[(long)c * TS];
      }
    }
    const int nch = (nblk - b + T - 1) / T;
    const auto yc = Ycol + (long)b * nchunk * TS + t;
    for (int c0 = part; c0 < nch; c0 += 8 * UW) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = c0 + UW * q;
        if (c < nch) acc[q] += yc[(long)c * TS];
      }
    }
    red[part][t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  // p_i at row s (first row of block 0) is needed by every block for the
  // next column: its S v part now, its panel part after the barrier
  if (next_col && part == 1) {
    const double acc = wave_sum(srow);
    if (t == 0) red4[1] = acc;
  }
  __syncthreads();
  // every wave's share of the panel corrections, of p_i (from c) and of the
  // next column (from row s of the panel, ys_row); wave 0 adds them up after
  // one more barrier and does the rest alone
  {
    double corr = 0.0, upd = 0.0;
    if (inrange) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int l = part + UW * q;
        if (l < i) corr += yv[q] * cs[2 * l + 1] - yp[q] * cs[2 * l];
      }
    }
    if (next_col && r >= s + 1 && r < N) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int l = part + UW * q;
        if (l < i) upd += yv[q] * ys_row[2 * l + 1] - yp[q] * ys_row[2 * l];
      }
    }
    red2[part][t] = corr;
    red3[part][t] = upd;
  }
  if (next_col && part == 2) {
    double acc = 0.0;
    if (t < i) acc = ys_row[2 * t] * cs[2 * t + 1] - ys_row[2 * t + 1] * cs[2 * t];
    acc = wave_sum(acc);
    if (t == 0) red4[2] = acc;
  }
  __syncthreads();
  if (part != 0) return;
  double p = 0.0;
  if (inrange) {
    double y = 0.0, corr = 0.0;
#pragma unroll
    for (int w = 0; w < UW; ++w) {
      y += red[w][t];
      corr += red2[w][t];
    }
    p = tau * (y + corr);
    Y1[r + (long)(2 * i + 1) * ldy] = p;
    Y2[r + (long)(2 * i) * ldy] = p;
    if (r > s) W[r + (long)j * ld] = vi;  // store v_i in place
  }
  if (!next_col) return;  // uniform
  const double sval_s = tau * (red4[1] + red4[2]);
  double nrm = 0.0;
  if (r >= s + 1 && r < N) {
    double upd = wrs;
#pragma unroll
    for (int w = 0; w < UW; ++w) upd += red3[w][t];
    upd += vi * sval_s - p;
    // the column as stored (rounded to T) is what the next reflector sees
    const double upds = (double)(WT)upd;
    W[r + (long)s * ld] = (WT)upd;
    if (r == s + 1) {
      ctrl->x0 = upds;
      if (s == N - 2) {
        // the last column has nothing below its subdiagonal: its reflector
        // is the identity (dlarfg with a zero norm)
        alpha[s] = -upds;
        tau_arr[s] = 0.0;
      }
    }
    if (r >= s + 2) nrm = upds * upds;
  }
  // only wave 0 holds rows of the column: a wave sum (the block sum it
  // replaces added the other waves' zeros)
  nrm = wave_sum(nrm);
  if (t == 0) normpart[b] = nrm;
}

// Workgroup prefixes of the batch launches of a whole panel, one workgroup
// per column j = k0 + blockIdx.x (i = blockIdx.x): row i of wgpre holds
// wgpre[2p] (matvec) and wgpre[2p + 1] (update), the workgroups of the
// problems before p that are still active at column j (problems are sorted
// by decreasing order, so the active ones come first and the others count
// zero).  One launch per panel instead of one per column.
template <class WT>
__global__ __launch_bounds__(1024) void k_plan(const Prob* __restrict__ probs, int nact, int k0,
                                               int stride, int* __restrict__ wgpre_all) {
  __shared__ int ssum[1024], usum[1024];
  const int tid = threadIdx.x;
  const int i = blockIdx.x, j = k0 + i;
  int* __restrict__ wgpre = wgpre_all + (long)i * stride;
  const int per = (nact + 1023) / 1024;
  const int p0 = min(nact, tid * per), p1 = min(nact, p0 + per);
  auto counts = [&](int p, int& cs, int& cu) {
    const int N = probs[p].N;
    if (j >= N - 2) {   // this problem is already reduced
      cs = cu = 0;
      return;
    }
    const int s = j + 1;
    const int nblk = (N - 1) / TS - s / TS + 1;
    cs = (int)symv_workgroups(nblk, symv_tiles<WT>(nblk), i);
    cu = nblk;
  };
  int ts = 0, tu = 0;
  for (int p = p0; p < p1; ++p) {
    int cs, cu;
    counts(p, cs, cu);
    ts += cs;
    tu += cu;
  }
  ssum[tid] = ts;
  usum[tid] = tu;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan
    const int a = tid >= off ? ssum[tid - off] : 0;
    const int c = tid >= off ? usum[tid - off] : 0;
    __syncthreads();
    ssum[tid] += a;
    usum[tid] += c;
    __syncthreads();
  }
  int es = ssum[tid] - ts, eu = usum[tid] - tu;
  BSE_GLOBAL int* __restrict__ pre = gbl(wgpre);
  for (int p = p0; p < p1; ++p) {
    int cs, cu;
    counts(p, cs, cu);
    pre[2 * p] = es;
    pre[2 * p + 1] = eu;
    es += cs;
    eu += cu;
  }
  if (tid == 1023) {
    pre[2 * nact] = ssum[1023];
    pre[2 * nact + 1] = usum[1023];
  }
}

}  // namespace

size_t sktrd_work_bytes(long N, long ld) {
  (void)N;
  const long nt = ld / TS;
  size_t bytes = 0;
  bytes += 2 * (size_t)ld * 2 * NBMAX * sizeof(double);            // Y1, Y2
  bytes += 2 * (size_t)nt * nt * TS * sizeof(double);             // Yrow, Ycol
  bytes += (size_t)nt * 2 * NBMAX * sizeof(double);               // dotpart
  bytes += (size_t)nt * sizeof(double);                           // normpart
  bytes += sizeof(Ctrl);                                          // ctrl
  return bytes + 7 * 256;
}

void sktrd_bind_work(char* base, long N, long ld, Prob* P) {
  (void)N;
  const long nt = ld / TS;
  char* p = base;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += round_up((long)bytes, 256);
    return q;
  };
  P->Y1 = reinterpret_cast<double*>(take((size_t)ld * 2 * NBMAX * sizeof(double)));
  P->Y2 = reinterpret_cast<double*>(take((size_t)ld * 2 * NBMAX * sizeof(double)));
  P->Yrow = reinterpret_cast<double*>(take((size_t)nt * nt * TS * sizeof(double)));
  P->Ycol = reinterpret_cast<double*>(take((size_t)nt * nt * TS * sizeof(double)));
  P->dotpart = reinterpret_cast<double*>(take((size_t)nt * 2 * NBMAX * sizeof(double)));
  P->normpart = reinterpret_cast<double*>(take((size_t)nt * sizeof(double)));
  P->ctrl = take(sizeof(Ctrl));
}

template <class WT>
static int sktrd_run(hipStream_t s, const Batch& b, KernelTimer* timer) {
  const int N0 = b.maxN();
  if (N0 < 2) return 0;
  const int nb = NBMAX;
  const int stride = 2 * (b.count + 1);   // ints per column of the prefix table
  for (int k0 = 0; k0 <= N0 - 2; k0 += nb) {
    const int nstart = b.active_N_above(k0 + 1);   // N - 2 >= k0
    BSE_LAUNCH(sk_start<WT>, dim3(1, 1, (unsigned)nstart), 256, 0, s, b.dev, k0);
    const int ncols = min(nb, N0 - 2 - k0);   // columns of this panel with a reflector
    if (nstart > 1 && b.wgpre != nullptr && ncols > 0) {   // the batch launches of this panel
      BSE_LAUNCH(k_plan<WT>, (unsigned)ncols, 1024, 0, s, b.dev, nstart, k0, stride, b.wgpre);
    }
    for (int i = 0; i < nb; ++i) {
      const int j = k0 + i;
      if (j >= N0 - 2) break;  // the last column has no reflector to apply
      const int nact = b.active_N_above(j + 2);   // problems with j < N - 2
      const int sidx = j + 1;
      const int R0 = sidx / TS;
      const int nblk0 = (N0 - 1) / TS - R0 + 1;
      // workgroups: a batch runs every problem's back to back (prefixes from
      // k_plan), a single problem its own row
      const bool packed = nact > 1 && b.wgpre != nullptr;
      long gx = 0, gu = 0;
      for (int q = 0; q < nact; ++q) {
        const int nbq = (b.host[q].N - 1) / TS - R0 + 1;
        gx += symv_workgroups(nbq, symv_tiles<WT>(nbq), i);
        gu += nbq;
      }
      const int* pre = packed ? b.wgpre + (long)i * stride : nullptr;
      const dim3 gs = packed ? dim3((unsigned)gx, 1, 1) : dim3((unsigned)gx, 1, (unsigned)nact);
      const dim3 gup = packed ? dim3((unsigned)gu, 1, 1) : dim3((unsigned)nblk0, 1, (unsigned)nact);
      const bool timed = timer && timer->used + 2 <= timer->cap;
      if (timed) BSE_HIP(hipEventRecord(timer->ev[timer->used], s));
      // the non-temporal hint once the largest trailing triangle is well past
      // the last-level cache (thresholds of 200, 300 and 400 MB measured on
      // the n = 8192 reduction; 300 MB was fastest)
      const double tri_bytes = 0.5 * sizeof(WT) * (double)(N0 - sidx) * (double)(N0 - sidx);
      if (tri_bytes > 300e6) BSE_LAUNCH((sk_symv<WT, true>), gs, 256, 0, s, b.dev, j, i, pre, nact);
      else BSE_LAUNCH((sk_symv<WT, false>), gs, 256, 0, s, b.dev, j, i, pre, nact);
      if (timed) {
        BSE_HIP(hipEventRecord(timer->ev[timer->used + 1], s));
        timer->used += 2;
        for (int q = 0; q < nact; ++q) {
          const double m = (double)(b.host[q].N - sidx);   // trailing order
          timer->bytes += sizeof(WT) * m * (m - 1.0) * 0.5;
        }
      }
      if (nblk0 > UPD_SMALL) BSE_LAUNCH((sk_update<WT, 16>), gup, 1024, 0, s, b.dev, j, i, pre, nact);
      else BSE_LAUNCH((sk_update<WT, 4>), gup, 256, 0, s, b.dev, j, i, pre, nact);
    }
    if constexpr (sizeof(WT) == 4)
      BSE_LAUNCH(k_y_to_f32, dim3((unsigned)((N0 + 255) / 256), 2 * NBMAX, (unsigned)nstart), 256, 0, s, b.dev, k0);
    BSE_TRY(gemm_batched(s, b, nstart, GOP_SKTRD_R2K, k0));
  }
  return 0;
}

int tile_table_get(int* tab) {
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < TILE_TAB; ++k) tab[p * TILE_TAB + k] = h_tiles[p][k];
  return 0;
}

int tile_table_set(const int* tab) {
  for (int p = 0; p < 2; ++p) {
    const int* t = tab + p * TILE_TAB;
    for (int k = 0; k < 3; ++k)
      if (t[k] < t[k + 1]) return set_error(-3, "tile table: thresholds must not increase");
    if (t[3] < 0) return set_error(-3, "tile table: negative threshold");
    for (int k = 4; k < TILE_TAB; ++k)
      if (t[k] < 1 || t[k] > TMAX) return set_error(-3, "tile table: tile counts must be in [1, 16]");
  }
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < TILE_TAB; ++k) h_tiles[p][k] = tab[p * TILE_TAB + k];
  return 0;
}

// the host table into the current device's constant copy
int tile_table_upload() {
  BSE_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tiles), h_tiles, sizeof(h_tiles), 0, hipMemcpyHostToDevice));
  return 0;
}

int sktrd_batched(hipStream_t s, const Batch& b, KernelTimer* timer) {
  if (b.count <= 0) return 0;
  if (b.host[0].prec == BSE_PREC_FP32_REFINE) return sktrd_run<float>(s, b, timer);
  return sktrd_run<double>(s, b, timer);
}

}  // namespace bse
