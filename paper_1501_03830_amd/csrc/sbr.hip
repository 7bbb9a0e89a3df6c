// Two-stage skew tridiagonalisation (successive band reduction), the route
// Section 3.3 names for moving the reduction's Level-2 work onto Level-3
// products.
//
// Stage 1, dense to band of width B = SBR_B.  For each panel of B columns at
// k0, the rows below the band (r0 = k0 + B .. N-1) are factored P = Q R by
// Householder reflectors (LAPACK dlarfg convention), Q = I - V T V^T; the
// trailing skew block becomes Q^T W22 Q.  With Y = W22 V T and S2 = T^T V^T Y
// (skew), Q^T W22 Q = W22 + V Y'^T - Y' V^T for Y' = Y - (1/2) V S2: the
// skew form of the symmetric two-sided block update (the term that the
// symmetric case splits in halves is skew here and is absorbed the same
// way).  W is kept as its strict lower triangle L (the upper triangle is
// zero), so W22 V = L V - L^T V is two triangular MFMA products and the
// rank-2B update touches the strict lower triangle only.
//
// The panel factorisation is one launch per panel, its column steps
// separated by a grid barrier.  Step j finishes the reflector of column
// j - 1 from the previous step's per-workgroup partial sums (every
// workgroup reduces them in the same order): with x that column
// below its diagonal, x^T x and x^T a_c for the columns c to its right were
// summed in one pass, so beta, tau and every tau v^T a_c follow without a
// second reduction (v = (x - beta e_1) / (x_0 - beta)); it then applies the
// reflector to its own rows and forms the partial sums of column j.
//
// Stage 2, band to tridiagonal (bulge chasing).  Sweep s annihilates column
// s below its subdiagonal with a reflector on rows s+1 .. s+B; applied from
// both sides it fills a block below the band, whose first column the next
// reflector (on the next B rows) annihilates, and so on down the matrix.
// Fill stays within 2B - 1 below the diagonal.  Steps of consecutive sweeps
// overlap only while sweep s - 1 is within two steps of sweep s, so step t
// of sweep s may run once sweep s - 1 has completed step t + 2 (found by
// tracking the entries every step reads and writes on a model of the
// algorithm).  One persistent launch runs the sweeps on a fixed set of
// workgroups (sweep s on workgroup s mod G, in order), each publishing its
// progress with a release store and waiting for its predecessor with
// acquire loads; the wait is bounded, and a workgroup that runs out of it
// raises an error flag that makes every other wait give up, so every
// workgroup exits.
#include <climits>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int BW = SBR_B;
constexpr int PR = 256;   // panel rows per workgroup, one per thread
constexpr int PP = BW + 1;  // partial sums per workgroup: x^T x, x^T a_c (c < BW)
constexpr int PMAX_WG = 128;   // panel workgroups at most (N <= 32768 + BW)
constexpr int CH_WG = 128;   // workgroups of the bulge-chasing launch
constexpr int DONE = INT_MAX;
constexpr long SPIN_MAX = 1L << 22;

// Sum over the 64 lanes of each of 16 values: each exchange hands half of
// the remaining values to the partner lane (17 shuffles).  On return lane l
// holds the total of value (l >> 2) & 15.
__device__ inline double wave_sum16(double (&x)[16]) {
  const int lane = threadIdx.x & 63;
  int off = 32;
#pragma unroll
  for (int h = 8; h >= 1; h >>= 1) {
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int q = 0; q < h; ++q) {
      const double snd = up ? x[q] : x[q + h];
      const double kp = up ? x[q + h] : x[q];
      x[q] = kp + __shfl_xor(snd, off, 64);
    }
    off >>= 1;
  }
  double r = x[0];
  r += __shfl_xor(r, 2, 64);
  r += __shfl_xor(r, 1, 64);
  return r;
}

// partial sums [2][nwg][PP], then row buffers [2][BW] (in P.Yrow)
__device__ inline double* panel_part(const Prob& P) { return P.Yrow; }

// The panel at k0, in one launch.  Workgroup g holds rows 256g .. 256g+255
// of the panel in registers (one row per thread, all B columns) for the
// whole factorisation.  Column step j finishes reflector j - 1 from the
// partial sums every workgroup published in step j - 1 (each workgroup
// reduces them in the same order), applies it to its rows, then publishes
// its partial sums for column j: x^T x and x^T a_c for the columns c to the
// right, from which beta, tau and every tau v^T a_c follow without a second
// reduction (v = (x - beta e_1) / (x_0 - beta)).  Steps are separated by a
// grid barrier made of one flag word per workgroup: a workgroup publishes
// its sums, then stores the number of the step it finished into its own
// flag (release); the next step waits until every flag has reached it, read
// by wave 0 with one load per flag in a single round trip (relaxed loads,
// then an acquire fence).  One word per writer avoids the serialised
// read-modify-writes of a shared arrival counter.  The wait is bounded; a
// workgroup that runs out of it raises the error flag, which ends every
// other wait, so all workgroups exit.  The grid (at most PMAX_WG
// workgroups) is far below what the device holds at once.
__device__ inline bool flags_wait(const int* flags, int nwg, int target, int* err) {
  const int lane = threadIdx.x & 63;
  long spins = 0;
  for (;;) {
    int lo = INT_MAX;
    for (int q = lane; q < nwg; q += 64)
      lo = min(lo, __hip_atomic_load(flags + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (__all(lo >= target)) break;
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > SPIN_MAX) {
      if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  // pairs with every flag's release store: their workgroups' sums are visible
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

__global__ __launch_bounds__(PR) void k_sbr_panel(const Prob* __restrict__ probs, int k0, int* __restrict__ flags,
                                                  int* __restrict__ err) {
  __shared__ double tot[PP];
  __shared__ double wv[BW];
  __shared__ double red[PR / 64][PP];
  __shared__ double stage[PMAX_WG * PP];
  __shared__ int ok_flag;
  const Prob& P = probs[0];
  const long ld = P.ld;
  const int N = P.N;
  const int r0 = k0 + BW;
  const int m = N - r0;
  const int nr = min(m - 1, BW);
  const int g = blockIdx.x, nwg = gridDim.x;
  const long i = (long)g * PR + threadIdx.x;   // panel row
  double* Pw = P.W + r0 + (long)k0 * ld;
  double* part = panel_part(P);
  double* rowbuf = part + 2L * nwg * PP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool in = i < m;
  double a[BW];
#pragma unroll
  for (int c = 0; c < BW; ++c) a[c] = in ? Pw[i + (long)c * ld] : 0.0;
  for (int j = 0; j <= nr; ++j) {
    if (j >= 1) {
      // wait for every workgroup's partial sums of column j - 1
      if (threadIdx.x < 64) {
        const bool ok = flags_wait(flags, nwg, j, err);
        if (threadIdx.x == 0) ok_flag = ok ? 1 : 0;
      }
      __syncthreads();
      if (!ok_flag) return;
      const int c0 = j - 1;
      const double* pp = part + (long)(c0 & 1) * nwg * PP;
      {
        constexpr int NS = (PMAX_WG * PP + PR - 1) / PR;
        double st[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
          const int e = threadIdx.x + u * PR;
          st[u] = (e < nwg * PP) ? pp[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NS; ++u) {
          const int e = threadIdx.x + u * PR;
          if (e < nwg * PP) stage[e] = st[u];
        }
      }
      __syncthreads();
      // column c summed over the workgroups in order, in four interleaved
      // partial chains combined in a fixed order
      for (int e = threadIdx.x; e < 4 * PP; e += PR) {
        const int c = e % PP, h = e / PP;
        double acc = 0.0;
        for (int q = h; q < nwg; q += 4) acc += stage[q * PP + c];
        red[h][c] = acc;
      }
      __syncthreads();
      if (threadIdx.x < PP)
        tot[threadIdx.x] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
      __syncthreads();
      const double* rb = rowbuf + (c0 & 1) * BW;
      const double sigma = tot[0];
      const double x0 = rb[c0];
      double beta = x0, tau = 0.0, scale = 0.0;
      if (sigma > 0.0) {
        beta = -copysign(sqrt(x0 * x0 + sigma), x0);
        tau = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
      if (threadIdx.x < BW) {
        const int c = threadIdx.x;
        wv[c] = (c > c0) ? tau * (rb[c] + scale * (tot[1 + c] - x0 * rb[c])) : 0.0;
      }
      __syncthreads();
      if (in && i >= c0) {
        // v_i = 1 on the diagonal row (which becomes beta), x_i scale below
        double xc = 0.0;
#pragma unroll
        for (int c = 0; c < BW; ++c) xc = (c == c0) ? a[c] : xc;
        const double vi = (i == c0) ? 1.0 : xc * scale;
        const double keep = (i == c0) ? beta : vi;
#pragma unroll
        for (int c = 0; c < BW; ++c) {
          if (c == c0) a[c] = keep;
          else if (c > c0) a[c] -= wv[c] * vi;
        }
      }
      if (g == 0 && threadIdx.x == 0) P.tau[k0 + c0] = tau;
    }
    if (j < nr) {
      // x = column j below row j (own rows), sums of x^2 (rows > j) and of
      // x a_c (rows >= j) for c > j; row j itself goes to the row buffer
      double xv = 0.0;
#pragma unroll
      for (int c = 0; c < BW; ++c) xv = (c == j) ? a[c] : xv;
      if (!(in && i >= j)) xv = 0.0;
      const double s0 = wave_sum((i > j && in) ? xv * xv : 0.0);
      if (lane == 0) red[wave][0] = s0;
#pragma unroll
      for (int gq = 0; gq < BW / 16; ++gq) {
        double pr[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) pr[q] = xv * a[16 * gq + q];
        const double t = wave_sum16(pr);
        if ((lane & 3) == 0) red[wave][1 + 16 * gq + (lane >> 2)] = t;
      }
      __syncthreads();
      double* mine = part + (long)(j & 1) * nwg * PP + (long)g * PP;
      if (threadIdx.x < PP) {
        const int c = threadIdx.x;
        double acc = 0.0;
        if (c == 0 || c - 1 > j) {
          for (int w = 0; w < PR / 64; ++w) acc += red[w][c];
        }
        mine[c] = acc;
      }
      if (i == j) {
        double* rb = rowbuf + (j & 1) * BW;
#pragma unroll
        for (int c = 0; c < BW; ++c)
          if (c >= j) rb[c] = a[c];
      }
      // arrive: this workgroup's sums of column j are published
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_store(flags + g, j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (in) {
#pragma unroll
    for (int c = 0; c < BW; ++c) Pw[i + (long)c * ld] = a[c];
  }
}

// Flags of the panel launch to zero (and the panels' error flag, before the
// first panel)
__global__ void k_sbr_panel_reset(int* __restrict__ flags, int* __restrict__ err) {
  if (flags)
    for (int q = threadIdx.x; q < PMAX_WG; q += blockDim.x) flags[q] = 0;
  if (err && threadIdx.x == 0) *err = 0;
}

// Explicit reflectors of the panel at k0 (ones on the diagonal, zeros
// above) into P.Vb, rows 0 .. m-1 of the panel.
__global__ __launch_bounds__(256) void k_sbr_extract(const Prob* __restrict__ probs, int k0) {
  const Prob& P = probs[0];
  const long ld = P.ld;
  const int r0 = k0 + BW;
  const int m = P.N - r0;
  const int nr = min(m - 1, BW);
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const BSE_GLOBAL double* __restrict__ Pw = gbl(P.W) + r0 + (long)k0 * ld;
  BSE_GLOBAL double* __restrict__ V = gbl(P.Vb);
  for (int c = 0; c < BW; ++c) {
    double v = 0.0;
    if (c < nr) v = (i < c) ? 0.0 : ((i == c) ? 1.0 : Pw[i + (long)c * ld]);
    V[i + (long)c * ld] = v;
  }
}

// T of the compact WY form Q = I - V T V^T from S = V^T V and tau (LAPACK
// dlarft, forward): T[j, j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] S[0:j, j].
__global__ __launch_bounds__(64) void k_sbr_T(const Prob* __restrict__ probs, int k0) {
  __shared__ double Ts[BW][BW + 1];
  const Prob& P = probs[0];
  const int m = P.N - (k0 + BW);
  const int nr = min(m - 1, BW);
  const BSE_GLOBAL double* __restrict__ S = gbl(P.S);
  const BSE_GLOBAL double* __restrict__ tau = gbl(P.tau) + k0;
  __shared__ double Ss[BW][BW + 1];
  const int r = threadIdx.x;
  for (int c = 0; c < BW; ++c) {
    Ts[r][c] = 0.0;
    Ss[r][c] = (r < nr && c < nr) ? S[r + c * BW] : 0.0;
  }
  __syncthreads();
  for (int jj = 0; jj < nr; ++jj) {
    const double tj = tau[jj];
    if (r < jj) {
      double acc = 0.0;
      for (int l = r; l < jj; ++l) acc += Ts[r][l] * Ss[l][jj];
      Ts[r][jj] = -tj * acc;
    } else if (r == jj) {
      Ts[r][jj] = tj;
    }
    __syncthreads();
  }
  BSE_GLOBAL double* __restrict__ T = gbl(P.S) + BW * BW;
  for (int c = 0; c < BW; ++c) T[r + c * BW] = Ts[r][c];
}

// Y1 = [V | Y'], Y2 = [Y' | -V] for the rank-2B update (Y' in P.W2)
__global__ __launch_bounds__(256) void k_sbr_pack(const Prob* __restrict__ probs, int k0) {
  const Prob& P = probs[0];
  const long ld = P.ld;
  const int m = P.N - (k0 + BW);
  const int nr = min(m - 1, BW);
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const BSE_GLOBAL double* __restrict__ V = gbl(P.Vb);
  const BSE_GLOBAL double* __restrict__ Y = gbl(P.W2);
  BSE_GLOBAL double* __restrict__ Y1 = gbl(P.Y1);
  BSE_GLOBAL double* __restrict__ Y2 = gbl(P.Y2);
  for (int c = 0; c < nr; ++c) {
    const double v = V[i + (long)c * ld], y = Y[i + (long)c * ld];
    Y1[i + (long)c * ld] = v;
    Y1[i + (long)(nr + c) * ld] = y;
    Y2[i + (long)c * ld] = y;
    Y2[i + (long)(nr + c) * ld] = -v;
  }
}

// Zero the chase's fill zone, B < i - j <= 2B (the panel reflectors of
// stage 1 were stored there); progress words to 0, error flag to 0.
__global__ __launch_bounds__(256) void k_sbr_prepare(const Prob* __restrict__ probs, int* __restrict__ prog,
                                                     int* __restrict__ err) {
  const Prob& P = probs[0];
  const long ld = P.ld;
  const int N = P.N;
  const long j = (long)blockIdx.x * 2 + (threadIdx.x >> 7);   // two columns per workgroup
  const int q = threadIdx.x & 127;                            // offset BW+1 .. 2BW
  if (j < N) {
    const long i = j + BW + 1 + q;
    if (q < BW && i < N) gbl(P.W)[i + j * ld] = 0.0;
    if (q == 0) prog[j] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
}

__device__ inline int load_progress(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The band is shared between the workgroups of consecutive sweeps, so the
// chase reads and writes it with relaxed atomic accesses at agent scope
// (coherent across the device's L2 caches without whole-cache write-backs);
// ordering comes from one release store of the progress word per step and,
// on the waiting side, an acquire fence after the relaxed load that saw it,
// made by one thread on either side of a workgroup barrier.
__device__ inline double ld_band(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_band(double* p, double x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bulge chasing, persistent: workgroup w runs sweeps w, w + G, ...
//
// One step (rows r0 .. r1 of the reflector, len <= B) works on four pieces,
// all loaded into registers at its start (lane = row, wave = group of
// columns) so that every global load of the step is in flight at once:
// the column col being annihilated; the block left of the reflector's rows
// (columns col+1 .. r0-1, wave w taking every fourth column); the diagonal
// block (lower part, wave w taking columns 16w .. 16w+15); and the block
// below (rows r1+1 .. r0+2B-1, same columns).  Then H = I - tau v v^T is
// applied: from the left to the left block, as W + v p^T - p v^T with
// p = tau W v to the diagonal block (v^T W v = 0 for skew W), and from the
// right to the block below.
// With store_v the reflectors are also written to W's upper triangle (free
// during the chase, whose band is the lower one) for the back-transformation:
// reflector (s, t) on rows r0 .. r0 + len - 1 in row s, columns r0 ..
// r0 + len - 1, tau in place of v's leading 1.  For fixed column the
// reflectors of consecutive sweeps are then consecutive rows, which is how
// the back-transformation reads them.
__global__ __launch_bounds__(256) void k_sbr_chase(const Prob* __restrict__ probs, int* __restrict__ prog,
                                                   int* __restrict__ err, int store_v) {
  __shared__ double v[BW];
  __shared__ double pv[BW];
  __shared__ double rpart[4][BW];
  __shared__ double csum[BW];
  __shared__ double coef[2];   // tau, and 1 if the reflector is not the identity
  __shared__ int abort_flag;
  const Prob& P = probs[0];
  const int N = P.N;
  const long ld = P.ld;
  double* __restrict__ W = P.W;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int s = blockIdx.x; s < N - 2; s += gridDim.x) {
    int col = s, r0 = s + 1, t = 0;
    while (r0 < N - 1) {
      const int r1 = min(r0 + BW - 1, N - 1);
      const int len = r1 - r0 + 1;
      if (s > 0) {
        if (tid == 0) {
          long spins = 0;
          int ok = 1;
          while (load_progress(prog + s - 1) < t + 3) {
            if (load_progress(err) != 0 || ++spins > SPIN_MAX) {
              ok = 0;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          if (!ok) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          // acquire fence after the relaxed load that saw the predecessor's
          // release store: its band writes happen before this step (a fence,
          // not a second acquire load: one memory round trip less per step)
          else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          abort_flag = !ok;
        }
        __syncthreads();
        if (abort_flag) return;
      }
      const int q0 = r1 + 1;
      const int q1 = min(r0 + 2 * BW - 1, N - 1);
      const int nq = q1 >= q0 ? q1 - q0 + 1 : 0;
      // loads: the column (wave 0), then the three blocks
      double x = 0.0;
      if (wave == 0 && lane < len) x = ld_band(W + (r0 + lane) + (long)col * ld);
      double aL[16], aD[16], aR[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = col + 1 + wave + 4 * q;
        aL[q] = (lane < len && c < r0) ? ld_band(W + (r0 + lane) + (long)c * ld) : 0.0;
        const int j = 16 * wave + q;
        aD[q] = (lane < len && j < lane) ? ld_band(W + (r0 + lane) + (long)(r0 + j) * ld) : 0.0;
        aR[q] = (lane < nq && j < len) ? ld_band(W + (q0 + lane) + (long)(r0 + j) * ld) : 0.0;
      }
      // (1) the reflector
      if (wave == 0) {
        const double sig = wave_sum((lane >= 1 && lane < len) ? x * x : 0.0);
        const double x0 = __shfl(x, 0, 64);
        double beta = x0, tau = 0.0, scale = 0.0;
        if (sig > 0.0) {
          beta = -copysign(sqrt(x0 * x0 + sig), x0);
          tau = (beta - x0) / beta;
          scale = 1.0 / (x0 - beta);
        }
        const double vl = (lane == 0) ? 1.0 : ((lane < len) ? x * scale : 0.0);
        v[lane] = vl;
        if (lane == 0) {
          coef[0] = tau;
          coef[1] = (sig > 0.0) ? 1.0 : 0.0;
        }
        if (store_v && lane < len) W[s + (long)(r0 + lane) * ld] = (lane == 0) ? tau : vl;
        if (lane < len) st_band(W + (r0 + lane) + (long)col * ld, (lane == 0) ? beta : 0.0);
      }
      __syncthreads();
      const double tau = coef[0];
      if (coef[1] != 0.0) {
        const double vi = v[lane];
        // (2) left block: w_c = tau v^T a_c, a_c -= w_c v
        {
          double pr[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) pr[q] = aL[q] * vi;
          const double tot = wave_sum16(pr);
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const double wc = tau * __shfl(tot, 4 * q, 64);
            aL[q] -= wc * vi;
          }
        }
        // (3) diagonal block, D = L - L^T with L its strict lower part:
        // rows of L v by thread partials, columns of L^T v by lane sums
        {
          double rs = 0.0, pr[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int j = 16 * wave + q;
            rs += aD[q] * ((j < BW) ? v[j] : 0.0);
            pr[q] = aD[q] * vi;
          }
          rpart[wave][lane] = rs;
          const double ct = wave_sum16(pr);
          if ((lane & 3) == 0) csum[16 * wave + (lane >> 2)] = ct;
          __syncthreads();
          if (tid < BW)
            pv[tid] = (tid < len) ? tau * (rpart[0][tid] + rpart[1][tid] + rpart[2][tid] + rpart[3][tid] - csum[tid])
                                  : 0.0;
          __syncthreads();
          const double pi = pv[lane];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int j = 16 * wave + q;
            aD[q] += vi * pv[j] - pi * v[j];
          }
        }
        // (4) block below: u = tau R v (row sums), R -= u v^T
        {
          double rs = 0.0;
#pragma unroll
          for (int q = 0; q < 16; ++q) rs += aR[q] * v[16 * wave + q];
          __syncthreads();
          rpart[wave][lane] = rs;
          __syncthreads();
          const double u = tau * (rpart[0][lane] + rpart[1][lane] + rpart[2][lane] + rpart[3][lane]);
#pragma unroll
          for (int q = 0; q < 16; ++q) aR[q] -= u * v[16 * wave + q];
        }
        // stores
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int c = col + 1 + wave + 4 * q;
          if (lane < len && c < r0) st_band(W + (r0 + lane) + (long)c * ld, aL[q]);
          const int j = 16 * wave + q;
          if (lane < len && j < lane) st_band(W + (r0 + lane) + (long)(r0 + j) * ld, aD[q]);
          if (lane < nq && j < len) st_band(W + (q0 + lane) + (long)(r0 + j) * ld, aR[q]);
        }
      }
      // release: this step's band writes, by one thread after the barrier
      __syncthreads();
      if (tid == 0) __hip_atomic_store(prog + s, t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      col = r0;
      r0 = r1 + 1;
      ++t;
    }
    __syncthreads();
    if (tid == 0) __hip_atomic_store(prog + s, DONE, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// alpha[k] = T[k, k+1] = -(subdiagonal entry)
__global__ __launch_bounds__(256) void k_sbr_alpha(const Prob* __restrict__ probs) {
  const Prob& P = probs[0];
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  if (k >= P.N - 1) return;
  gbl(P.alpha)[k] = -gbl(P.W)[(k + 1) + k * P.ld];
}

// The chase's fill zone (B < i - j <= 2B) holds the part of the band
// reduction's reflectors next to the band.  With eigenvectors wanted it is
// copied out before the chase zeroes it (restore = 0: W -> buf) and back
// afterwards (restore = 1), B doubles per column in buf.
__global__ __launch_bounds__(256) void k_sbr_fill(const Prob* __restrict__ probs, double* __restrict__ buf,
                                                  int restore) {
  const Prob& P = probs[0];
  const long ld = P.ld;
  const int N = P.N;
  const long j = (long)blockIdx.x * 4 + (threadIdx.x >> 6);   // four columns per workgroup
  const int q = threadIdx.x & 63;
  if (j >= N) return;
  const long i = j + BW + 1 + q;
  if (i >= N) return;
  BSE_GLOBAL double* __restrict__ w = gbl(P.W) + i + j * ld;
  BSE_GLOBAL double* __restrict__ c = gbl(buf) + j * BW + q;
  if (restore) *w = *c;
  else *c = *w;
}

// ---- back-transformation with the chase's reflectors (Q2) ----
//
// Q2 = H(0,0) H(0,1) ... H(1,0) ... in the order the chase made them (sweep
// s, step t), so Q2 Z applies them last first.  Reflector (s, t) acts on rows
// s + 1 + B t .. s + B + B t, and two of them overlap only if they are of the
// same step and close sweeps, or of neighbouring steps.  They are applied in
// groups: group (sb, t) holds the step-t reflectors of the B sweeps
// s0 = B sb .. s0 + B - 1, on the window of 2B - 1 rows from R0 = s0 + 1 + B t
// (reflector l of the group covers window rows l .. l + B - 1), as one block
// reflector I - V T V^T (T upper triangular, dlarft forward).  Reflector
// (s, t) overlaps only reflectors of step t of sweeps less than B apart, of
// step t - 1 of the B sweeps after s and of step t + 1 of the B sweeps before
// s; of each such pair the one made later must be applied first.  Blocks of
// sweeps last first, inside a block the steps first to last, inside a group
// the sweeps last first, meet every one of these.  Sweep block sb has
// nsb - sb groups.
__host__ __device__ inline int q2_nsb(long N) { return N > 2 ? (int)((N - 2 + BW - 1) / BW) : 0; }
__host__ __device__ inline long q2_group(int nsb, int sb, int t) {
  return (long)sb * nsb - (long)sb * (sb - 1) / 2 + t;
}

// The group's reflectors into Vs[l][i] (reflector l at window row l + i,
// leading 1 explicit) and their tau: reflector l exists if sweep s0 + l has a
// step t (s0 + l <= N - 3 and R0 + l < N - 1); one that does not is zero
// with tau 0.  Lanes run over l, so each load reads consecutive rows of one
// column of W's upper triangle.
__device__ inline void q2_load_V(const BSE_GLOBAL double* __restrict__ W, long ld, int N, int s0, int R0,
                                 double (*Vs)[BW + 1], double* taus) {
  const int tid = threadIdx.x, l = tid & 63;
  const int s = s0 + l;
  const bool live = s <= N - 3 && R0 + l < N - 1;
  for (int m = tid >> 6; m < 2 * BW - 1; m += 4) {
    const int i = m - l;
    if (i < 0 || i >= BW) continue;
    const long R = (long)R0 + m;
    double v = (live && R < N) ? W[s + R * ld] : 0.0;
    if (i == 0) {
      if (taus) taus[l] = v;
      v = live ? 1.0 : 0.0;
    }
    Vs[l][i] = v;
  }
}

// T of every group (one workgroup per group): S = V^T V over the window,
// then T[j, j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] S[0:j, j].
__global__ __launch_bounds__(256) void k_sbr_q2T(const Prob* __restrict__ probs, double* __restrict__ Tbuf) {
  __shared__ double Vs[BW][BW + 1];
  __shared__ double Ss[BW][BW + 1];
  __shared__ double Ts[BW][BW + 1];
  __shared__ double taus[BW];
  const Prob& P = probs[0];
  const int N = P.N;
  const long ld = P.ld;
  const int nsb = q2_nsb(N);
  const long g = blockIdx.x;
  int lo = 0, hi = nsb - 1;   // the last sweep block whose first group is at or before g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (q2_group(nsb, mid, 0) <= g) lo = mid;
    else hi = mid - 1;
  }
  const int sb = lo, t = (int)(g - q2_group(nsb, sb, 0));
  const int s0 = BW * sb, R0 = s0 + 1 + BW * t;
  const int tid = threadIdx.x;
  q2_load_V(gbl(P.W), ld, N, s0, R0, Vs, taus);
  for (int idx = tid; idx < BW * BW; idx += 256) Ts[idx & 63][idx >> 6] = 0.0;
  __syncthreads();
  for (int idx = tid; idx < BW * BW; idx += 256) {
    const int k = idx & 63, j = idx >> 6;
    double acc = 0.0;
    if (k < j) {
      const int d = j - k;   // window row k + i = j + (i - d)
      for (int i = d; i < BW; ++i) acc += Vs[k][i] * Vs[j][i - d];
    }
    Ss[k][j] = acc;
  }
  __syncthreads();
  for (int j = 0; j < BW; ++j) {
    const double tj = taus[j];
    if (tid < j) {
      double acc = 0.0;
      for (int q = tid; q < j; ++q) acc += Ts[tid][q] * Ss[q][j];
      Ts[tid][j] = -tj * acc;
    } else if (tid == j) {
      Ts[j][j] = tj;
    }
    __syncthreads();
  }
  BSE_GLOBAL double* __restrict__ T = gbl(Tbuf) + g * (BW * BW);
  for (int idx = tid; idx < BW * BW; idx += 256) T[idx] = Ts[idx & 63][idx >> 6];
}

// Z <- Q2 Z.  Workgroup c owns columns 64c .. 64c + 63 of Z and applies every
// group to them in the order above, so workgroups never wait for each other.
// The window of the current group lives in an LDS ring of 2B rows (global
// row R in slot (R - s0 - 1) mod 2B): the next group of the same sweep block
// starts B rows lower, so only its last B rows are new and the first B rows
// of the current one leave.  Per group, on the matrix cores:
//   W1 = V^T Zwin  (64 x 64; the band of V limits a row tile to 79 window rows)
//   W2 = T W1      (T upper triangular)
//   Zwin -= V W2
// Eight wavefronts, two per SIMD: wave w owns the 16 columns 16 (w mod 4) ..
// and half h = w / 4 of the row tiles of each product, split so that both
// halves issue the same number of MFMAs.  The group's T and the next
// group's new rows of Z and reflectors are loaded into registers at the
// start of a group, so their latency hides behind its products.  In a
// 16 x 16 block of v_mfma_f64_16x16x4f64 the A operand of lane L is
// A[L mod 16][L / 16], the B operand B[L / 16][L mod 16], and accumulator
// element v of lane L is D[4v + L / 16][L mod 16].
constexpr int QC = 64;    // columns of Z per workgroup
constexpr int QT = 512;   // threads per workgroup
constexpr int VLD = BW + 2;   // row stride of Vs: rows l and l + 1 of a band diagonal fall in different banks
constexpr int ZPF = BW * QC / QT;   // prefetched Z entries per thread
constexpr int VPF = BW * BW / QT;   // reflector entries per thread

// Reflector entries of group (s0, R0) that thread tid loads: lane l = tid mod
// 64 (reflector l), phase p = tid / 64, the window rows m = l + i of its band
// with m = p mod 8: i = ((p - l) mod 8) + 8 u, so every thread takes exactly
// VPF entries and eight neighbouring lanes read eight consecutive rows of one
// column of W's upper triangle.  Loads are unconditional (an entry outside
// the reflector reads W[0] and is masked out when stored): a load under a
// branch, or a select on its value, makes the compiler wait for it at once,
// and these are meant to stay in flight through a whole group.
__device__ inline void q2_fetch_V(const BSE_GLOBAL double* __restrict__ W, long ld, int N, int s0, int R0,
                                  double (&v)[VPF], unsigned& mask) {
  const int tid = threadIdx.x, l = tid & 63;
  const int i0 = ((tid >> 6) - l) & 7;
  const int s = s0 + l;
  const bool live = s <= N - 3 && R0 + l < N - 1;
  mask = 0;
#pragma unroll
  for (int u = 0; u < VPF; ++u) {
    const int i = i0 + 8 * u;
    const long R = (long)R0 + l + i;
    const bool ok = live && i > 0 && R < N;
    v[u] = W[ok ? s + R * ld : 0];
    mask |= (ok ? 1u : 0u) << u;
  }
}
// V[l + i][l] into Vs[l][i] (the leading 1 explicit)
__device__ inline void q2_put_V(const double (&v)[VPF], unsigned mask, int N, int s0, int R0, double (*Vs)[VLD]) {
  const int tid = threadIdx.x, l = tid & 63;
  const int i0 = ((tid >> 6) - l) & 7;
  const bool live = s0 + l <= N - 3 && R0 + l < N - 1;
#pragma unroll
  for (int u = 0; u < VPF; ++u) {
    const int i = i0 + 8 * u;
    Vs[l][i] = (i == 0) ? (live ? 1.0 : 0.0) : (((mask >> u) & 1u) ? v[u] : 0.0);
  }
}
// Window rows B - 1 .. 2B - 2 of the group at R1 (the rows it has beyond the
// previous group's window), lanes along rows; unconditional loads as above.
__device__ inline void q2_fetch_Z(const BSE_GLOBAL double* __restrict__ Z, long ld, int N, int c0, int R1,
                                  double (&z)[ZPF], unsigned& mask) {
  mask = 0;
#pragma unroll
  for (int u = 0; u < ZPF; ++u) {
    const int idx = threadIdx.x + QT * u;
    const int m = (BW - 1) + idx % BW, c = idx / BW;
    const long R = (long)R1 + m;
    const bool ok = R < N && c0 + c < N;
    z[u] = Z[ok ? R + (long)(c0 + c) * ld : 0];
    mask |= (ok ? 1u : 0u) << u;
  }
}

// The three products of one group for half H of the row tiles (H is a
// compile-time constant, so every tile's range of K steps is fixed and the
// loops carry no branches; two independent accumulators are interleaved
// throughout).  tr holds this wave's 20 MFMA A operands of T: i-tile
// it0 = H (16 - 4 it0 K steps from k = 16 it0), then i-tile it1 = 3 - H.
template <int H>
__device__ inline void q2_products(double (*Zs)[QC + 1], double (*Vs)[VLD], double (*Ws)[QC + 1],
                                   double (&tr)[20], const BSE_GLOBAL double* __restrict__ Tnext, int base,
                                   int cl) {
  const int lane = threadIdx.x & 63, kq = lane >> 4, li = lane & 15;
  auto zrow = [&](int m) { return (base + m) & (2 * BW - 1); };
  // W1 = V^T Zwin: l-tiles 2H and 2H + 1, window rows 16 lt .. 16 lt + 79
  {
    d4_t a0 = d4_t{0.0, 0.0, 0.0, 0.0}, a1 = a0;
    const int la = 32 * H + li, lb = la + 16;
#pragma unroll 4
    for (int st = 0; st < 20; ++st) {
      const int ma = 32 * H + 4 * st + kq, mb = ma + 16;
      const double za = Zs[zrow(ma)][cl];
      const double zb = (mb < 2 * BW - 1) ? Zs[zrow(mb)][cl] : 0.0;   // row 2B - 1 is outside the window
      const int ia = ma - la, ib = mb - lb;
      const double va = (ia >= 0 && ia < BW) ? Vs[la][ia] : 0.0;
      const double vb = (ib >= 0 && ib < BW) ? Vs[lb][ib] : 0.0;
      a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(va, za, a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(vb, zb, a1, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Ws[32 * H + 4 * v + kq][cl] = a0[v];
      Ws[32 * H + 16 + 4 * v + kq][cl] = a1[v];
    }
  }
  __syncthreads();
  // W2 = T W1: i-tiles it0 = H (n0 K steps), it1 = 3 - H (n1 steps), T[i][k] = 0 for k < i
  {
    constexpr int it0 = H, it1 = 3 - H, n0 = 16 - 4 * it0, n1 = 16 - 4 * it1;
    d4_t a0 = d4_t{0.0, 0.0, 0.0, 0.0}, a1 = a0;
#pragma unroll
    for (int st = 0; st < n0; ++st) {
      a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(tr[st], Ws[16 * it0 + 4 * st + kq][cl], a0, 0, 0, 0);
      if (st < n1) a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(tr[n0 + st], Ws[16 * it1 + 4 * st + kq][cl], a1, 0, 0, 0);
    }
    // the next group's T into the same registers: a group's time to arrive
    if (Tnext) {
#pragma unroll
      for (int st = 0; st < n0; ++st) tr[st] = Tnext[(16 * it0 + li) + (long)(16 * it0 + 4 * st + kq) * BW];
#pragma unroll
      for (int st = 0; st < n1; ++st) tr[n0 + st] = Tnext[(16 * it1 + li) + (long)(16 * it1 + 4 * st + kq) * BW];
    }
    __syncthreads();   // every wave has read W1
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Ws[16 * it0 + 4 * v + kq][cl] = a0[v];
      Ws[16 * it1 + 4 * v + kq][cl] = a1[v];
    }
  }
  __syncthreads();
  // Zwin -= V W2: m-tile mt needs l in [16 mt - 63, 16 mt + 15]; the tiles
  // go in pairs of equal step counts: H = 0: (3, 4) and (0, 7); H = 1:
  // (2, 5) and (1, 6)
  auto pair = [&](auto MA, auto MB) {
    constexpr int ma = decltype(MA)::value, mb = decltype(MB)::value;
    constexpr int sa = (16 * ma - 64 > 0) ? 16 * ma - 64 : 0, sb = (16 * mb - 64 > 0) ? 16 * mb - 64 : 0;
    constexpr int ea = (16 * ma + 16 < BW) ? 16 * ma + 16 : BW;
    constexpr int ns = (ea - sa) / 4;
    d4_t a0, a1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      a0[v] = Zs[zrow(16 * ma + 4 * v + kq)][cl];
      a1[v] = Zs[zrow(16 * mb + 4 * v + kq)][cl];
    }
    const int mra = 16 * ma + li, mrb = 16 * mb + li;
#pragma unroll 4
    for (int st = 0; st < ns; ++st) {
      const int la = sa + 4 * st + kq, lb = sb + 4 * st + kq;
      const int ia = mra - la, ib = mrb - lb;
      const double va = (ia >= 0 && ia < BW) ? -Vs[la][ia] : 0.0;
      const double vb = (ib >= 0 && ib < BW) ? -Vs[lb][ib] : 0.0;
      a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(va, Ws[la][cl], a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(vb, Ws[lb][cl], a1, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Zs[zrow(16 * ma + 4 * v + kq)][cl] = a0[v];
      Zs[zrow(16 * mb + 4 * v + kq)][cl] = a1[v];
    }
  };
  if constexpr (H == 0) {
    pair(std::integral_constant<int, 3>{}, std::integral_constant<int, 4>{});
    pair(std::integral_constant<int, 0>{}, std::integral_constant<int, 7>{});
  } else {
    pair(std::integral_constant<int, 2>{}, std::integral_constant<int, 5>{});
    pair(std::integral_constant<int, 1>{}, std::integral_constant<int, 6>{});
  }
  __syncthreads();
}

__global__ __launch_bounds__(QT) void k_sbr_q2(const Prob* __restrict__ probs, const double* __restrict__ Tbuf) {
  __shared__ double Zs[2 * BW][QC + 1];
  __shared__ double Vs[BW][VLD];
  __shared__ double Ws[BW][QC + 1];
  const Prob& P = probs[0];
  const int N = P.N;
  const long ld = P.ld;
  const int nsb = q2_nsb(N);
  const int c0 = blockIdx.x * QC;
  if (c0 >= N) return;   // uniform
  BSE_GLOBAL double* __restrict__ Z = gbl(P.Z);
  const BSE_GLOBAL double* __restrict__ W = gbl(P.W);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ct = wave & 3, h = wave >> 2;
  const int cl = 16 * ct + (lane & 15);   // this lane's column in the B operands and results
  const int kq = lane >> 4, li = lane & 15;
  // row tiles of this half: W1 l-tiles {2h, 2h+1} (20 steps each); W2
  // i-tiles {0, 3} or {1, 2} (20 steps in all); Zwin m-tiles {0, 3, 4, 7}
  // or {1, 2, 5, 6} (40 steps in all)
  const int it0 = h ? 1 : 0, it1 = h ? 2 : 3;
  const int nk0 = 16 - 4 * it0;   // k steps of i-tile it0 (T[i][k] = 0 for k < i)
  double zpf[ZPF], vpf[VPF], tr[20];
  unsigned zmask = 0, vmask = 0;
  for (int sb = nsb - 1; sb >= 0; --sb) {
    const int s0 = BW * sb, nt = nsb - sb;
    for (int t = 0; t < nt; ++t) {
      const int R0 = s0 + 1 + BW * t;
      const int base = BW * t;   // slot of window row m: (base + m) mod 2B
      if (t == 0) {
        // first group of the block: the whole window and its reflectors; the
        // ring's 128th slot (outside every window) is zeroed, so that it never
        // holds uninitialised data (it only meets zero entries of V)
        for (int idx = tid; idx < (2 * BW - 1) * QC; idx += QT) {
          const int m = idx % (2 * BW - 1), c = idx / (2 * BW - 1);
          const long R = (long)R0 + m;
          Zs[(base + m) & (2 * BW - 1)][c] = (R < N && c0 + c < N) ? Z[R + (long)(c0 + c) * ld] : 0.0;
        }
        for (int c = tid; c < QC; c += QT) Zs[(base + 2 * BW - 1) & (2 * BW - 1)][c] = 0.0;
        q2_fetch_V(W, ld, N, s0, R0, vpf, vmask);
      } else {
        // rows 63 .. 126 of this window, fetched during the previous group
#pragma unroll
        for (int u = 0; u < ZPF; ++u) {
          const int idx = tid + QT * u;
          const int m = (BW - 1) + idx % BW, c = idx / BW;
          Zs[(base + m) & (2 * BW - 1)][c] = ((zmask >> u) & 1u) ? zpf[u] : 0.0;
        }
      }
      q2_put_V(vpf, vmask, N, s0, R0, Vs);
      // this group's T: in registers since the previous group's W2 step,
      // except for the first group
      if (sb == nsb - 1 && t == 0) {
        const BSE_GLOBAL double* __restrict__ Tg = gbl(Tbuf) + q2_group(nsb, sb, t) * (BW * BW);
#pragma unroll
        for (int j = 0; j < 20; ++j) {
          const int it = (j < nk0) ? it0 : it1;
          const int k0 = (j < nk0) ? 16 * it0 + 4 * j : 16 * it1 + 4 * (j - nk0);
          tr[j] = Tg[(16 * it + li) + (long)(k0 + kq) * BW];
        }
      }
      // the group after this one: (sb, t + 1), else the first of block sb - 1
      const long gnext = (t + 1 < nt) ? q2_group(nsb, sb, t + 1) : (sb > 0 ? q2_group(nsb, sb - 1, 0) : -1);
      const BSE_GLOBAL double* __restrict__ Tnext = gnext >= 0 ? gbl(Tbuf) + gnext * (BW * BW) : nullptr;
      // the next group's rows and reflectors
      if (t + 1 < nt) {
        q2_fetch_Z(Z, ld, N, c0, R0 + BW, zpf, zmask);
        q2_fetch_V(W, ld, N, s0, R0 + BW, vpf, vmask);
      }
      __syncthreads();
      if (h == 0) q2_products<0>(Zs, Vs, Ws, tr, Tnext, base, cl);
      else q2_products<1>(Zs, Vs, Ws, tr, Tnext, base, cl);
      // rows leaving the window: the first B (a fixed count per thread), or
      // all of it after the block's last group
      if (t + 1 < nt && c0 + QC <= N) {
        // rows R0 .. R0 + 63 lie above row N - 1 when the block has a next
        // group: no bounds to test, straight-line stores
#pragma unroll
        for (int u = 0; u < BW * QC / QT; ++u) {
          const int idx = tid + QT * u;
          const int m = idx % BW, c = idx / BW;
          Z[(long)R0 + m + (long)(c0 + c) * ld] = Zs[(base + m) & (2 * BW - 1)][c];
        }
      } else if (t + 1 < nt) {
#pragma unroll
        for (int u = 0; u < BW * QC / QT; ++u) {
          const int idx = tid + QT * u;
          const int m = idx % BW, c = idx / BW;
          const long R = (long)R0 + m;
          if (R < N && c0 + c < N) Z[R + (long)(c0 + c) * ld] = Zs[(base + m) & (2 * BW - 1)][c];
        }
      } else {
        for (int idx = tid; idx < (2 * BW - 1) * QC; idx += QT) {
          const int m = idx % (2 * BW - 1), c = idx / (2 * BW - 1);
          const long R = (long)R0 + m;
          if (R < N && c0 + c < N) Z[R + (long)(c0 + c) * ld] = Zs[(base + m) & (2 * BW - 1)][c];
        }
      }
      __syncthreads();   // the next group's rows reuse these slots
    }
  }
}

}  // namespace

size_t sbr_q2_T_bytes(long N) {
  const long nsb = q2_nsb(N);
  return (size_t)(nsb * (nsb + 1) / 2) * BW * BW * sizeof(double);
}

int sbr_q2_apply(hipStream_t s, const Batch& b) {
  if (b.count != 1) return set_error(BSE_EUNSUPPORTED, "the two-stage reduction runs one problem at a time");
  const Prob& P = b.host[0];
  const int N = P.N;
  const int nsb = q2_nsb(N);
  if (nsb == 0) return 0;
  const long ng = (long)nsb * (nsb + 1) / 2;
  BSE_LAUNCH(k_sbr_q2T, dim3((unsigned)ng), dim3(256), 0, s, b.dev, P.inv);
  BSE_LAUNCH(k_sbr_q2, dim3((unsigned)((N + QC - 1) / QC)), dim3(QT), 0, s, b.dev, P.inv);
  return 0;
}

int sbr_single(hipStream_t s, const Batch& b, int* work, bool vectors) {
  if (b.count != 1) return set_error(BSE_EUNSUPPORTED, "the two-stage reduction runs one problem at a time");
  const Prob& P = b.host[0];
  const int N = P.N;
  if (N < 2) return 0;
  // work (P.Ycol, ld * ld / 32 ints): progress words [N], the chase's error
  // word, the panels' error word at N + 2, the panel flags from N + 4.  The
  // panels' error word is read after the chase whether or not a panel ran
  // (orders up to BW + 1 have none), so it is cleared first.
  int* flags = work + N + 4;
  if (N - BW >= 2 && (long)N + 4 + PMAX_WG > P.ld * P.ld / 32)
    return set_error(BSE_EUNSUPPORTED, "two-stage reduction: work area too small");
  BSE_LAUNCH(k_sbr_panel_reset, dim3(1), dim3(64), 0, s, nullptr, work + N + 2);
  for (int k0 = 0;; k0 += BW) {
    const int r0 = k0 + BW;
    const int m = N - r0;
    if (m < 2) break;
    const int nr = m - 1 < BW ? m - 1 : BW;
    const unsigned nwg = (unsigned)((m + PR - 1) / PR);
    if (nwg > (unsigned)PMAX_WG) return set_error(BSE_EUNSUPPORTED, "two-stage reduction: order too large");
    BSE_LAUNCH(k_sbr_panel_reset, dim3(1), dim3(PMAX_WG), 0, s, flags, nullptr);
    BSE_LAUNCH(k_sbr_panel, dim3(nwg), dim3(PR), 0, s, b.dev, k0, flags, work + N + 2);
    BSE_LAUNCH(k_sbr_extract, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, b.dev, k0);
    BSE_TRY(gemm_batched(s, b, 1, GOP_SBR_X, k0));
    BSE_TRY(gemm_batched(s, b, 1, GOP_SBR_XT, k0));
    BSE_TRY(gemm_batched(s, b, 1, GOP_SBR_S, k0));
    BSE_LAUNCH(k_sbr_T, dim3(1), dim3(64), 0, s, b.dev, k0);
    BSE_TRY(gemm_batched(s, b, 1, GOP_SBR_Y, k0));
    BSE_TRY(gemm_batched(s, b, 1, GOP_SBR_Z, k0));
    BSE_TRY(gemm_batched(s, b, 1, GOP_SBR_S2, k0));
    BSE_TRY(gemm_batched(s, b, 1, GOP_SBR_YY, k0));
    BSE_LAUNCH(k_sbr_pack, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, b.dev, k0);
    BSE_TRY(gemm_batched(s, b, 1, GOP_SBR_R2K, k0));
  }
  int* prog = work;
  int* err = work + N;
  // the band reduction's reflectors next to the band, kept in Z (free until
  // the eigenvectors are scattered into it: ld x ld >= N x B doubles)
  if (vectors) BSE_LAUNCH(k_sbr_fill, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, b.dev, P.Z, 0);
  BSE_LAUNCH(k_sbr_prepare, dim3((unsigned)((N + 1) / 2)), dim3(256), 0, s, b.dev, prog, err);
  if (N > 2) {
    const unsigned G = (unsigned)(N - 2 < CH_WG ? N - 2 : CH_WG);
    BSE_LAUNCH(k_sbr_chase, dim3(G), dim3(256), 0, s, b.dev, prog, err, vectors ? 1 : 0);
  }
  if (vectors) BSE_LAUNCH(k_sbr_fill, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, b.dev, P.Z, 1);
  BSE_LAUNCH(k_sbr_alpha, dim3((unsigned)((N - 1 + 255) / 256)), dim3(256), 0, s, b.dev);
  int herr[3] = {0, 0, 0};
  BSE_HIP(hipMemcpyAsync(herr, err, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  BSE_HIP(hipStreamSynchronize(s));
  if (herr[0] != 0) return set_error(BSE_EDEVICE, "bulge chasing: a sweep waited too long for its predecessor");
  if (herr[2] != 0) return set_error(BSE_EDEVICE, "two-stage panel: a workgroup waited too long at a column barrier");
  return 0;
}

}  // namespace bse
