// FP64 matrix multiply on the gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
//   C = alpha * op(A) * op(B) + beta * C      (column-major)
//
// Used for every dense contraction of the chain: the Cholesky trailing
// update, W = L^T J L, the skew rank-2k update of the tridiagonalisation,
// the block-reflector applications, the products with L and the Gram
// matrices of the reorthogonalisation.  Options:
//   c_uplo  0: full C;  1: lower triangle incl. diagonal;  2: strictly lower
//           (only tiles touching the requested triangle are launched)
//   a_tri   the stored A is lower triangular: the K loop skips its zeros
//   b_tri   the stored B is lower triangular
//
// Tiling: a 256-thread workgroup (4 wavefronts in a 2 x 2 arrangement) owns a
// 64 x 64 or 128 x 128 C tile (each wave 2 x 2 or 4 x 4 MFMA blocks of
// 16 x 16); K steps of 16 are staged through LDS with a register prefetch of
// the next slab.  The epilogue goes through LDS so that C is read and written
// a whole column (64 or 128 consecutive doubles) per instruction.  Products
// with few output tiles and a long K (V^T Z in the reflector application)
// are split along K into a scratch buffer and summed by a second kernel.
#include <cstdlib>

#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int BK = 16, PAD = 2;

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
  int tiles_m, tiles_n;
  int splits, kchunk;
  double* part;  // split-K partial products [splits][M x N], ld M
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int BM, int BN, bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmParams p) {
  constexpr int WM = BM / 2, WN = BN / 2;   // sub-tile of one wave
  constexpr int FM = WM / 16, FN = WN / 16; // MFMA blocks per wave
  constexpr int AS = BK * (BM + PAD), BS = BK * (BN + PAD);
  constexpr int EPC = 64;                   // columns per epilogue pass
  constexpr int CS = EPC * (BM + 1);
  constexpr int SMEM = cmax(2 * (AS + BS), CS);
  __shared__ double smem[SMEM];
  // LDS layout: A buffers at [0, 2 AS), B buffers at [2 AS, 2 AS + 2 BS)

  int tile = blockIdx.x, slice = 0;
  if (p.splits > 1) {
    slice = tile % p.splits;
    tile /= p.splits;
  }
  int tm, tn;
  if (p.c_uplo) {
    tri_index(tile, tm, tn);
  } else {
    tm = tile % p.tiles_m;
    tn = tile / p.tiles_m;
  }
  const int i0 = tm * BM, j0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;

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
    if (!TA) {  // A[i + k lda]: BK columns of BM contiguous rows
      constexpr int TPC = BM / EA;      // threads per column
      const int kk = tid / TPC, ii = (tid % TPC) * EA;
      const int k = k0 + kk;
#pragma unroll
      for (int q = 0; q < EA; ++q) {
        const int i = i0 + ii + q;
        ra[q] = (i < p.M && k < kend) ? p.A[(long)i + (long)k * p.lda] : 0.0;
      }
    } else {    // A[k + i lda]: BM columns of BK contiguous rows
      constexpr int TPC = BK / EA;
      const int ii = tid / TPC, kk = (tid % TPC) * EA;
      const int i = i0 + ii;
#pragma unroll
      for (int q = 0; q < EA; ++q) {
        const int k = k0 + kk + q;
        ra[q] = (i < p.M && k < kend) ? p.A[(long)k + (long)i * p.lda] : 0.0;
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
    if (!TB) {  // B[k + j ldb]: BN columns of BK contiguous rows
      constexpr int TPC = BK / EB;
      const int jj = tid / TPC, kk = (tid % TPC) * EB;
      const int j = j0 + jj;
#pragma unroll
      for (int q = 0; q < EB; ++q) {
        const int k = k0 + kk + q;
        rb[q] = (j < p.N && k < kend) ? p.B[(long)k + (long)j * p.ldb] : 0.0;
      }
    } else {    // B[j + k ldb]: BK columns of BN contiguous rows
      constexpr int TPC = BN / EB;
      const int kk = tid / TPC, jj = (tid % TPC) * EB;
      const int k = k0 + kk;
#pragma unroll
      for (int q = 0; q < EB; ++q) {
        const int j = j0 + jj + q;
        rb[q] = (j < p.N && k < kend) ? p.B[(long)j + (long)k * p.ldb] : 0.0;
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

  // Epilogue through LDS, EPC columns at a time.  In a 16 x 16 f64 block the
  // entry (i, j) lives in lane 16 (i mod 4) + j, accumulator element i / 4.
  double* Cs = smem;  // Cs[c * (BM + 1) + r]
  const bool split = p.splits > 1;
#pragma unroll
  for (int c0 = 0; c0 < BN; c0 += EPC) {
    __syncthreads();
    if (wc * WN >= c0 && wc * WN < c0 + EPC) {
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          const int cl = wc * WN + b * 16 + (lane & 15) - c0;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rl = wr * WM + a * 16 + (lane >> 4) + 4 * v;
            Cs[cl * (BM + 1) + rl] = acc[a][b][v];
          }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < EPC * BM; idx += 256) {
      const int rl = idx % BM, cl = idx / BM;
      const int row = i0 + rl, col = j0 + c0 + cl;
      if (row >= p.M || col >= p.N) continue;
      if (p.c_uplo == 1 && row < col) continue;
      if (p.c_uplo == 2 && row <= col) continue;
      const double val = Cs[cl * (BM + 1) + rl];
      if (split) {
        p.part[(long)slice * p.M * p.N + (long)row + (long)col * p.M] = val;
      } else {
        double* c = p.C + (long)row + (long)col * p.ldc;
        const double out = p.alpha * val;
        *c = (p.beta == 0.0) ? out : out + p.beta * (*c);
      }
    }
  }
}

// C = alpha * sum_s part[s] + beta * C over the (uplo-restricted) M x N
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmParams p) {
  const long r = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const long c0 = (long)blockIdx.y * 64 + (threadIdx.x >> 6) * 16;
  if (r >= p.M) return;
  for (int q = 0; q < 16; ++q) {
    const long c = c0 + q;
    if (c >= p.N) break;
    if (p.c_uplo == 1 && r < c) continue;
    if (p.c_uplo == 2 && r <= c) continue;
    double s = 0.0;
    for (int k = 0; k < p.splits; ++k) s += p.part[(long)k * p.M * p.N + r + c * p.M];
    double* cp = p.C + r + c * p.ldc;
    const double out = p.alpha * s;
    *cp = (p.beta == 0.0) ? out : out + p.beta * (*cp);
  }
}

template <int BM, int BN>
void launch(hipStream_t s, bool ta, bool tb, dim3 grid, const GemmParams& p) {
  if (!ta && !tb) gemm_f64_kernel<BM, BN, false, false><<<grid, 256, 0, s>>>(p);
  else if (!ta && tb) gemm_f64_kernel<BM, BN, false, true><<<grid, 256, 0, s>>>(p);
  else if (ta && !tb) gemm_f64_kernel<BM, BN, true, false><<<grid, 256, 0, s>>>(p);
  else gemm_f64_kernel<BM, BN, true, true><<<grid, 256, 0, s>>>(p);
}

thread_local double* g_scratch = nullptr;
thread_local size_t g_scratch_bytes = 0;

}  // namespace

void gemm_set_scratch(double* scratch, size_t bytes) {
  g_scratch = scratch;
  g_scratch_bytes = bytes;
}

int gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
             long lda, const double* B, long ldb, double beta, double* C, long ldc, int c_uplo,
             int a_tri, int b_tri) {
  if (M <= 0 || N <= 0) return 0;
  if (c_uplo && M != N)
    return set_hip_error(hipErrorInvalidValue, "gemm: triangular C must be square", __FILE__, __LINE__);
  GemmParams p;
  p.M = M;
  p.N = N;
  p.K = K < 0 ? 0 : K;
  p.A = A;
  p.lda = lda;
  p.B = B;
  p.ldb = ldb;
  p.C = C;
  p.ldc = ldc;
  p.alpha = alpha;
  p.beta = beta;
  p.c_uplo = c_uplo;
  p.a_tri = a_tri;
  p.b_tri = b_tri;
  p.splits = 1;
  p.kchunk = p.K;
  p.part = nullptr;
  // large, compute-bound products use 128 x 128 tiles
  const long t128 = (long)((M + 127) / 128) * ((N + 127) / 128);
  // (measured on gfx950: at one wave per SIMD the 128 x 128 tile is slower than
  // 64 x 64 at four, so it is only selected when BSE_GEMM128 is set)
  static const bool allow128 = getenv("BSE_GEMM128") != nullptr;
  const bool big = allow128 && M >= 256 && N >= 256 && K >= 256 && (c_uplo ? t128 / 2 : t128) >= 512;
  const int BMs = big ? 128 : 64;
  p.tiles_m = (M + BMs - 1) / BMs;
  p.tiles_n = (N + BMs - 1) / BMs;
  long ntiles = c_uplo ? (long)p.tiles_m * (p.tiles_m + 1) / 2 : (long)p.tiles_m * p.tiles_n;
  // few output tiles and a long K: split K (partials in the scratch buffer)
  if (!big && ntiles < 512 && p.K >= 2048 && g_scratch != nullptr) {
    int splits = (int)((1024 + ntiles - 1) / ntiles);
    splits = splits > 16 ? 16 : splits;
    const int maxk = p.K / 512;
    splits = splits > maxk ? maxk : splits;
    while (splits > 1 && (size_t)splits * M * N * sizeof(double) > g_scratch_bytes) --splits;
    if (splits > 1) {
      p.splits = splits;
      p.kchunk = round_up((p.K + splits - 1) / splits, BK);
      p.part = g_scratch;
    }
  }
  const dim3 grid((unsigned)(ntiles * p.splits));
  if (big) launch<128, 128>(s, ta, tb, grid, p);
  else launch<64, 64>(s, ta, tb, grid, p);
  BSE_LAUNCHED();
  if (p.splits > 1) {
    k_splitk_reduce<<<dim3((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64)), 256, 0, s>>>(p);
    BSE_LAUNCHED();
  }
  return 0;
}

}  // namespace bse
