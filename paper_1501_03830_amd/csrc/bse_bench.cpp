// Native driver of the C ABI, without Python: times bse_solve on one
// synthetic problem already resident in device memory, or runs a plain
// device copy kernel of known size (used to calibrate HBM byte counters).
//
//   bse_bench solve <n> <solves>     FP64 solve with vectors and weights
//   bse_bench copy <MiB> <launches>  dst[i] = src[i] over MiB of doubles
//
// The synthetic problem has the structure of the benchmark generator: A =
// diag(u), u in [1, 10], plus a Hermitian Gaussian kernel of scale 0.3 /
// sqrt(n); B = complex symmetric Gaussian of scale 0.05 / sqrt(n); a unit
// dipole vector.  Numbers come from a splitmix64 stream (not the Python
// generator), so eigenvalues differ from the Python runs; data-independent
// quantities (kernel durations, bytes moved) do not.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/bse.h"

namespace {

#define CHECK_HIP(x)                                                                  \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      fprintf(stderr, "%s failed: %s (line %d)\n", #x, hipGetErrorString(e_), __LINE__); \
      return 1;                                                                       \
    }                                                                                 \
  } while (0)

struct Rng {
  unsigned long long s;
  unsigned long long next() {
    unsigned long long z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {   // Box-Muller
    double u1 = uniform(), u2 = uniform();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

__global__ void copy_kernel(const double* __restrict__ src, double* __restrict__ dst, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

int run_copy(long mib, int launches) {
  const long n = mib * (1L << 20) / 8;
  double *src, *dst;
  CHECK_HIP(hipMalloc(&src, n * 8));
  CHECK_HIP(hipMalloc(&dst, n * 8));
  CHECK_HIP(hipMemset(src, 0, n * 8));
  for (int i = 0; i < launches; ++i) copy_kernel<<<4096, 256>>>(src, dst, n);
  CHECK_HIP(hipGetLastError());
  CHECK_HIP(hipDeviceSynchronize());
  printf("{\"copy\": {\"bytes_read_per_launch\": %ld, \"bytes_written_per_launch\": %ld, \"launches\": %d}}\n",
         n * 8, n * 8, launches);
  CHECK_HIP(hipFree(src));
  CHECK_HIP(hipFree(dst));
  return 0;
}

int run_solve(int n, int solves) {
  const long nn = (long)n * n;
  std::vector<double> A(2 * nn, 0.0), B(2 * nn, 0.0), d(4L * n);
  Rng rng{12345};
  const double sa = 0.3 / std::sqrt((double)n), sb = 0.05 / std::sqrt((double)n);
  // column-major lower triangles (the solver reads only those)
  for (int j = 0; j < n; ++j) {
    A[2 * ((long)j + (long)j * n)] = 1.0 + 9.0 * rng.uniform() + sa * rng.normal();
    for (int i = j + 1; i < n; ++i) {
      A[2 * ((long)i + (long)j * n)] = sa * rng.normal() * 0.7071067811865476;
      A[2 * ((long)i + (long)j * n) + 1] = sa * rng.normal() * 0.7071067811865476;
    }
    for (int i = j; i < n; ++i) {
      B[2 * ((long)i + (long)j * n)] = sb * rng.normal() * 0.7071067811865476;
      B[2 * ((long)i + (long)j * n) + 1] = sb * rng.normal() * 0.7071067811865476;
    }
  }
  double nrm = 0.0;
  for (auto& x : d) {
    x = rng.normal();
    nrm += x * x;
  }
  for (auto& x : d) x /= std::sqrt(nrm);
  double *dA, *dB, *dd, *lam, *X, *w;
  CHECK_HIP(hipMalloc(&dA, 16 * nn));
  CHECK_HIP(hipMalloc(&dB, 16 * nn));
  CHECK_HIP(hipMalloc(&dd, 32L * n));
  CHECK_HIP(hipMalloc(&lam, 8L * n));
  CHECK_HIP(hipMalloc(&X, 32 * nn));
  CHECK_HIP(hipMalloc(&w, 16L * n));
  CHECK_HIP(hipMemcpy(dA, A.data(), 16 * nn, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dB, B.data(), 16 * nn, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dd, d.data(), 32L * n, hipMemcpyHostToDevice));
  bse_ctx* ctx = nullptr;
  if (bse_ctx_create(&ctx, 0, nullptr, 0, nullptr) != 0) {
    fprintf(stderr, "bse_ctx_create: %s\n", bse_last_error());
    return 1;
  }
  for (int k = 0; k < solves; ++k) {
    bse_report rep;
    const auto t0 = std::chrono::steady_clock::now();
    const int info = bse_solve(ctx, n, dA, n, dB, n, BSE_PREC_FP64, BSE_WANT_VECTORS | BSE_WANT_WEIGHTS, lam, X,
                               2 * n, dd, nullptr, w, &rep);
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info != 0) {
      fprintf(stderr, "bse_solve returned %d: %s\n", info, bse_last_error());
      return 1;
    }
    printf("{\"solve\": %d, \"n\": %d, \"s\": %.4f, \"device_ms\": %.2f, \"sktrd_ms\": %.2f}\n", k, n, s,
           rep.total_ms, rep.stage_ms[BSE_STAGE_SKTRD]);
    fflush(stdout);
  }
  bse_ctx_destroy(ctx);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 4) {
    fprintf(stderr, "usage: %s solve <n> <solves> | copy <MiB> <launches>\n", argv[0]);
    return 2;
  }
  if (!strcmp(argv[1], "copy")) return run_copy(atol(argv[2]), atoi(argv[3]));
  if (!strcmp(argv[1], "solve")) return run_solve(atoi(argv[2]), atoi(argv[3]));
  fprintf(stderr, "unknown mode %s\n", argv[1]);
  return 2;
}
