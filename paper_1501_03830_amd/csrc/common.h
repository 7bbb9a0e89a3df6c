// Shared definitions for the gfx950 kernels of the Bethe-Salpeter solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/bse.h"

namespace bse {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// Leading dimension used for every N x N device matrix: a multiple of 64 so
// that 64 x 64 tiles are aligned, with all tiles of the padded square
// allocated (kernels read whole tiles and mask, they never read past ld x ld).
inline long round_up(long x, long m) { return (x + m - 1) / m * m; }
// Leading dimension of every N x N matrix of a problem: whole 64 x 64 tiles
// (a padded leading dimension measured slower for the matvec).
inline long square_ld(long N) { return round_up(N < 64 ? 64 : N, 64); }

// Record a HIP failure for bse_last_error() and turn it into BSE_EDEVICE.
int set_hip_error(hipError_t e, const char* what, const char* file, int line);
// Record a message for bse_last_error() and return code.
int set_error(int code, const char* msg);

// Host-only dry run of a launch plan (bse_plan_check): while it is on for
// the calling thread, runtime calls wrapped in BSE_HIP are skipped and
// kernels are checked but not launched.
bool dry_run();

#define BSE_HIP(call)                                                        \
  do {                                                                       \
    if (!::bse::dry_run()) {                                                 \
      hipError_t e_ = (call);                                                \
      if (e_ != hipSuccess) return ::bse::set_hip_error(e_, #call, __FILE__, __LINE__); \
    }                                                                        \
  } while (0)

#define BSE_LAUNCHED()                                                       \
  do {                                                                       \
    hipError_t e_ = hipGetLastError();                                       \
    if (e_ != hipSuccess) return ::bse::set_hip_error(e_, "kernel launch", __FILE__, __LINE__); \
  } while (0)

#define BSE_TRY(expr)                                                        \
  do {                                                                       \
    int rc_ = (expr);                                                        \
    if (rc_ != 0) return rc_;                                                \
  } while (0)

// Every kernel launch is checked against the device's dispatch limits first
// (grid dimensions >= 1, grid x workgroup within the 32-bit work-item count
// of a dispatch packet in each dimension, workgroup <= 1024 work-items,
// dynamic LDS <= 160 KiB, kernel arguments <= 4 KiB) and recorded for the
// dry run; a violation is an error (BSE_EDEVICE with the kernel's name), not
// a dispatch.
int check_launch(const char* name, dim3 grid, dim3 block, size_t dyn_lds, size_t kernarg_bytes);

template <class... P>
constexpr size_t kernarg_bytes() {
  size_t off = 0;
  ((off = (off + alignof(P) - 1) / alignof(P) * alignof(P) + sizeof(P)), ...);
  return off;
}

template <class... P, class... A>
inline int launch_kernel(const char* name, void (*kern)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s,
                         A&&... args) {
  BSE_TRY(check_launch(name, grid, block, lds, kernarg_bytes<P...>()));
  if (dry_run()) return 0;
  kern<<<grid, block, lds, s>>>(static_cast<P>(args)...);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_hip_error(e, name, __FILE__, __LINE__);
  return 0;
}

// kernel<<<grid, block, lds, stream>>>(args...), checked; a kernel name with
// template arguments goes in parentheses
#define BSE_LAUNCH(kern, ...) BSE_TRY(::bse::launch_kernel(#kern, kern, __VA_ARGS__))

// Everything one problem of a (possibly one-element) batch needs on the
// device: its sizes, the caller's input/output buffers and its own slice of
// the workspace.  Kernels read it from a device array indexed by the problem
// number (blockIdx.z), so one launch can serve many problems of different
// sizes.
struct Prob {
  int n, N;             // order of A and B, and of the real embedding (N = 2n)
  long ld;              // leading dimension of every N x N workspace matrix
  const double* A;      // complex n x n, column-major, lower triangle used
  long lda;
  const double* B;
  long ldb;
  double* lambda;       // n positive eigenvalues (output)
  double* X;            // complex 2n x n (output) or null
  long ldx;
  const double* dr;     // complex 2n dipoles or null
  const double* dl;
  double* w;            // complex n weights (output) or null
  unsigned flags;
  int uoff;             // reflector k of the back-transformation acts on rows k + uoff ..:
                        // SBR_B after the two-stage reduction, 1 (or 0) after the one-stage one
  // workspace
  double *L, *W, *Z, *Vt, *inv, *alpha, *tau, *e2, *scal, *shift, *gscr;
  size_t gscr_bytes;
  int* cid;
  int* info;            // info[0]: Cholesky of M, info[1]: Cholesky of the Gram matrix
  // tridiagonalisation work
  double *Y1, *Y2, *Yrow, *Ycol, *dotpart, *normpart;
  void* ctrl;
  // back-transformation work
  double *Vb, *S, *W1, *W2;
  float *Vb32, *W2f;    // FP32 copies of Vb and W2 (mixed precision)
  float* Z32;           // FP32 basis of the mixed-precision back-transformation (in R4)
  // mixed-precision path (prec == BSE_PREC_FP32_REFINE)
  int prec;
  float* W32;           // FP32 copy of W reduced to tridiagonal form (ld x ld)
  float *Y1f, *Y2f;     // FP32 copies of Y1, Y2 for the rank-2k update (in R3)
  double *R1, *R2, *R3, *R4;   // refinement work, ld x ld each
  double* refmax;       // refinement: per-tile partial maxima (2 per tile)
  double* refout;       // refinement: [largest correction, clamped pairs] (header)
  int* refstate;        // refinement: sweeps done once converged, else 0 (header)
  int* reorth;          // 1: run the cluster Gram-Schmidt (header)
  double* gdef;         // largest |G - I| inside a cluster, first pass (header)
  int* perm;            // n: output column j takes eigenpair perm[j]
  // refinement clusters of close pairs (mixed-precision path)
  int* clstart;         // n: first pair of the cluster of pair k
  int* clflag;          // n: at a cluster's first pair, 1 when it needs the exact rotation
  double* clmax;        // n: at a cluster's first pair, largest entry of its rotation minus I
  double* clT;          // n x REF_CMAX4 doubles: the rotation of the cluster starting at pair k
  // real problems (FLAG_REAL_IN): A, B real n x n; X is assembled in the
  // workspace and its real part written to Xr (2n x n doubles, ld ldxr)
  double* Xr;
  long ldxr;
};

// Internal descriptor flag (beside BSE_WANT_*): A and B are real (FP64)
// matrices, the real Bethe-Salpeter problem of eq. H-real (Algorithm 2).
constexpr unsigned FLAG_REAL_IN = 1u << 16;

// Refinement clusters: at most this many pairs (a 2c x 2c rotation per
// cluster, stored in 4 c_max^2 doubles at the cluster's first pair's slot).
constexpr int REF_CMAX = 16;
constexpr int REF_CMAX4 = 4 * REF_CMAX;

// info[1] value of a mixed-precision problem whose refinement did not reach
// its stopping test within the sweep limit (a Gram-Schmidt failure is > 0).
constexpr int INFO_NOCONV = -1;

// Address-space views of pointers taken from a descriptor.  A pointer loaded
// from memory is generic to the compiler, which then emits flat instructions
// (they also hold the LDS counter, so LDS waits stall on global loads) and
// never scalar loads.  Every buffer here is global memory, so kernels re-type
// descriptor pointers with gbl(); ro() additionally declares the data
// read-only for the whole kernel (no thread of the launch writes it), which
// lets wave-uniform reads use the scalar cache.
#define BSE_GLOBAL __attribute__((address_space(1)))
#define BSE_CONST __attribute__((address_space(4)))
template <class T>
__device__ inline BSE_GLOBAL T* gbl(T* p) {
  return (BSE_GLOBAL T*)p;
}
template <class T>
__device__ inline const BSE_CONST T* ro(const T* p) {
  return (const BSE_CONST T*)p;
}

// Row/column decomposition of a linear index over the lower triangle of an
// nt x nt tile grid: t = R (R + 1) / 2 + C with 0 <= C <= R < nt.
__device__ inline void tri_index(long t, int& R, int& C) {
  long r = (long)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  R = (int)r;
  C = (int)(t - r * (r + 1) / 2);
}

// A value known to be equal in every lane, moved to scalar registers.
__device__ inline double uniform_double(double x) {
  const unsigned long long u = __double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(u & 0xffffffffu));
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a wavefront; every lane gets the total.
__device__ inline double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum for blockDim.x <= 1024 (multiple of 64).  `red` must hold
// blockDim.x / 64 doubles.  Every thread returns the total.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

}  // namespace bse
