// Solver driver and C ABI: stage sequencing, workspace layout, argument
// checking and timing for the chain of Algorithm 1 / Algorithm 3.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

struct bse_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void* arena = nullptr;        // caller-provided workspace (not owned)
  size_t arena_bytes = 0;
  void* own = nullptr;          // library-owned workspace
  size_t own_bytes = 0;
  hipEvent_t ev[BSE_NUM_STAGES + 1] = {};
  bool events = false;
  bool timing = false;               // per-launch timing of the skew matvec
  std::vector<hipEvent_t> kev;       // event pool for it
};

namespace bse {

namespace {
thread_local std::string g_last_error;
}

long ld_pad() {
  static long pad = [] {
    const char* e = getenv("BSE_LD_PAD");
    long v = e ? atol(e) : 0;
    if (v < 0) v = 0;
    return round_up(v, 64);
  }();
  return pad;
}

int set_hip_error(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  g_last_error = buf;
  return BSE_EDEVICE;
}

static int set_error(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

// ------------------------------------------------------------------------
// Workspace layout for one solve of order n (N = 2n), FP64.
// ------------------------------------------------------------------------
struct Plan {
  long N = 0, n = 0, ld = 0;
  size_t off_L = 0, off_W = 0, off_Z = 0, off_Vt = 0, off_inv = 0, off_small = 0, off_sk = 0,
         off_bt = 0, off_linv = 0, off_gscr = 0;
  size_t gscr_bytes = 0;
  size_t total = 0;
  int nb = 64, nbq = 64;
};

static Plan make_plan(long N) {
  Plan p;
  p.N = N;
  p.n = N / 2;
  p.ld = square_ld(N);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    size_t o = cur;
    cur += (size_t)round_up((long)bytes, 256);
    return o;
  };
  const size_t sq = (size_t)p.ld * p.ld * sizeof(double);
  p.off_L = take(sq);
  p.off_W = take(sq);
  p.off_Z = take(sq);
  p.off_Vt = take((size_t)p.n * N * sizeof(double));
  // inverse iteration factors (4 double arrays + 1 byte array, N x n each);
  // later reused for the n x n Gram matrix of the reorthogonalisation
  p.off_inv = take((size_t)4 * N * p.n * sizeof(double) + (size_t)N * p.n + 256);
  p.off_small = take((size_t)(4 * p.ld + 3 * p.n + 64) * sizeof(double));
  p.off_sk = take(sktrd_work_bytes(N, p.ld, p.nb));
  p.off_bt = take(backtr_work_bytes(N, p.ld, p.nbq));
  p.off_linv = take(64 * 64 * sizeof(double));
  p.gscr_bytes = (size_t)16 * 64 * p.ld * sizeof(double);   // split-K partials
  p.off_gscr = take(p.gscr_bytes);
  p.total = cur;
  return p;
}

struct Bufs {
  double *L, *W, *Z, *Vt, *inv, *alpha, *tau, *e2, *scal, *shift, *lam_tmp, *linv;
  int *cid, *info;
  SktrdWork sk;
  BacktrWork bt;
};

static void bind(const Plan& p, char* base, Bufs* b) {
  b->L = reinterpret_cast<double*>(base + p.off_L);
  b->W = reinterpret_cast<double*>(base + p.off_W);
  b->Z = reinterpret_cast<double*>(base + p.off_Z);
  b->Vt = reinterpret_cast<double*>(base + p.off_Vt);
  b->inv = reinterpret_cast<double*>(base + p.off_inv);
  double* sm = reinterpret_cast<double*>(base + p.off_small);
  b->alpha = sm;
  b->tau = sm + p.ld;
  b->e2 = sm + 2 * p.ld;
  b->lam_tmp = sm + 3 * p.ld;
  b->shift = sm + 4 * p.ld;
  b->scal = sm + 4 * p.ld + p.n;
  b->cid = reinterpret_cast<int*>(sm + 4 * p.ld + p.n + 16);
  b->info = reinterpret_cast<int*>(sm + 4 * p.ld + 3 * p.n + 32);
  b->linv = reinterpret_cast<double*>(base + p.off_linv);
  gemm_set_scratch(reinterpret_cast<double*>(base + p.off_gscr), p.gscr_bytes);
  sktrd_bind_work(base + p.off_sk, p.N, p.ld, p.nb, &b->sk);
  backtr_bind_work(base + p.off_bt, p.N, p.ld, p.nbq, &b->bt);
}

static int get_workspace(bse_ctx* ctx, size_t bytes, char** base) {
  if (ctx->arena) {
    if (bytes > ctx->arena_bytes) return set_error(BSE_ENOMEM, "workspace exceeds the caller's arena");
    *base = static_cast<char*>(ctx->arena);
    return 0;
  }
  if (ctx->own_bytes < bytes) {
    if (ctx->own) {
      BSE_HIP(hipStreamSynchronize(ctx->stream));
      BSE_HIP(hipFree(ctx->own));
      ctx->own = nullptr;
      ctx->own_bytes = 0;
    }
    BSE_HIP(hipMalloc(&ctx->own, bytes));
    ctx->own_bytes = bytes;
  }
  *base = static_cast<char*>(ctx->own);
  return 0;
}

static int ensure_events(bse_ctx* ctx) {
  if (ctx->events) return 0;
  for (int i = 0; i <= BSE_NUM_STAGES; ++i) BSE_HIP(hipEventCreate(&ctx->ev[i]));
  ctx->events = true;
  return 0;
}

static int mark(bse_ctx* ctx, bool timed, int i) {
  if (timed) BSE_HIP(hipEventRecord(ctx->ev[i], ctx->stream));
  return 0;
}

static int read_info(bse_ctx* ctx, const int* info_dev, int* info) {
  BSE_HIP(hipMemcpyAsync(info, info_dev, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  BSE_HIP(hipStreamSynchronize(ctx->stream));
  return 0;
}

// The chain for one problem.  lambda: device n doubles.  X: device complex
// 2n x n (ldx in complex elements) or NULL.
static int solve_fp64(bse_ctx* ctx, int n, const double* A, long lda, const double* B, long ldb,
                      unsigned flags, double* lambda, double* X, long ldx, const double* dr,
                      const double* dl, double* w, bse_report* rep) {
  const long N = 2L * n;
  const Plan p = make_plan(N);
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, p.total, &base));
  Bufs b;
  bind(p, base, &b);
  hipStream_t s = ctx->stream;
  const bool timed = rep != nullptr;
  if (timed) BSE_TRY(ensure_events(ctx));
  const bool vectors = (flags & BSE_WANT_VECTORS) != 0 && X != nullptr;

  BSE_TRY(mark(ctx, timed, 0));
  BSE_TRY(launch_build_M(s, n, A, lda, B, ldb, b.L, p.ld));
  BSE_TRY(mark(ctx, timed, 1));
  BSE_TRY(potrf_f64(s, (int)N, b.L, p.ld, b.info, b.linv));
  BSE_TRY(mark(ctx, timed, 2));
  int info = 0;
  BSE_TRY(read_info(ctx, b.info, &info));
  if (info != 0) return info;
  BSE_TRY(form_W(s, (int)N, b.L, p.ld, b.W, p.ld, false));
  BSE_TRY(mark(ctx, timed, 3));
  KernelTimer ktimer;
  if (ctx->timing) {
    const size_t need = 2 * (size_t)(N > 2 ? N - 2 : 0);
    while (ctx->kev.size() < need) {
      hipEvent_t e;
      BSE_HIP(hipEventCreate(&e));
      ctx->kev.push_back(e);
    }
    ktimer.ev = ctx->kev.data();
    ktimer.cap = (int)ctx->kev.size();
  }
  BSE_TRY(sktrd_f64(s, (int)N, b.W, p.ld, b.alpha, b.tau, b.sk, ctx->timing ? &ktimer : nullptr));
  BSE_TRY(mark(ctx, timed, 4));
  BSE_TRY(tridiag_bisect(s, (int)N, b.alpha, b.e2, b.scal, lambda));
  BSE_TRY(mark(ctx, timed, 5));
  if (vectors) {
    BSE_TRY(tridiag_invit(s, (int)N, b.alpha, b.scal, lambda, b.shift, b.inv, b.Vt));
    BSE_TRY(mark(ctx, timed, 6));
    BSE_TRY(tridiag_reorth(s, (int)N, lambda, b.scal, b.Vt, b.inv, b.cid, b.info, b.linv));
    BSE_TRY(mark(ctx, timed, 7));
    BSE_TRY(scatter_DV(s, (int)N, b.Vt, b.Z, p.ld));
    BSE_TRY(apply_U(s, (int)N, b.W, p.ld, b.tau, b.Z, p.ld, (int)N, b.bt));
    BSE_TRY(mark(ctx, timed, 8));
    // G = L Z into the W buffer (the reflectors are no longer needed)
    BSE_TRY(gemm_f64(s, false, false, (int)N, (int)N, (int)N, 1.0, b.L, p.ld, b.Z, p.ld, 0.0, b.W, p.ld, 0,
                     1, 0));
    BSE_TRY(mark(ctx, timed, 9));
    BSE_TRY(finish_X(s, n, b.W, p.ld, lambda, X, ldx));
    const bool weights = (flags & BSE_WANT_WEIGHTS) != 0 && dr != nullptr && w != nullptr;
    BSE_TRY(phase_and_weights(s, n, X, ldx, weights ? dr : nullptr, weights ? (dl ? dl : dr) : nullptr,
                              weights ? w : nullptr));
  } else {
    for (int i = 6; i <= 9; ++i) BSE_TRY(mark(ctx, timed, i));
  }
  BSE_TRY(mark(ctx, timed, 10));
  BSE_HIP(hipStreamSynchronize(s));
  if (vectors) {
    BSE_TRY(read_info(ctx, b.info, &info));
    if (info != 0) return set_error(BSE_EDEVICE, "cluster Gram matrix not positive definite");
  }
  if (timed) {
    memset(rep, 0, sizeof(*rep));
    float ms = 0.f;
    for (int i = 0; i < BSE_NUM_STAGES; ++i) {
      BSE_HIP(hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]));
      rep->stage_ms[i] = ms;
    }
    BSE_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[BSE_NUM_STAGES]));
    rep->total_ms = ms;
    rep->n = n;
    rep->prec = BSE_PREC_FP64;
    rep->workspace_bytes = p.total;
    if (ctx->timing) {
      double tot = 0.0;
      for (int i = 0; i + 1 < ktimer.used; i += 2) {
        BSE_HIP(hipEventElapsedTime(&ms, ktimer.ev[i], ktimer.ev[i + 1]));
        tot += ms;
      }
      rep->symv_ms = tot;
      rep->symv_bytes = ktimer.bytes;
      rep->symv_launches = ktimer.used / 2;
    }
  }
  return 0;
}

static int prologue(bse_ctx* ctx) {
  if (!ctx) return set_error(-1, "null context");
  BSE_HIP(hipSetDevice(ctx->device));
  return 0;
}

}  // namespace bse

using namespace bse;

extern "C" {

int bse_version(void) { return 100; }

const char* bse_last_error(void) { return g_last_error.c_str(); }

int bse_ctx_create(bse_ctx** ctx, int device, void* arena, size_t arena_bytes, void* stream) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  *ctx = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) return set_hip_error(e == hipSuccess ? hipErrorNoDevice : e, "hipGetDeviceCount", __FILE__, __LINE__);
  if (device < 0 || device >= count) return set_error(-2, "invalid device");
  if (!arena && arena_bytes) return set_error(-4, "arena_bytes without arena");
  BSE_HIP(hipSetDevice(device));
  bse_ctx* c = new bse_ctx();
  c->device = device;
  c->arena = arena;
  c->arena_bytes = arena_bytes;
  c->stream = static_cast<hipStream_t>(stream);
  *ctx = c;
  return 0;
}

int bse_ctx_destroy(bse_ctx* ctx) {
  if (!ctx) return 0;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->own) (void)hipFree(ctx->own);
  if (ctx->events)
    for (int i = 0; i <= BSE_NUM_STAGES; ++i) (void)hipEventDestroy(ctx->ev[i]);
  for (hipEvent_t e : ctx->kev) (void)hipEventDestroy(e);
  delete ctx;
  return 0;
}

int bse_ctx_set_timing(bse_ctx* ctx, int enable) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  ctx->timing = enable != 0;
  return 0;
}

size_t bse_footprint_bytes(int n, int prec, unsigned flags) {
  (void)flags;
  if (n <= 0 || prec != BSE_PREC_FP64) return 0;
  return make_plan(2L * n).total;
}

int bse_solve(bse_ctx* ctx, int n, const void* A, int lda, const void* B, int ldb, int prec,
              unsigned flags, double* lambda, void* X, int ldx, const void* d_r, const void* d_l,
              void* w, bse_report* rep) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (n <= 0) return set_error(-2, "n must be positive");
  if (!A) return set_error(-3, "A is NULL");
  if (lda < n) return set_error(-4, "lda < n");
  if (!B) return set_error(-5, "B is NULL");
  if (ldb < n) return set_error(-6, "ldb < n");
  if (prec != BSE_PREC_FP64) return set_error(-7, "unsupported precision policy");
  if (flags & ~(BSE_WANT_VECTORS | BSE_WANT_WEIGHTS)) return set_error(-8, "unknown flags");
  if (!lambda) return set_error(-9, "lambda is NULL");
  const bool vec = (flags & BSE_WANT_VECTORS) != 0;
  const bool wts = (flags & BSE_WANT_WEIGHTS) != 0;
  if (wts && !vec) return set_error(-8, "weights need eigenvectors");
  if (vec && !X) return set_error(-10, "X is NULL");
  if (vec && ldx < 2 * n) return set_error(-11, "ldx < 2n");
  if (wts && !d_r) return set_error(-12, "d_r is NULL");
  if (wts && !w) return set_error(-14, "w is NULL");
  BSE_TRY(prologue(ctx));
  return solve_fp64(ctx, n, static_cast<const double*>(A), lda, static_cast<const double*>(B), ldb, flags,
                    lambda, static_cast<double*>(X), ldx, static_cast<const double*>(d_r),
                    static_cast<const double*>(d_l), static_cast<double*>(w), rep);
}

// ---------------------------------------------------------------- stages

int bse_build_M(bse_ctx* ctx, int n, const void* A, int lda, const void* B, int ldb, double* M, int ldm) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (n <= 0) return set_error(-2, "n must be positive");
  if (!A) return set_error(-3, "A is NULL");
  if (lda < n) return set_error(-4, "lda < n");
  if (!B) return set_error(-5, "B is NULL");
  if (ldb < n) return set_error(-6, "ldb < n");
  if (!M) return set_error(-7, "M is NULL");
  if (ldm < 2 * n) return set_error(-8, "ldm < 2n");
  BSE_TRY(prologue(ctx));
  BSE_TRY(launch_build_M(ctx->stream, n, static_cast<const double*>(A), lda, static_cast<const double*>(B), ldb,
                         M, ldm));
  BSE_HIP(hipStreamSynchronize(ctx->stream));
  return 0;
}

int bse_potrf(bse_ctx* ctx, int N, double* M, int ldm) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (N <= 0) return set_error(-2, "N must be positive");
  if (!M) return set_error(-3, "M is NULL");
  if (ldm < N) return set_error(-4, "ldm < N");
  BSE_TRY(prologue(ctx));
  const Plan p = make_plan(N);
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, p.total, &base));
  Bufs b;
  bind(p, base, &b);
  hipStream_t s = ctx->stream;
  BSE_TRY(copy_matrix(s, N, N, M, ldm, b.L, p.ld));
  BSE_TRY(zero_upper(s, N, b.L, p.ld));
  BSE_TRY(potrf_f64(s, N, b.L, p.ld, b.info, b.linv));
  BSE_TRY(copy_matrix(s, N, N, b.L, p.ld, M, ldm));
  int info = 0;
  BSE_TRY(read_info(ctx, b.info, &info));
  return info;
}

int bse_form_W(bse_ctx* ctx, int N, const double* L, int ldl, double* W, int ldw) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (N <= 0 || (N & 1)) return set_error(-2, "N must be positive and even");
  if (!L) return set_error(-3, "L is NULL");
  if (ldl < N) return set_error(-4, "ldl < N");
  if (!W) return set_error(-5, "W is NULL");
  if (ldw < N) return set_error(-6, "ldw < N");
  BSE_TRY(prologue(ctx));
  const Plan p = make_plan(N);
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, p.total, &base));
  Bufs b;
  bind(p, base, &b);
  hipStream_t s = ctx->stream;
  BSE_TRY(copy_matrix(s, N, N, L, ldl, b.L, p.ld));
  BSE_TRY(zero_upper(s, N, b.L, p.ld));
  BSE_TRY(form_W(s, N, b.L, p.ld, b.W, p.ld, true));
  BSE_TRY(copy_matrix(s, N, N, b.W, p.ld, W, ldw));
  BSE_HIP(hipStreamSynchronize(s));
  return 0;
}

int bse_sktrd(bse_ctx* ctx, int N, double* W, int ldw, double* alpha, double* tau) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (N < 2) return set_error(-2, "N must be >= 2");
  if (!W) return set_error(-3, "W is NULL");
  if (ldw < N) return set_error(-4, "ldw < N");
  if (!alpha) return set_error(-5, "alpha is NULL");
  if (!tau) return set_error(-6, "tau is NULL");
  BSE_TRY(prologue(ctx));
  const Plan p = make_plan(N);
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, p.total, &base));
  Bufs b;
  bind(p, base, &b);
  hipStream_t s = ctx->stream;
  BSE_TRY(copy_matrix(s, N, N, W, ldw, b.W, p.ld));
  BSE_TRY(sktrd_f64(s, N, b.W, p.ld, b.alpha, b.tau, b.sk));
  BSE_TRY(copy_matrix(s, N, N, b.W, p.ld, W, ldw));
  BSE_HIP(hipMemcpyAsync(alpha, b.alpha, (N - 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  BSE_HIP(hipMemcpyAsync(tau, b.tau, (N - 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  BSE_HIP(hipStreamSynchronize(s));
  return 0;
}

int bse_tridiag_eig(bse_ctx* ctx, int N, const double* alpha, double* lambda, double* V, int ldv) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (N < 2 || (N & 1)) return set_error(-2, "N must be even and >= 2");
  if (!alpha) return set_error(-3, "alpha is NULL");
  if (!lambda) return set_error(-4, "lambda is NULL");
  if (V && ldv < N) return set_error(-6, "ldv < N");
  BSE_TRY(prologue(ctx));
  const Plan p = make_plan(N);
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, p.total, &base));
  Bufs b;
  bind(p, base, &b);
  hipStream_t s = ctx->stream;
  BSE_HIP(hipMemcpyAsync(b.alpha, alpha, (N - 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  BSE_TRY(tridiag_bisect(s, N, b.alpha, b.e2, b.scal, lambda));
  if (V) {
    BSE_TRY(tridiag_invit(s, N, b.alpha, b.scal, lambda, b.shift, b.inv, b.Vt));
    BSE_TRY(tridiag_reorth(s, N, lambda, b.scal, b.Vt, b.inv, b.cid, b.info, b.linv));
    BSE_TRY(transpose_to(s, N / 2, N, b.Vt, N / 2, V, ldv));
    int info = 0;
    BSE_TRY(read_info(ctx, b.info, &info));
    if (info != 0) return set_error(BSE_EDEVICE, "cluster Gram matrix not positive definite");
  }
  BSE_HIP(hipStreamSynchronize(s));
  return 0;
}

}  // extern "C"
