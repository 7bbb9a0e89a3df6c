// Solver driver and C ABI: stage sequencing, workspace layout, argument
// checking and timing for the chain of Algorithm 1 / Algorithm 3.
//
// Every solve runs as a batch: one descriptor (Prob) per problem, sorted by
// decreasing order, uploaded once, and one launch per step of the chain for
// all problems that still have work at that step.  bse_solve is a batch of
// one; bse_solve_batched hands many independent problems of uneven sizes to
// the same kernels.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "driver.h"
#include "serve.h"


namespace bse {

namespace {
thread_local std::string g_last_error;
}

int set_hip_error(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  g_last_error = buf;
  return BSE_EDEVICE;
}

int set_error(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

static int set_errorf(int code, const char* fmt, int i) {
  char buf[256];
  snprintf(buf, sizeof(buf), fmt, i);
  g_last_error = buf;
  return code;
}

// ------------------------------------------------------------------------
// Workspace layout of one problem of order N = 2n, FP64, relative to the
// start of its block.
// ------------------------------------------------------------------------
struct Plan {
  long N = 0, n = 0, ld = 0;
  int prec = BSE_PREC_FP64;
  size_t off_L = 0, off_W = 0, off_Z = 0, off_Vt = 0, off_inv = 0, off_small = 0, off_sk = 0,
         off_bt = 0, off_gscr = 0;
  size_t gscr_bytes = 0;
  // mixed-precision path only
  size_t off_W32 = 0, off_R = 0, off_refmax = 0, off_perm = 0, off_cl = 0;
  size_t total = 0;
};

static Plan make_plan(long N, int prec) {
  Plan p;
  p.N = N;
  p.prec = prec;
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
  // (and for the compact-WY factors of the two-stage back-transformation)
  p.off_inv = take(std::max((size_t)4 * N * p.n * sizeof(double) + (size_t)N * p.n + 256, sbr_q2_T_bytes(N)));
  // alpha, tau, e2 (ld each), shift (n), scal (16), cid (n ints)
  p.off_small = take((size_t)(3 * p.ld + p.n + 16) * sizeof(double) + (size_t)p.n * sizeof(int));
  p.off_sk = take(sktrd_work_bytes(N, p.ld));
  p.off_bt = take(backtr_work_bytes(N, p.ld));
  // split-K partial products: only products of large problems are split
  p.gscr_bytes = (N > 2048) ? (size_t)16 * 64 * p.ld * sizeof(double) : 0;
  if (p.gscr_bytes) p.off_gscr = take(p.gscr_bytes);
  if (prec == BSE_PREC_FP32_REFINE) {
    p.off_W32 = take((size_t)p.ld * p.ld * sizeof(float));
    p.off_R = take(4 * sq);   // R1..R4
    const size_t nt = (size_t)(p.ld / 64);
    p.off_refmax = take(2 * nt * nt * sizeof(double));
    p.off_perm = take((size_t)p.n * sizeof(int));
    // clusters: start and flag (ints), maxima and rotations (doubles)
    p.off_cl = take((size_t)p.n * (2 * sizeof(int) + (1 + REF_CMAX4) * sizeof(double)) + 256);
  }
  p.total = cur;
  return p;
}

size_t problem_bytes(long N, int prec) { return make_plan(N, prec).total; }

// Descriptor array, then per slot: two info words, the refinement state word
// and two refinement maxima.
static size_t hdr_info_off(int count) { return (size_t)round_up((long)(count * sizeof(Prob)), 256); }
static size_t hdr_state_off(int count) { return hdr_info_off(count) + (size_t)round_up((long)(count * 2 * sizeof(int)), 256); }
static size_t hdr_reorth_off(int count) { return hdr_state_off(count) + (size_t)round_up((long)(count * sizeof(int)), 256); }
static size_t hdr_ref_off(int count) { return hdr_reorth_off(count) + (size_t)round_up((long)(count * sizeof(int)), 256); }
static size_t hdr_gdef_off(int count) { return hdr_ref_off(count) + (size_t)round_up((long)(count * 2 * sizeof(double)), 256); }
static size_t hdr_wgpre_off(int count) { return hdr_gdef_off(count) + (size_t)round_up((long)(count * sizeof(double)), 256); }
// workgroup prefixes of the tridiagonalisation: one row of 2 (count + 1) per
// column of a panel
size_t header_bytes(int count) {
  return hdr_wgpre_off(count) + (size_t)round_up((long)(SKTRD_NB * 2 * (count + 1) * sizeof(int)), 256);
}

// Workspace pointers of one problem.
static void bind_problem(const Plan& p, char* base, Prob* P) {
  P->n = (int)p.n;
  P->N = (int)p.N;
  P->ld = p.ld;
  P->L = reinterpret_cast<double*>(base + p.off_L);
  P->W = reinterpret_cast<double*>(base + p.off_W);
  P->Z = reinterpret_cast<double*>(base + p.off_Z);
  P->Vt = reinterpret_cast<double*>(base + p.off_Vt);
  P->inv = reinterpret_cast<double*>(base + p.off_inv);
  double* sm = reinterpret_cast<double*>(base + p.off_small);
  P->alpha = sm;
  P->tau = sm + p.ld;
  P->e2 = sm + 2 * p.ld;
  P->shift = sm + 3 * p.ld;
  P->scal = sm + 3 * p.ld + p.n;
  P->cid = reinterpret_cast<int*>(sm + 3 * p.ld + p.n + 16);
  P->gscr = p.gscr_bytes ? reinterpret_cast<double*>(base + p.off_gscr) : nullptr;
  P->gscr_bytes = p.gscr_bytes;
  sktrd_bind_work(base + p.off_sk, p.N, p.ld, P);
  backtr_bind_work(base + p.off_bt, p.N, p.ld, P);
  P->prec = p.prec;
  if (p.prec == BSE_PREC_FP32_REFINE) {
    P->W32 = reinterpret_cast<float*>(base + p.off_W32);
    double* R = reinterpret_cast<double*>(base + p.off_R);
    const size_t sq = (size_t)p.ld * p.ld;
    P->R1 = R;
    P->R2 = R + sq;
    P->R3 = R + 2 * sq;
    P->R4 = R + 3 * sq;
    P->Z32 = reinterpret_cast<float*>(P->R4);
    // R3 is free until the refinement: the reduction's FP32 panel copies
    P->Y1f = reinterpret_cast<float*>(P->R3);
    P->Y2f = P->Y1f + (size_t)p.ld * 2 * SKTRD_NB;
    P->refmax = reinterpret_cast<double*>(base + p.off_refmax);
    P->perm = reinterpret_cast<int*>(base + p.off_perm);
    char* cl = base + p.off_cl;
    P->clmax = reinterpret_cast<double*>(cl);
    P->clT = P->clmax + p.n;
    P->clstart = reinterpret_cast<int*>(P->clT + (size_t)p.n * REF_CMAX4);
    P->clflag = P->clstart + p.n;
  }
}

static int get_workspace(bse_ctx* ctx, size_t bytes, char** base) {
  if (ctx->arena) {
    if (bytes > ctx->arena_bytes) return set_error(BSE_ENOMEM, "workspace exceeds the caller's arena");
    *base = static_cast<char*>(ctx->arena);
    return 0;
  }
  if (ctx->own_bytes < bytes) {
    if (ctx->own) {
      BSE_HIP(hipStreamSynchronize(ctx->lane.stream));
      BSE_HIP(hipFree(ctx->own));
      ctx->own = nullptr;
      ctx->own_bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->own, bytes);
    if (e != hipSuccess) {
      ctx->own = nullptr;
      (void)hipGetLastError();
      if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return set_error(BSE_ENOMEM, "device workspace allocation failed");
      return set_hip_error(e, "hipMalloc", __FILE__, __LINE__);
    }
    ctx->own_bytes = bytes;
  }
  *base = static_cast<char*>(ctx->own);
  return 0;
}

// Pinned host mirrors for `count` descriptors (the lane's stream is idle
// between calls, so the old buffers can be released).
int lane_reserve(Lane* L, int count) {
  if (L->hcap >= count) return 0;
  if (L->hprobs) BSE_HIP(hipHostFree(L->hprobs));
  if (L->hinfo) BSE_HIP(hipHostFree(L->hinfo));
  if (L->hstate) BSE_HIP(hipHostFree(L->hstate));
  if (L->hrefout) BSE_HIP(hipHostFree(L->hrefout));
  L->hprobs = nullptr;
  L->hinfo = nullptr;
  L->hstate = nullptr;
  L->hrefout = nullptr;
  L->hcap = 0;
  const int cap = std::max(count, 16);
  BSE_HIP(hipHostMalloc(reinterpret_cast<void**>(&L->hprobs), cap * sizeof(Prob), hipHostMallocDefault));
  BSE_HIP(hipHostMalloc(reinterpret_cast<void**>(&L->hinfo), cap * 2 * sizeof(int), hipHostMallocDefault));
  BSE_HIP(hipHostMalloc(reinterpret_cast<void**>(&L->hstate), cap * sizeof(int), hipHostMallocDefault));
  BSE_HIP(hipHostMalloc(reinterpret_cast<void**>(&L->hrefout), cap * 2 * sizeof(double), hipHostMallocDefault));
  L->hcap = cap;
  return 0;
}

void lane_release(Lane* L) {
  for (auto& g : L->gcache) (void)hipGraphExecDestroy(g.exec);
  L->gcache.clear();
  if (L->cap) (void)hipStreamDestroy(L->cap);
  L->cap = nullptr;
  if (L->events)
    for (int i = 0; i <= BSE_NUM_STAGES; ++i) (void)hipEventDestroy(L->ev[i]);
  L->events = false;
  for (hipEvent_t e : L->kev) (void)hipEventDestroy(e);
  L->kev.clear();
  if (L->hprobs) (void)hipHostFree(L->hprobs);
  if (L->hinfo) (void)hipHostFree(L->hinfo);
  if (L->hstate) (void)hipHostFree(L->hstate);
  if (L->hrefout) (void)hipHostFree(L->hrefout);
  L->hprobs = nullptr;
  L->hinfo = nullptr;
  L->hstate = nullptr;
  L->hrefout = nullptr;
  L->hcap = 0;
}

static int ensure_events(Lane* L) {
  if (L->events) return 0;
  for (int i = 0; i <= BSE_NUM_STAGES; ++i) BSE_HIP(hipEventCreate(&L->ev[i]));
  L->events = true;
  return 0;
}

static int mark(Lane* L, bool timed, int i) {
  if (timed) BSE_HIP(hipEventRecord(L->ev[i], L->stream));
  return 0;
}

int setup_batch(Lane* L, int count, const long* Ns, int prec, char* header, char* const* bases, Setup* S) {
  BSE_TRY(lane_reserve(L, count));
  S->count = count;
  S->dprobs = reinterpret_cast<Prob*>(header);
  S->dinfo = reinterpret_cast<int*>(header + hdr_info_off(count));
  S->dstate = reinterpret_cast<int*>(header + hdr_state_off(count));
  S->dreorth = reinterpret_cast<int*>(header + hdr_reorth_off(count));
  S->dref = reinterpret_cast<double*>(header + hdr_ref_off(count));
  S->dwgpre = reinterpret_cast<int*>(header + hdr_wgpre_off(count));
  S->total = header_bytes(count);
  for (int i = 0; i < count; ++i) {
    const Plan plan = make_plan(Ns[i], prec);
    Prob& P = L->hprobs[i];
    memset(&P, 0, sizeof(P));
    bind_problem(plan, bases[i], &P);
    P.info = S->dinfo + 2 * i;
    P.refstate = S->dstate + i;
    P.reorth = S->dreorth + i;
    P.refout = S->dref + 2 * i;
    P.gdef = reinterpret_cast<double*>(header + hdr_gdef_off(count)) + i;
    S->total += plan.total;
  }
  return 0;
}

// Workspace from the context (arena or own allocation) for problems of
// orders Ns[0..count), laid out header first, then problem by problem.
static int setup_ctx_batch(bse_ctx* ctx, int count, const long* Ns, int prec, Setup* S) {
  size_t total = header_bytes(count);
  std::vector<size_t> offs(count);
  for (int i = 0; i < count; ++i) {
    offs[i] = total;
    total += problem_bytes(Ns[i], prec);
  }
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, total, &base));
  std::vector<char*> bases(count);
  for (int i = 0; i < count; ++i) bases[i] = base + offs[i];
  return setup_batch(&ctx->lane, count, Ns, prec, base, bases.data(), S);
}

static int upload(Lane* L, const Setup& S, int count) {
  BSE_HIP(hipMemcpyAsync(S.dprobs, L->hprobs, count * sizeof(Prob), hipMemcpyHostToDevice, L->stream));
  return 0;
}

static int read_infos(Lane* L, const Setup& S, int count) {
  BSE_HIP(hipMemcpyAsync(L->hinfo, S.dinfo, count * 2 * sizeof(int), hipMemcpyDeviceToHost, L->stream));
  BSE_HIP(hipStreamSynchronize(L->stream));
  return 0;
}

// The chain for a batch whose descriptors (sorted by decreasing N) are in
// L->hprobs[0..count).  On return L->hinfo holds, per original slot,
// info[0] (Cholesky of M, > 0 = not definite) and info[1] (Cholesky of a
// cluster Gram matrix, > 0 = reorthogonalisation failed).
// Stages in the order they run (event i marks the start of stage order[i]).
static const int kStageOrder[BSE_NUM_STAGES] = {
    BSE_STAGE_BUILD_M, BSE_STAGE_POTRF,   BSE_STAGE_FORM_W,  BSE_STAGE_SKTRD,   BSE_STAGE_BISECT, BSE_STAGE_INVIT,
    BSE_STAGE_REORTH,  BSE_STAGE_APPLY_U, BSE_STAGE_REFINE,  BSE_STAGE_APPLY_L, BSE_STAGE_FINISH};

// The chain after the Cholesky of M: W, the reduction, the tridiagonal
// eigensolve and the back-transformation, for the live problems of b.
static int chain_tail(hipStream_t s, Lane* L, const Setup& S, const Batch& b, bool vectors, bool mixed, bool two,
                      bool timed, int& ev, KernelTimer* ktimer, RefineStats* rstats) {
  // the reduction reads W's lower triangle (the mixed path an FP32 copy of
  // it; its refinement works from L, W = L^T J L)
  BSE_TRY(form_W_batched(s, b, false));
  // the two-stage reduction keeps W as its strict lower triangle over a zero
  // upper triangle
  if (two) BSE_TRY(zero_upper(s, L->hprobs[0].N, L->hprobs[0].W, L->hprobs[0].ld));
  if (mixed) BSE_TRY(to_f32_batched(s, b));
  BSE_TRY(mark(L, timed, ev++));
  if (two) BSE_TRY(sbr_single(s, b, reinterpret_cast<int*>(L->hprobs[0].Ycol), vectors || mixed));
  else BSE_TRY(sktrd_batched(s, b, ktimer));
  BSE_TRY(mark(L, timed, ev++));
  BSE_TRY(bisect_batched(s, b));
  BSE_TRY(mark(L, timed, ev++));
  // the refinement needs the eigenvector basis even when only eigenvalues
  // are wanted
  if (vectors || mixed) {
    BSE_TRY(invit_batched(s, b));
    BSE_TRY(mark(L, timed, ev++));
    BSE_TRY(reorth_batched(s, b, S.dreorth, L->hstate, S.count));
    BSE_TRY(mark(L, timed, ev++));
    BSE_TRY(apply_UD_batched(s, b));
    BSE_TRY(mark(L, timed, ev++));
    if (mixed) {
      RefineIO io;
      io.dstate = S.dstate;
      io.dout = S.dref;
      io.hstate = L->hstate;
      io.hout = L->hrefout;
      io.nslots = S.count;
      BSE_TRY(refine_batched(s, b, io, rstats));
    }
    BSE_TRY(mark(L, timed, ev++));
    // the mixed path applies L for its eigenvalues as well
    if (vectors || mixed) {
      BSE_TRY(gemm_batched(s, b, b.count, GOP_APPLY_L, 0));
      BSE_TRY(mark(L, timed, ev++));
      if (mixed) BSE_TRY(refine_final_batched(s, b));
      if (vectors) BSE_TRY(finish_batched(s, b));
      if (vectors && b.count == 1 && (b.host[0].flags & FLAG_REAL_IN)) BSE_TRY(real_output_single(s, b));
    } else {
      BSE_TRY(mark(L, timed, ev++));
    }
  } else {
    for (int i = 0; i < 5; ++i) BSE_TRY(mark(L, timed, ev++));
  }
  return 0;
}

// The chain tail as a graph: looked up by the batch shape (the launches'
// grids and arguments depend only on the live problems' orders, the policy,
// whether vectors are wanted and the address of the descriptor header; the
// caller's buffers and the workspace addresses are read by the kernels from
// the descriptors, which are uploaded per call), captured on the lane's
// own stream at the first call of a shape and replayed on the lane's stream.
static int chain_tail_graph(Lane* L, const Setup& S, const Batch& b, bool vectors) {
  std::vector<long> key;
  key.reserve(6 + b.count);
  key.push_back(b.count);
  key.push_back(b.host[0].prec);
  key.push_back(vectors ? 1 : 0);
  key.push_back((long)reinterpret_cast<intptr_t>(S.dprobs));
  key.push_back((long)reinterpret_cast<intptr_t>(S.dwgpre));
  for (int i = 0; i < b.count; ++i) key.push_back(b.host[i].N);
  size_t hit = L->gcache.size();
  for (size_t i = 0; i < L->gcache.size(); ++i)
    if (L->gcache[i].key == key) hit = i;
  if (hit == L->gcache.size()) {
    if (!L->cap) BSE_HIP(hipStreamCreateWithFlags(&L->cap, hipStreamNonBlocking));
    BSE_HIP(hipStreamBeginCapture(L->cap, hipStreamCaptureModeThreadLocal));
    int ev = 0;
    RefineStats rs;
    const int rc = chain_tail(L->cap, L, S, b, vectors, false, false, false, ev, nullptr, &rs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(L->cap, &graph);
    if (rc != 0) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return set_hip_error(e, "hipStreamEndCapture", __FILE__, __LINE__);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return set_hip_error(ei, "hipGraphInstantiate", __FILE__, __LINE__);
    constexpr size_t kMaxGraphs = 8;
    if (L->gcache.size() >= kMaxGraphs) {
      (void)hipGraphExecDestroy(L->gcache.front().exec);
      L->gcache.erase(L->gcache.begin());
    }
    Lane::GraphEntry g;
    g.key = std::move(key);
    g.exec = exec;
    L->gcache.push_back(std::move(g));
    hit = L->gcache.size() - 1;
    ++L->graph_captures;
  } else {
    ++L->graph_replays;
  }
  BSE_HIP(hipGraphLaunch(L->gcache[hit].exec, L->stream));
  return 0;
}

int run_chain(Lane* L, const Setup& S, int count, bool vectors, bse_report* rep) {
  hipStream_t s = L->stream;
  const bool timed = rep != nullptr;
  if (timed) BSE_TRY(ensure_events(L));
  // a single problem with BSE_TWO_STAGE takes the two-stage reduction, whose
  // first-stage reflectors the back-transformation applies at row offset SBR_B
  for (int i = 0; i < count; ++i)
    L->hprobs[i].uoff = (count == 1 && (L->hprobs[i].flags & BSE_TWO_STAGE) != 0) ? SBR_B : 1;
  BSE_TRY(upload(L, S, count));
  Batch b;
  b.count = count;
  b.host = L->hprobs;
  b.dev = S.dprobs;
  b.wgpre = S.dwgpre;
  const int prec = count > 0 ? L->hprobs[0].prec : BSE_PREC_FP64;
  const bool mixed = prec == BSE_PREC_FP32_REFINE;
  int ev = 0;

  BSE_TRY(mark(L, timed, ev++));
  BSE_TRY(build_M_batched(s, b));
  BSE_TRY(mark(L, timed, ev++));
  BSE_TRY(potrf_batched(s, b, 0, true));
  BSE_TRY(mark(L, timed, ev++));
  BSE_TRY(read_infos(L, S, count));
  // drop the problems whose M is not definite; the rest keep their order
  int live = 0;
  for (int i = 0; i < count; ++i) {
    const Prob& P = L->hprobs[i];
    if (L->hinfo[P.info - S.dinfo] == 0) {
      if (live != i) L->hprobs[live] = P;
      ++live;
    }
  }
  if (live < count) {
    b.count = live;
    if (live > 0) BSE_TRY(upload(L, S, live));
  }
  const bool two = b.count == 1 && (L->hprobs[0].flags & BSE_TWO_STAGE) != 0;
  const bool real_in = b.count == 1 && (L->hprobs[0].flags & FLAG_REAL_IN) != 0;
  KernelTimer ktimer;
  if (L->timing && b.count > 0) {
    const long N0 = b.maxN();
    const size_t need = 2 * (size_t)(N0 > 2 ? N0 - 2 : 0);
    while (L->kev.size() < need) {
      hipEvent_t e;
      BSE_HIP(hipEventCreate(&e));
      L->kev.push_back(e);
    }
    ktimer.ev = L->kev.data();
    ktimer.cap = (int)L->kev.size();
  }
  RefineStats rstats;
  // graph replay: FP64 chains without host decisions after the Cholesky
  const bool graph = L->graphs && !L->timing && !mixed && !two && !real_in && b.count > 0;
  if (graph) {
    // the tail's stage events are not recorded: its time goes to form_W
    BSE_TRY(chain_tail_graph(L, S, b, vectors));
    for (; ev < BSE_NUM_STAGES; ++ev) BSE_TRY(mark(L, timed, ev));
  } else {
    BSE_TRY(chain_tail(s, L, S, b, vectors, mixed, two, timed, ev, L->timing ? &ktimer : nullptr, &rstats));
  }
  BSE_TRY(mark(L, timed, ev++));
  BSE_TRY(read_infos(L, S, count));
  if (timed) {
    memset(rep, 0, sizeof(*rep));
    float ms = 0.f;
    for (int i = 0; i < BSE_NUM_STAGES; ++i) {
      BSE_HIP(hipEventElapsedTime(&ms, L->ev[i], L->ev[i + 1]));
      rep->stage_ms[kStageOrder[i]] = ms;
    }
    BSE_HIP(hipEventElapsedTime(&ms, L->ev[0], L->ev[BSE_NUM_STAGES]));
    rep->total_ms = ms;
    rep->prec = prec;
    rep->workspace_bytes = S.total;
    rep->refine_sweeps = rstats.sweeps;
    rep->refine_first_correction = rstats.first_correction;
    rep->refine_correction = rstats.last_correction;
    rep->graph = graph ? 1 : 0;
    if (L->timing) {
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

bool valid_prec(int prec) { return prec == BSE_PREC_FP64 || prec == BSE_PREC_FP32_REFINE; }

int check_solve_args(int n, const void* A, int lda, const void* B, int ldb, int prec, unsigned flags,
                     const double* lambda, const void* X, int ldx, const void* d_r, const void* w,
                     bool need_B) {
  if (n <= 0) return set_error(-2, "n must be positive");
  if (!A) return set_error(-3, "A is NULL");
  if (lda < n) return set_error(-4, "lda < n");
  if (need_B && !B) return set_error(-5, "B is NULL");
  if (need_B && ldb < n) return set_error(-6, "ldb < n");
  if (!valid_prec(prec)) return set_error(-7, "unsupported precision policy");
  if (flags & ~(BSE_WANT_VECTORS | BSE_WANT_WEIGHTS | BSE_TWO_STAGE | BSE_EIGVEC_TWISTED)) return set_error(-8, "unknown flags");
  if (!lambda) return set_error(-9, "lambda is NULL");
  const bool vec = (flags & BSE_WANT_VECTORS) != 0;
  const bool wts = (flags & BSE_WANT_WEIGHTS) != 0;
  if (wts && !vec) return set_error(-8, "weights need eigenvectors");
  if ((flags & BSE_TWO_STAGE) && prec != BSE_PREC_FP64)
    return set_error(BSE_EUNSUPPORTED, "the two-stage reduction runs the FP64 path only");
  if (vec && !X) return set_error(-10, "X is NULL");
  if (vec && ldx < 2 * n) return set_error(-11, "ldx < 2n");
  if (wts && !d_r) return set_error(-12, "d_r is NULL");
  if (wts && !w) return set_error(-14, "w is NULL");
  return 0;
}

int solve_single_in(Lane* L, char* base, int n, const void* A, int lda, const void* B, int ldb, int prec,
                    unsigned flags, double* lambda, void* X, int ldx, const void* d_r, const void* d_l,
                    void* w, bse_report* rep) {
  const long N = 2L * n;
  char* pbase = base + header_bytes(1);
  Setup S;
  BSE_TRY(setup_batch(L, 1, &N, prec, base, &pbase, &S));
  const bool vec = (flags & BSE_WANT_VECTORS) != 0;
  Prob& P = L->hprobs[0];
  P.A = static_cast<const double*>(A);
  P.lda = lda;
  P.B = static_cast<const double*>(B);
  P.ldb = ldb;
  P.lambda = lambda;
  P.X = static_cast<double*>(X);
  P.ldx = ldx;
  P.dr = static_cast<const double*>(d_r);
  P.dl = static_cast<const double*>(d_l);
  P.w = static_cast<double*>(w);
  P.flags = flags;
  BSE_TRY(run_chain(L, S, 1, vec, rep));
  if (rep) rep->n = n;
  const int code = info_code(L->hinfo[0], L->hinfo[1], vec);
  if (code == BSE_EDEVICE) return set_error(BSE_EDEVICE, "cluster Gram matrix not positive definite");
  if (code == BSE_ENOCONV) return set_error(BSE_ENOCONV, "refinement did not converge within the sweep limit");
  return code;
}

static int prologue(bse_ctx* ctx) {
  if (!ctx) return set_error(-1, "null context");
  BSE_HIP(hipSetDevice(ctx->device));
  return 0;
}

// One problem of order N for the stage entry points.
static int setup_single(bse_ctx* ctx, long N, Setup* S) { return setup_ctx_batch(ctx, 1, &N, BSE_PREC_FP64, S); }

static Batch single_batch(bse_ctx* ctx, const Setup& S) {
  Batch b;
  b.count = 1;
  b.host = ctx->lane.hprobs;
  b.dev = S.dprobs;
  b.wgpre = S.dwgpre;
  return b;
}

}  // namespace bse

using namespace bse;

extern "C" {

int bse_version(void) { return 10100; }

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
  // the allocation-free entry point's workspace address on this device
  BSE_TRY(noalloc_init_device(device));
  // the matvec tile table in force, also on this device
  BSE_TRY(tile_table_upload());
  bse_ctx* c = new bse_ctx();
  c->device = device;
  c->arena = arena;
  c->arena_bytes = arena_bytes;
  c->lane.stream = static_cast<hipStream_t>(stream);
  c->lane.graphs = true;
  *ctx = c;
  return 0;
}

int bse_ctx_destroy(bse_ctx* ctx) {
  if (!ctx) return 0;
  (void)hipSetDevice(ctx->device);
  if (ctx->server) server_destroy(ctx->server);
  (void)hipStreamSynchronize(ctx->lane.stream);
  if (ctx->own) (void)hipFree(ctx->own);
  lane_release(&ctx->lane);
  delete ctx;
  return 0;
}

int bse_get_tile_table(int* table) {
  if (!table) return set_error(-1, "table is NULL");
  return tile_table_get(table);
}

int bse_set_tile_table(bse_ctx* ctx, const int* table) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (!table) return set_error(-2, "table is NULL");
  BSE_TRY(prologue(ctx));
  BSE_HIP(hipStreamSynchronize(ctx->lane.stream));
  BSE_TRY(tile_table_set(table));
  BSE_TRY(tile_table_upload());
  // captured graphs hold grids sized with the old table
  for (auto& g : ctx->lane.gcache) (void)hipGraphExecDestroy(g.exec);
  ctx->lane.gcache.clear();
  return 0;
}

int bse_ctx_set_graphs(bse_ctx* ctx, int enable) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  ctx->lane.graphs = enable != 0;
  return 0;
}

int bse_ctx_set_timing(bse_ctx* ctx, int enable) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  ctx->lane.timing = enable != 0;
  return 0;
}

size_t bse_footprint_bytes(int n, int prec, unsigned flags) {
  if (n <= 0 || !valid_prec(prec)) return 0;
  return header_bytes(1) + make_plan(2L * n, run_prec(prec, flags)).total;
}

size_t bse_footprint_batched_bytes(int count, const int* n, int prec, unsigned flags) {
  if (count <= 0 || !n || !valid_prec(prec)) return 0;
  size_t total = header_bytes(count);
  for (int i = 0; i < count; ++i) {
    if (n[i] <= 0) return 0;
    total += make_plan(2L * n[i], run_prec(prec, flags)).total;
  }
  return total;
}

int bse_solve(bse_ctx* ctx, int n, const void* A, int lda, const void* B, int ldb, int prec,
              unsigned flags, double* lambda, void* X, int ldx, const void* d_r, const void* d_l,
              void* w, bse_report* rep) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  BSE_TRY(check_solve_args(n, A, lda, B, ldb, prec, flags, lambda, X, ldx, d_r, w));
  BSE_TRY(prologue(ctx));
  prec = run_prec(prec, flags);
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, header_bytes(1) + problem_bytes(2L * n, prec), &base));
  return solve_single_in(&ctx->lane, base, n, A, lda, B, ldb, prec, flags, lambda, X, ldx, d_r, d_l, w, rep);
}

int bse_solve_tda(bse_ctx* ctx, int n, const void* A, int lda, int prec, unsigned flags, double* lambda,
                  void* X, int ldx, const void* d_r, const void* d_l, void* w, bse_report* rep) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  // argument numbers of bse_solve_tda: B and ldb are absent
  int rc = check_solve_args(n, A, lda, nullptr, n, prec, flags, lambda, X, ldx, d_r, w, false);
  if (rc <= -7) rc += 2;
  if (rc != 0) return rc;
  BSE_TRY(prologue(ctx));
  prec = run_prec(prec, flags);
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, header_bytes(1) + problem_bytes(2L * n, prec), &base));
  return solve_single_in(&ctx->lane, base, n, A, lda, nullptr, n, prec, flags, lambda, X, ldx, d_r, d_l, w, rep);
}

int bse_solve_real(bse_ctx* ctx, int n, const double* A, int lda, const double* B, int ldb, int prec,
                   unsigned flags, double* lambda, double* X, int ldx, const void* d_r, const void* d_l, void* w,
                   bse_report* rep) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  BSE_TRY(check_solve_args(n, A, lda, B, ldb, prec, flags, lambda, X, ldx, d_r, w));
  BSE_TRY(prologue(ctx));
  prec = run_prec(prec, flags);
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, header_bytes(1) + problem_bytes(2L * n, prec), &base));
  Lane* L = &ctx->lane;
  const long N = 2L * n;
  char* pbase = base + header_bytes(1);
  Setup S;
  BSE_TRY(setup_batch(L, 1, &N, prec, base, &pbase, &S));
  const bool vec = (flags & BSE_WANT_VECTORS) != 0;
  Prob& P = L->hprobs[0];
  P.A = A;
  P.lda = lda;
  P.B = B;
  P.ldb = ldb;
  P.lambda = lambda;
  // the complex eigenvectors are assembled in the Z buffer (free once G =
  // L Z is formed; ld >= 2n rows by n complex columns fit), then written
  // to X as real vectors
  P.X = vec ? P.Z : nullptr;
  P.ldx = 2L * n;
  P.Xr = X;
  P.ldxr = ldx;
  P.dr = static_cast<const double*>(d_r);
  P.dl = static_cast<const double*>(d_l);
  P.w = static_cast<double*>(w);
  P.flags = flags | FLAG_REAL_IN;
  BSE_TRY(run_chain(L, S, 1, vec, rep));
  if (rep) rep->n = n;
  const int code = info_code(L->hinfo[0], L->hinfo[1], vec);
  if (code == BSE_EDEVICE) return set_error(BSE_EDEVICE, "no orthonormal real eigenvector basis");
  if (code == BSE_ENOCONV) return set_error(BSE_ENOCONV, "refinement did not converge within the sweep limit");
  return code;
}

int bse_solve_batched(bse_ctx* ctx, int count, const int* n, const void* const* A, const int* lda,
                      const void* const* B, const int* ldb, int prec, unsigned flags,
                      double* const* lambda, void* const* X, const int* ldx, const void* const* d,
                      void* const* w, int* info, bse_report* rep) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (count < 0) return set_error(-2, "count is negative");
  if (count == 0) return 0;
  if (!n) return set_error(-3, "n is NULL");
  if (!A) return set_error(-4, "A is NULL");
  if (!lda) return set_error(-5, "lda is NULL");
  if (!B) return set_error(-6, "B is NULL");
  if (!ldb) return set_error(-7, "ldb is NULL");
  if (!valid_prec(prec)) return set_error(-8, "unsupported precision policy");
  if (flags & ~(BSE_WANT_VECTORS | BSE_WANT_WEIGHTS | BSE_EIGVEC_TWISTED)) return set_error(-9, "unknown flags");
  if (!lambda) return set_error(-10, "lambda is NULL");
  const bool vec = (flags & BSE_WANT_VECTORS) != 0;
  const bool wts = (flags & BSE_WANT_WEIGHTS) != 0;
  if (wts && !vec) return set_error(-9, "weights need eigenvectors");
  if (vec && !X) return set_error(-11, "X is NULL");
  if (vec && !ldx) return set_error(-12, "ldx is NULL");
  if (wts && !d) return set_error(-13, "d is NULL");
  if (wts && !w) return set_error(-14, "w is NULL");
  if (!info) return set_error(-15, "info is NULL");
  for (int i = 0; i < count; ++i) {
    if (n[i] <= 0) return set_errorf(-3, "n[%d] must be positive", i);
    if (!A[i]) return set_errorf(-4, "A[%d] is NULL", i);
    if (lda[i] < n[i]) return set_errorf(-5, "lda[%d] < n", i);
    if (!B[i]) return set_errorf(-6, "B[%d] is NULL", i);
    if (ldb[i] < n[i]) return set_errorf(-7, "ldb[%d] < n", i);
    if (!lambda[i]) return set_errorf(-10, "lambda[%d] is NULL", i);
    if (vec && !X[i]) return set_errorf(-11, "X[%d] is NULL", i);
    if (vec && ldx[i] < 2 * n[i]) return set_errorf(-12, "ldx[%d] < 2n", i);
    if (wts && !d[i]) return set_errorf(-13, "d[%d] is NULL", i);
    if (wts && !w[i]) return set_errorf(-14, "w[%d] is NULL", i);
  }
  BSE_TRY(prologue(ctx));
  prec = run_prec(prec, flags);
  // descriptors sorted by decreasing n (stable)
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return n[a] > n[b2]; });
  std::vector<long> Ns(count);
  for (int k = 0; k < count; ++k) Ns[k] = 2L * n[order[k]];
  Setup S;
  BSE_TRY(setup_ctx_batch(ctx, count, Ns.data(), prec, &S));
  for (int k = 0; k < count; ++k) {
    const int i = order[k];
    Prob& P = ctx->lane.hprobs[k];
    P.A = static_cast<const double*>(A[i]);
    P.lda = lda[i];
    P.B = static_cast<const double*>(B[i]);
    P.ldb = ldb[i];
    P.lambda = lambda[i];
    P.X = vec ? static_cast<double*>(X[i]) : nullptr;
    P.ldx = vec ? ldx[i] : 0;
    P.dr = wts ? static_cast<const double*>(d[i]) : nullptr;
    P.dl = nullptr;
    P.w = wts ? static_cast<double*>(w[i]) : nullptr;
    P.flags = flags;
  }
  BSE_TRY(run_chain(&ctx->lane, S, count, vec, rep));
  if (rep) rep->n = n[order[0]];
  for (int k = 0; k < count; ++k) {
    const int i = order[k];
    const int i0 = ctx->lane.hinfo[2 * k], i1 = ctx->lane.hinfo[2 * k + 1];
    info[i] = info_code(i0, i1, vec);
  }
  return 0;
}

// ---------------------------------------------------------------- serving

static int check_request(const bse_request* r) {
  if (!r) return set_error(-2, "request is NULL");
  if (r->n <= 0) return set_error(-2, "request: n must be positive");
  if (!r->A) return set_error(-2, "request: A is NULL");
  if (r->lda < r->n) return set_error(-2, "request: lda < n");
  if (!r->B) return set_error(-2, "request: B is NULL");
  if (r->ldb < r->n) return set_error(-2, "request: ldb < n");
  if (!valid_prec(r->prec)) return set_error(-2, "request: unsupported precision policy");
  if (r->flags & ~(BSE_WANT_VECTORS | BSE_WANT_WEIGHTS | BSE_EIGVEC_TWISTED)) return set_error(-2, "request: unknown flags");
  if (!r->lambda) return set_error(-2, "request: lambda is NULL");
  const bool vec = (r->flags & BSE_WANT_VECTORS) != 0;
  const bool wts = (r->flags & BSE_WANT_WEIGHTS) != 0;
  if (wts && !vec) return set_error(-2, "request: weights need eigenvectors");
  if (vec && !r->X) return set_error(-2, "request: X is NULL");
  if (vec && r->ldx < 2 * r->n) return set_error(-2, "request: ldx < 2n");
  if (wts && !r->d_r) return set_error(-2, "request: d_r is NULL");
  if (wts && !r->w) return set_error(-2, "request: w is NULL");
  return 0;
}

int bse_serve_config(bse_ctx* ctx, size_t pool_bytes, int slots, int max_batch) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (ctx->server) return set_error(BSE_EBUSY, "the server is already running");
  if (slots < 0 || slots > 16) return set_error(-3, "slots must be in [0, 16]");
  if (max_batch < 0 || max_batch > 4096) return set_error(-4, "max_batch must be in [0, 4096]");
  BSE_TRY(prologue(ctx));
  return server_create(ctx->device, pool_bytes, slots, max_batch, &ctx->server);
}

int bse_submit(bse_ctx* ctx, const bse_request* req, uint64_t* ticket) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  BSE_TRY(check_request(req));
  if (!ticket) return set_error(-3, "ticket is NULL");
  BSE_TRY(prologue(ctx));
  if (!ctx->server) BSE_TRY(server_create(ctx->device, 0, 0, 0, &ctx->server));
  bse_request r = *req;
  r.prec = run_prec(r.prec, r.flags);
  return server_submit(ctx->server, &r, ctx->lane.stream, ticket);
}

int bse_poll(bse_ctx* ctx, uint64_t ticket, int* state, int* info) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (!ctx->server) return set_error(BSE_ENOTICKET, "unknown ticket");
  return server_poll(ctx->server, ticket, state, info);
}

int bse_release(bse_ctx* ctx, uint64_t ticket) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (!ctx->server) return set_error(BSE_ENOTICKET, "unknown ticket");
  return server_release(ctx->server, ticket);
}

int bse_ticket_times(bse_ctx* ctx, uint64_t ticket, double* t_submit_us, double* t_start_us, double* t_done_us) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (!ctx->server) return set_error(BSE_ENOTICKET, "unknown ticket");
  return server_times(ctx->server, ticket, t_submit_us, t_start_us, t_done_us);
}

int bse_serve_stats(bse_ctx* ctx, bse_serve_counters* stats) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (!stats) return set_error(-2, "stats is NULL");
  if (!ctx->server) {
    memset(stats, 0, sizeof(*stats));
    return 0;
  }
  return server_stats(ctx->server, stats);
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
  BSE_TRY(lane_reserve(&ctx->lane, 1));
  char* base = nullptr;
  BSE_TRY(get_workspace(ctx, header_bytes(1), &base));
  Prob& P = ctx->lane.hprobs[0];
  memset(&P, 0, sizeof(P));
  P.n = n;
  P.N = 2 * n;
  P.A = static_cast<const double*>(A);
  P.lda = lda;
  P.B = static_cast<const double*>(B);
  P.ldb = ldb;
  P.L = M;  // the embedding is written straight into the caller's matrix
  P.ld = ldm;
  Setup S;
  S.dprobs = reinterpret_cast<Prob*>(base);
  BSE_TRY(upload(&ctx->lane, S, 1));
  BSE_TRY(build_M_batched(ctx->lane.stream, single_batch(ctx, S)));
  BSE_HIP(hipStreamSynchronize(ctx->lane.stream));
  return 0;
}

int bse_potrf(bse_ctx* ctx, int N, double* M, int ldm) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (N <= 0) return set_error(-2, "N must be positive");
  if (!M) return set_error(-3, "M is NULL");
  if (ldm < N) return set_error(-4, "ldm < N");
  BSE_TRY(prologue(ctx));
  Setup S;
  BSE_TRY(setup_single(ctx, N, &S));
  const Prob& P = ctx->lane.hprobs[0];
  hipStream_t s = ctx->lane.stream;
  BSE_TRY(upload(&ctx->lane, S, 1));
  BSE_TRY(copy_matrix(s, N, N, M, ldm, P.L, P.ld));
  BSE_TRY(zero_upper(s, N, P.L, P.ld));
  BSE_TRY(potrf_batched(s, single_batch(ctx, S), 0, true));
  BSE_TRY(copy_matrix(s, N, N, P.L, P.ld, M, ldm));
  BSE_TRY(read_infos(&ctx->lane, S, 1));
  return ctx->lane.hinfo[0];
}

int bse_form_W(bse_ctx* ctx, int N, const double* L, int ldl, double* W, int ldw) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (N <= 0 || (N & 1)) return set_error(-2, "N must be positive and even");
  if (!L) return set_error(-3, "L is NULL");
  if (ldl < N) return set_error(-4, "ldl < N");
  if (!W) return set_error(-5, "W is NULL");
  if (ldw < N) return set_error(-6, "ldw < N");
  BSE_TRY(prologue(ctx));
  Setup S;
  BSE_TRY(setup_single(ctx, N, &S));
  const Prob& P = ctx->lane.hprobs[0];
  hipStream_t s = ctx->lane.stream;
  BSE_TRY(upload(&ctx->lane, S, 1));
  BSE_TRY(copy_matrix(s, N, N, L, ldl, P.L, P.ld));
  BSE_TRY(zero_upper(s, N, P.L, P.ld));
  BSE_TRY(form_W_batched(s, single_batch(ctx, S), true));
  BSE_TRY(copy_matrix(s, N, N, P.W, P.ld, W, ldw));
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
  Setup S;
  BSE_TRY(setup_single(ctx, N, &S));
  const Prob& P = ctx->lane.hprobs[0];
  hipStream_t s = ctx->lane.stream;
  BSE_TRY(upload(&ctx->lane, S, 1));
  BSE_TRY(copy_matrix(s, N, N, W, ldw, P.W, P.ld));
  BSE_TRY(sktrd_batched(s, single_batch(ctx, S), nullptr));
  BSE_TRY(copy_matrix(s, N, N, P.W, P.ld, W, ldw));
  BSE_HIP(hipMemcpyAsync(alpha, P.alpha, (N - 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  BSE_HIP(hipMemcpyAsync(tau, P.tau, (N - 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  BSE_HIP(hipStreamSynchronize(s));
  return 0;
}

int bse_sktrd2(bse_ctx* ctx, int N, double* W, int ldw, double* alpha) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (N < 2) return set_error(-2, "N must be >= 2");
  if (!W) return set_error(-3, "W is NULL");
  if (ldw < N) return set_error(-4, "ldw < N");
  if (!alpha) return set_error(-5, "alpha is NULL");
  BSE_TRY(prologue(ctx));
  Setup S;
  BSE_TRY(setup_single(ctx, N, &S));
  const Prob& P = ctx->lane.hprobs[0];
  hipStream_t s = ctx->lane.stream;
  BSE_TRY(upload(&ctx->lane, S, 1));
  BSE_TRY(copy_matrix(s, N, N, W, ldw, P.W, P.ld));
  BSE_TRY(zero_upper(s, N, P.W, P.ld));
  BSE_TRY(sbr_single(s, single_batch(ctx, S), reinterpret_cast<int*>(P.Ycol), false));
  BSE_TRY(copy_matrix(s, N, N, P.W, P.ld, W, ldw));
  BSE_HIP(hipMemcpyAsync(alpha, P.alpha, (N - 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  BSE_HIP(hipStreamSynchronize(s));
  return 0;
}

int bse_tridiag_eig_flags(bse_ctx* ctx, int N, const double* alpha, double* lambda, double* V, int ldv,
                          unsigned flags) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (N < 2 || (N & 1)) return set_error(-2, "N must be even and >= 2");
  if (!alpha) return set_error(-3, "alpha is NULL");
  if (!lambda) return set_error(-4, "lambda is NULL");
  if (V && ldv < N) return set_error(-6, "ldv < N");
  if (flags & ~BSE_EIGVEC_TWISTED) return set_error(-7, "unknown flags");
  BSE_TRY(prologue(ctx));
  Setup S;
  BSE_TRY(setup_single(ctx, N, &S));
  Prob& P = ctx->lane.hprobs[0];
  P.lambda = lambda;
  P.flags = flags;
  hipStream_t s = ctx->lane.stream;
  BSE_TRY(upload(&ctx->lane, S, 1));
  const Batch b = single_batch(ctx, S);
  BSE_HIP(hipMemcpyAsync(P.alpha, alpha, (N - 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  BSE_TRY(bisect_batched(s, b));
  if (V) {
    BSE_TRY(invit_batched(s, b));
    BSE_TRY(reorth_batched(s, b, S.dreorth, ctx->lane.hstate, S.count));
    BSE_TRY(transpose_to(s, N / 2, N, P.Vt, N / 2, V, ldv));
    BSE_TRY(read_infos(&ctx->lane, S, 1));
    if (ctx->lane.hinfo[1] != 0) return set_error(BSE_EDEVICE, "cluster Gram matrix not positive definite");
  }
  BSE_HIP(hipStreamSynchronize(s));
  return 0;
}

int bse_tridiag_eig(bse_ctx* ctx, int N, const double* alpha, double* lambda, double* V, int ldv) {
  return bse_tridiag_eig_flags(ctx, N, alpha, lambda, V, ldv, 0u);
}

}  // extern "C"
