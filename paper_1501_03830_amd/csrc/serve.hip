// Request server: continuous batching of independent eigensolves.
//
// Requests are queued by bse_submit.  A fixed set of slots -- each a host
// worker thread with its own HIP stream -- takes work from the queue: the
// oldest request that fits in the free device memory, together with queued
// requests of similar size (order within a factor of two) up to a batch
// limit, is solved as one batch through the batched chain (one launch per
// step for all members).  Requests that arrive while other batches are on
// the device are admitted as soon as a slot and memory are free, so their
// work overlaps with the running batches on the device.
//
// Memory: one device pool, carved by a first-fit allocator into one region
// per request (its factors, reflectors and eigenvector workspace) and one
// small descriptor region per batch.  A request's region stays resident
// after it completes, until bse_release.  Admission is by the footprint of
// bse_footprint_bytes; the oldest request is never bypassed by a later one
// that would take memory it needs (no starvation of large requests).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "driver.h"
#include "serve.h"

namespace bse {

namespace {

constexpr size_t ALIGN = 256;

// First-fit allocator over [0, size) with coalescing of free blocks.
class PoolAlloc {
 public:
  void init(size_t size) {
    free_.clear();
    free_[0] = size;
    size_ = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + ALIGN - 1) / ALIGN * ALIGN;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
  size_t size_ = 0, used_ = 0;
};

struct Req {
  bse_request r{};
  long N = 0;
  size_t bytes = 0;     // workspace footprint
  size_t off = 0;       // region in the pool while admitted or resident
  bool has_region = false;
  int state = BSE_QUEUED;
  int info = 0;
  hipEvent_t ready = nullptr;   // recorded on the caller's stream at submission
  double t_submit = 0, t_start = 0, t_done = 0;
};

double now_us(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct Server {
  int device = 0;
  char* pool = nullptr;
  PoolAlloc alloc;
  int max_batch = 64;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<Lane> lanes;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  // statistics
  long long batches = 0, solved = 0, max_inflight = 0, inflight = 0;
  size_t peak_used = 0;
};

namespace {

bool same_kind(const Req& a, const Req& b) {
  return ((a.r.flags ^ b.r.flags) & BSE_WANT_VECTORS) == 0 && a.r.prec == b.r.prec;
}

// Runs one batch on lane k; called without the lock held.
int solve_batch(Server* S, int k, std::vector<Req*>& batch, size_t hdr_off) {
  Lane* L = &S->lanes[k];
  std::sort(batch.begin(), batch.end(), [](const Req* a, const Req* b) { return a->N > b->N; });
  const int count = (int)batch.size();
  std::vector<long> Ns(count);
  std::vector<char*> bases(count);
  for (int i = 0; i < count; ++i) {
    Ns[i] = batch[i]->N;
    bases[i] = S->pool + batch[i]->off;
  }
  Setup St;
  BSE_TRY(setup_batch(L, count, Ns.data(), batch[0]->r.prec, S->pool + hdr_off, bases.data(), &St));
  for (int i = 0; i < count; ++i) {
    const bse_request& r = batch[i]->r;
    Prob& P = L->hprobs[i];
    P.A = static_cast<const double*>(r.A);
    P.lda = r.lda;
    P.B = static_cast<const double*>(r.B);
    P.ldb = r.ldb;
    P.lambda = r.lambda;
    const bool vec = (r.flags & BSE_WANT_VECTORS) != 0;
    P.X = vec ? static_cast<double*>(r.X) : nullptr;
    P.ldx = vec ? r.ldx : 0;
    P.dr = static_cast<const double*>(r.d_r);
    P.dl = static_cast<const double*>(r.d_l);
    P.w = static_cast<double*>(r.w);
    P.flags = r.flags;
  }
  // inputs written on the caller's stream before bse_submit are complete
  // before this batch reads them
  for (int i = 0; i < count; ++i) BSE_HIP(hipStreamWaitEvent(L->stream, batch[i]->ready, 0));
  const bool vectors = (batch[0]->r.flags & BSE_WANT_VECTORS) != 0;
  BSE_TRY(run_chain(L, St, count, vectors, nullptr));
  for (int i = 0; i < count; ++i) {
    const int i0 = L->hinfo[2 * i], i1 = L->hinfo[2 * i + 1];
    batch[i]->info = info_code(i0, i1, vectors);
  }
  return 0;
}

void worker(Server* S, int k) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (!S->stop) {
    if (S->queue.empty()) {
      S->cv.wait(lk);
      continue;
    }
    // the oldest request, then companions of similar size and kind
    const uint64_t head_t = S->queue.front();
    Req& head = S->reqs[head_t];
    size_t hdr_off = 0;
    if (!S->alloc.alloc(header_bytes(S->max_batch), &hdr_off)) {
      S->cv.wait(lk);
      continue;
    }
    if (!S->alloc.alloc(head.bytes, &head.off)) {
      S->alloc.release(hdr_off, header_bytes(S->max_batch));
      S->cv.wait(lk);   // wait for memory: a release or a finished batch
      continue;
    }
    head.has_region = true;
    std::vector<uint64_t> tickets{head_t};
    std::vector<Req*> batch{&head};
    for (auto it = S->queue.begin() + 1; it != S->queue.end() && (int)batch.size() < S->max_batch; ++it) {
      Req& q = S->reqs[*it];
      if (!same_kind(q, head)) continue;
      if (q.r.n * 2 < head.r.n || q.r.n > 2 * head.r.n) continue;
      if (!S->alloc.alloc(q.bytes, &q.off)) continue;
      q.has_region = true;
      tickets.push_back(*it);
      batch.push_back(&q);
    }
    for (uint64_t t : tickets) S->queue.erase(std::find(S->queue.begin(), S->queue.end(), t));
    const double ts = now_us(S->t0);
    for (Req* r : batch) {
      r->state = BSE_RUNNING;
      r->t_start = ts;
    }
    S->inflight += (long long)batch.size();
    S->max_inflight = std::max(S->max_inflight, S->inflight);
    S->peak_used = std::max(S->peak_used, S->alloc.used());
    ++S->batches;
    lk.unlock();
    const int rc = solve_batch(S, k, batch, hdr_off);
    lk.lock();
    const double td = now_us(S->t0);
    S->alloc.release(hdr_off, header_bytes(S->max_batch));
    for (Req* r : batch) {
      if (rc != 0) r->info = rc;
      r->state = (r->info == 0) ? BSE_DONE : BSE_FAILED;
      r->t_done = td;
      (void)hipEventDestroy(r->ready);
      r->ready = nullptr;
    }
    S->inflight -= (long long)batch.size();
    S->solved += (long long)batch.size();
    S->cv.notify_all();
  }
}

}  // namespace

int server_create(int device, size_t pool_bytes, int slots, int max_batch, Server** out) {
  *out = nullptr;
  BSE_HIP(hipSetDevice(device));
  if (pool_bytes == 0) {
    size_t fr = 0, tot = 0;
    BSE_HIP(hipMemGetInfo(&fr, &tot));
    pool_bytes = fr / 2;
  }
  pool_bytes = pool_bytes / ALIGN * ALIGN;
  if (slots <= 0) slots = 4;
  if (max_batch <= 0) max_batch = 64;
  Server* S = new Server();
  S->device = device;
  S->max_batch = max_batch;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&S->pool), pool_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return set_error(BSE_ENOMEM, "request pool allocation failed");
  }
  S->alloc.init(pool_bytes);
  S->lanes.resize(slots);
  for (int k = 0; k < slots; ++k) {
    e = hipStreamCreateWithFlags(&S->lanes[k].stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (int q = 0; q < k; ++q) (void)hipStreamDestroy(S->lanes[q].stream);
      (void)hipFree(S->pool);
      delete S;
      return set_hip_error(e, "hipStreamCreateWithFlags", __FILE__, __LINE__);
    }
  }
  for (int k = 0; k < slots; ++k) S->workers.emplace_back(worker, S, k);
  *out = S;
  return 0;
}

void server_destroy(Server* S) {
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv.notify_all();
  }
  for (auto& t : S->workers) t.join();
  for (auto& kv : S->reqs)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  for (auto& L : S->lanes) {
    (void)hipStreamSynchronize(L.stream);
    lane_release(&L);
    (void)hipStreamDestroy(L.stream);
  }
  (void)hipFree(S->pool);
  delete S;
}

int server_submit(Server* S, const bse_request* r, hipStream_t caller, uint64_t* ticket) {
  Req q;
  q.r = *r;
  q.N = 2L * r->n;
  q.bytes = problem_bytes(q.N, r->prec);
  if (q.bytes + header_bytes(S->max_batch) > S->alloc.size())
    return set_error(BSE_ENOMEM, "request footprint exceeds the request pool");
  BSE_HIP(hipEventCreateWithFlags(&q.ready, hipEventDisableTiming));
  hipError_t e = hipEventRecord(q.ready, caller);
  if (e != hipSuccess) {
    (void)hipEventDestroy(q.ready);
    return set_hip_error(e, "hipEventRecord", __FILE__, __LINE__);
  }
  std::lock_guard<std::mutex> g(S->mu);
  q.t_submit = now_us(S->t0);
  const uint64_t t = S->next_ticket++;
  S->reqs.emplace(t, q);
  S->queue.push_back(t);
  *ticket = t;
  S->cv.notify_all();
  return 0;
}

int server_poll(Server* S, uint64_t ticket, int* state, int* info) {
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(BSE_ENOTICKET, "unknown ticket");
  if (state) *state = it->second.state;
  if (info) *info = it->second.info;
  return 0;
}

int server_release(Server* S, uint64_t ticket) {
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(BSE_ENOTICKET, "unknown ticket");
  Req& q = it->second;
  if (q.state == BSE_RUNNING) return set_error(BSE_EBUSY, "request is running");
  if (q.state == BSE_QUEUED) {
    S->queue.erase(std::find(S->queue.begin(), S->queue.end(), ticket));
    (void)hipEventDestroy(q.ready);
  }
  if (q.has_region) S->alloc.release(q.off, q.bytes);
  S->reqs.erase(it);
  S->cv.notify_all();
  return 0;
}

int server_times(Server* S, uint64_t ticket, double* ts, double* tb, double* td) {
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(BSE_ENOTICKET, "unknown ticket");
  if (ts) *ts = it->second.t_submit;
  if (tb) *tb = it->second.t_start;
  if (td) *td = it->second.t_done;
  return 0;
}

int server_stats(Server* S, bse_serve_counters* st) {
  std::lock_guard<std::mutex> g(S->mu);
  memset(st, 0, sizeof(*st));
  st->pool_bytes = S->alloc.size();
  st->used_bytes = S->alloc.used();
  st->peak_used_bytes = S->peak_used;
  st->queued = (long long)S->queue.size();
  st->inflight = S->inflight;
  st->max_inflight = S->max_inflight;
  st->batches = S->batches;
  st->solved = S->solved;
  st->slots = (int)S->lanes.size();
  return 0;
}

}  // namespace bse
