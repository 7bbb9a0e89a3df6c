// Allocation-free solve (bse_solve_noalloc) for callers that cannot allocate
// device or pinned host memory: code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc.
//
// The workspace of one problem (batch header, then the problem's matrices)
// lives in a file-scope device array of fixed size, one copy per device.  In
// host code the array's name is only a stand-in for the symbol, not a device
// address: its address on each device is looked up once, with that device
// current, when the first context on the device is created, and only that
// address is ever handed to kernels.  The host mirrors of the descriptor and
// the info words are static host arrays, one set per device.
//
// The array is shared by every call on a device and keeps the last call's
// contents; the chain writes every workspace entry before reading it (as it
// does with a reused context workspace), so nothing needs clearing.  Calls
// that overlap on one device (two host threads, or two streams) race on the
// array and on the host mirrors: serialise them.
#include <cstring>
#include <mutex>

#include "driver.h"

namespace bse {

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[BSE_NOALLOC_MAX_BYTES];

struct DeviceState {
  char* scratch = nullptr;   // device address of `scratch` on this device
  Prob probs[1];             // host mirror of the descriptor
  int info[2];
  int state[1];
  double refout[2];
};

std::mutex g_mu;
DeviceState g_dev[kMaxDevices];

}  // namespace

int noalloc_init_device(int device) {
  if (device < 0 || device >= kMaxDevices) return set_error(BSE_EUNSUPPORTED, "device index beyond the no-alloc table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_dev[device].scratch) return 0;
  void* p = nullptr;
  BSE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return set_error(BSE_EDEVICE, "no device address for the no-alloc scratch array");
  g_dev[device].scratch = static_cast<char*>(p);
  return 0;
}

}  // namespace bse

using namespace bse;

extern "C" size_t bse_noalloc_max_bytes(void) { return BSE_NOALLOC_MAX_BYTES; }

extern "C" int bse_solve_noalloc(bse_ctx* ctx, int n, const void* A, int lda, const void* B, int ldb, int prec,
                                 unsigned flags, double* lambda, void* X, int ldx, const void* d_r,
                                 const void* d_l, void* w) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  BSE_TRY(check_solve_args(n, A, lda, B, ldb, prec, flags, lambda, X, ldx, d_r, w));
  prec = run_prec(prec, flags);
  const size_t need = header_bytes(1) + problem_bytes(2L * n, prec);
  if (need > (size_t)BSE_NOALLOC_MAX_BYTES)
    return set_error(BSE_ENOMEM, "problem too large for the no-alloc scratch array (bse_noalloc_max_bytes)");
  if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_dev[ctx->device].scratch)
    return set_error(BSE_EDEVICE, "no-alloc scratch array not set up on this device");
  BSE_HIP(hipSetDevice(ctx->device));
  DeviceState& D = g_dev[ctx->device];
  Lane L;                    // no events, no timing, static host mirrors
  L.stream = ctx->lane.stream;
  L.hprobs = D.probs;
  L.hinfo = D.info;
  L.hstate = D.state;
  L.hrefout = D.refout;
  L.hcap = 1;
  return solve_single_in(&L, D.scratch, n, A, lda, B, ldb, prec, flags, lambda, X, ldx, d_r, d_l, w, nullptr);
}
