// Launch checks and the host-only dry run of a launch plan.
//
// check_launch() is called before every kernel launch of the library.  It
// rejects a launch that the dispatch packet cannot express (an empty grid
// dimension, more than 2^32 - 1 work-items in one dimension, a workgroup of
// more than 1024 work-items) or that exceeds the LDS or kernel-argument
// limits, instead of handing it to the runtime.
//
// bse_plan_check() runs the solve driver for given problem sizes with the
// dry-run flag on: every runtime call is skipped, every launch is checked
// and recorded but not made, and the device-to-host reads the driver makes
// (info words, refinement states) read as zeros, i.e. the path where every
// problem is definite and the refinement takes every sweep.  No GPU is
// needed: it checks the launch sequence the library would issue, at any size.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "driver.h"

namespace bse {

namespace {

struct KernelStats {
  long launches = 0;
  unsigned gmin[3] = {~0u, ~0u, ~0u};
  unsigned gmax[3] = {0, 0, 0};
  unsigned bmax = 0;
  size_t kmax = 0;
  size_t lmax = 0;
};

thread_local bool t_dry = false;
thread_local std::map<std::string, KernelStats>* t_rec = nullptr;

constexpr unsigned long long kMaxWorkItems = 0xffffffffull;   // per dimension of a dispatch packet
constexpr size_t kMaxLds = 160 * 1024;
constexpr size_t kMaxKernarg = 4096;

}  // namespace

bool dry_run() { return t_dry; }

int check_launch(const char* name, dim3 grid, dim3 block, size_t dyn_lds, size_t kernarg_bytes) {
  const unsigned g[3] = {grid.x, grid.y, grid.z};
  const unsigned b[3] = {block.x, block.y, block.z};
  char why[160] = {0};
  if (g[0] == 0 || g[1] == 0 || g[2] == 0) snprintf(why, sizeof(why), "an empty grid dimension");
  else if (b[0] == 0 || b[1] == 0 || b[2] == 0 || (unsigned long long)b[0] * b[1] * b[2] > 1024)
    snprintf(why, sizeof(why), "a workgroup of %u x %u x %u", b[0], b[1], b[2]);
  else if (g[1] > 65535 || g[2] > 65535) snprintf(why, sizeof(why), "grid y or z above 65535");
  else {
    for (int d = 0; d < 3; ++d)
      if ((unsigned long long)g[d] * b[d] > kMaxWorkItems) snprintf(why, sizeof(why), "more than 2^32 - 1 work-items in dimension %d", d);
  }
  if (!why[0] && dyn_lds > kMaxLds) snprintf(why, sizeof(why), "%zu bytes of dynamic LDS", dyn_lds);
  if (!why[0] && kernarg_bytes > kMaxKernarg) snprintf(why, sizeof(why), "%zu bytes of kernel arguments", kernarg_bytes);
  if (why[0]) {
    char buf[512];
    snprintf(buf, sizeof(buf), "launch of %s with grid (%u, %u, %u) x (%u, %u, %u): %s", name, g[0], g[1], g[2], b[0], b[1],
             b[2], why);
    return set_error(BSE_EDEVICE, buf);
  }
  if (t_rec) {
    KernelStats& k = (*t_rec)[name];
    ++k.launches;
    for (int d = 0; d < 3; ++d) {
      k.gmin[d] = std::min(k.gmin[d], g[d]);
      k.gmax[d] = std::max(k.gmax[d], g[d]);
    }
    k.bmax = std::max(k.bmax, b[0] * b[1] * b[2]);
    k.kmax = std::max(k.kmax, kernarg_bytes);
    k.lmax = std::max(k.lmax, dyn_lds);
  }
  return 0;
}

}  // namespace bse

using namespace bse;

extern "C" int bse_plan_check(int count, const int* n, int prec, unsigned flags, char* summary, size_t summary_bytes) {
  if (count <= 0) return set_error(-1, "count must be positive");
  if (!n) return set_error(-2, "n is NULL");
  if (!valid_prec(prec)) return set_error(-3, "unsupported precision policy");
  if (flags & ~(BSE_WANT_VECTORS | BSE_WANT_WEIGHTS | BSE_TWO_STAGE | BSE_EIGVEC_TWISTED)) return set_error(-4, "unknown flags");
  if ((flags & BSE_TWO_STAGE) && count != 1) return set_error(-4, "the two-stage reduction runs one problem at a time");
  for (int i = 0; i < count; ++i)
    if (n[i] <= 0) return set_error(-2, "n must be positive");
  const bool vec = (flags & BSE_WANT_VECTORS) != 0;
  prec = run_prec(prec, flags);
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
  std::vector<long> Ns(count);
  for (int k = 0; k < count; ++k) Ns[k] = 2L * n[order[k]];
  // addresses only: nothing is dereferenced on the host or launched
  char* fake = reinterpret_cast<char*>(0x100000000000ull);
  std::vector<char*> bases(count);
  size_t off = header_bytes(count);
  for (int k = 0; k < count; ++k) {
    bases[k] = fake + off;
    off += problem_bytes(Ns[k], prec);
  }
  std::vector<Prob> hprobs(count);
  std::vector<int> hinfo(2 * count, 0), hstate(count, 0);
  std::vector<double> hrefout(2 * count, 0.0);
  Lane L;
  L.hprobs = hprobs.data();
  L.hinfo = hinfo.data();
  L.hstate = hstate.data();
  L.hrefout = hrefout.data();
  L.hcap = count;
  std::map<std::string, KernelStats> rec;
  t_dry = true;
  t_rec = &rec;
  Setup S;
  int rc = setup_batch(&L, count, Ns.data(), prec, fake, bases.data(), &S);
  if (rc == 0) {
    for (int k = 0; k < count; ++k) {
      Prob& P = L.hprobs[k];
      P.A = reinterpret_cast<const double*>(fake);
      P.lda = n[order[k]];
      P.B = reinterpret_cast<const double*>(fake);
      P.ldb = n[order[k]];
      P.lambda = reinterpret_cast<double*>(fake);
      P.X = vec ? reinterpret_cast<double*>(fake) : nullptr;
      P.ldx = vec ? 2 * n[order[k]] : 0;
      P.flags = flags;
    }
    rc = run_chain(&L, S, count, vec, nullptr);
  }
  t_dry = false;
  t_rec = nullptr;
  if (summary && summary_bytes) {
    std::string out;
    long total = 0;
    for (auto& kv : rec) total += kv.second.launches;
    char line[512];
    snprintf(line, sizeof(line), "status %d launches %ld workspace %zu\n", rc, total, off);
    out += line;
    for (auto& kv : rec) {
      const KernelStats& k = kv.second;
      snprintf(line, sizeof(line), "%s launches %ld grid_min %u %u %u grid_max %u %u %u block_max %u kernarg_max %zu lds_max %zu\n",
               kv.first.c_str(), k.launches, k.gmin[0], k.gmin[1], k.gmin[2], k.gmax[0], k.gmax[1], k.gmax[2], k.bmax,
               k.kmax, k.lmax);
      out += line;
    }
    const size_t m = std::min(out.size(), summary_bytes - 1);
    memcpy(summary, out.data(), m);
    summary[m] = 0;
  }
  return rc;
}
