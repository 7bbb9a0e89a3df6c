// Internal interface between the solve driver (solver.hip) and the request
// server (serve.hip): per-problem workspace layout, execution lanes and the
// batched chain of Algorithm 1 / Algorithm 3.
#pragma once

#include <vector>

#include "common.h"
#include "kernels.h"

namespace bse {

// Execution resources of one chain at a time: a stream and pinned host
// mirrors of the batch descriptors and info words.
struct Lane {
  hipStream_t stream = nullptr;
  Prob* hprobs = nullptr;   // pinned host mirror of the descriptors
  int* hinfo = nullptr;     // pinned host copy of the info words
  int* hstate = nullptr;    // pinned host copy of the refinement state words
  double* hrefout = nullptr;   // pinned host copy of the refinement maxima
  int hcap = 0;
  hipEvent_t ev[BSE_NUM_STAGES + 1] = {};
  bool events = false;
  bool timing = false;                 // per-launch timing of the skew matvec
  std::vector<hipEvent_t> kev;         // event pool for it
  // graph replay of the chain after the Cholesky (FP64 batches): captured
  // once per batch shape on a stream of the lane's own, replayed on `stream`
  bool graphs = false;
  hipStream_t cap = nullptr;
  struct GraphEntry {
    std::vector<long> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<GraphEntry> gcache;      // most recently used last
  long graph_captures = 0, graph_replays = 0;
};
int lane_reserve(Lane* L, int count);   // host mirrors for `count` problems
void lane_release(Lane* L);             // frees events and host mirrors

// Device workspace of one problem of order N (bytes, 256-aligned) and of the
// descriptor/info header of a batch of `count` problems.
size_t problem_bytes(long N, int prec);
size_t header_bytes(int count);

// Descriptor storage of a batch in device memory.
struct Setup {
  int count = 0;            // descriptor slots
  Prob* dprobs = nullptr;   // device descriptors (count)
  int* dinfo = nullptr;     // device info words, 2 per problem slot
  int* dstate = nullptr;    // device refinement state words, 1 per slot
  int* dreorth = nullptr;   // device Gram-Schmidt flags, 1 per slot
  double* dref = nullptr;   // device refinement maxima, 2 per slot
  int* dwgpre = nullptr;    // device workgroup prefixes, SKTRD_NB rows of 2 (count + 1)
  size_t total = 0;         // workspace bytes of the batch (for reports)
};
// Header at `header` (header_bytes(count)); descriptor slot i gets the
// workspace at bases[i] (problem_bytes(Ns[i], prec)) and info words 2i, 2i+1.
// The host mirror L->hprobs[0..count) is filled; callers then set the
// caller-buffer fields (A, B, lambda, X, ...).
int setup_batch(Lane* L, int count, const long* Ns, int prec, char* header, char* const* bases, Setup* S);

// The chain for the batch in L->hprobs[0..count) (sorted by decreasing N).
// Blocks until the device work is done.  On return L->hinfo[2i], [2i+1]
// hold, for descriptor slot i, the Cholesky info of M (> 0: not definite)
// and of the cluster Gram matrix (> 0: reorthogonalisation failed).
int run_chain(Lane* L, const Setup& S, int count, bool vectors, bse_report* rep);

int set_error(int code, const char* msg);

// Return code of one problem from its info words: info[0] (Cholesky of M,
// > 0: not definite) first, then info[1]: INFO_NOCONV (refinement not
// converged) or > 0 (cluster Gram matrix not definite, with eigenvectors).
inline int info_code(int i0, int i1, bool vectors) {
  if (i0 != 0) return i0;
  if (i1 == INFO_NOCONV) return BSE_ENOCONV;
  if (vectors && i1 > 0) return BSE_EDEVICE;
  return 0;
}

bool valid_prec(int prec);
// The precision policy a call runs with: BSE_PREC_FP32_REFINE refines an
// eigenvector basis, so a call that wants eigenvalues only runs the FP64
// path (faster than the FP32 reduction plus the refinement, and as accurate).
inline int run_prec(int prec, unsigned flags) {
  return (prec == BSE_PREC_FP32_REFINE && !(flags & BSE_WANT_VECTORS)) ? BSE_PREC_FP64 : prec;
}
// Argument checks of bse_solve from argument 2 on (0 or -i with the message
// for bse_last_error()).
int check_solve_args(int n, const void* A, int lda, const void* B, int ldb, int prec, unsigned flags,
                     const double* lambda, const void* X, int ldx, const void* d_r, const void* w,
                     bool need_B = true);
// One problem (arguments already checked) on the lane's stream, with its
// workspace at `base`: the batch header (header_bytes(1)) and then the
// problem (problem_bytes(2n, prec)).  B == NULL solves the Tamm-Dancoff
// Hamiltonian (B = 0).  Returns what bse_solve returns.
int solve_single_in(Lane* L, char* base, int n, const void* A, int lda, const void* B, int ldb, int prec,
                    unsigned flags, double* lambda, void* X, int ldx, const void* d_r, const void* d_l,
                    void* w, bse_report* rep);

// Set-up of the allocation-free entry point on the current device (once per
// device; noalloc.hip).
int noalloc_init_device(int device);

}  // namespace bse

// A context: device, the caller's stream, workspace and the request server.
namespace bse { struct Server; }
struct bse_ctx {
  int device = 0;
  void* arena = nullptr;        // caller-provided workspace (not owned)
  size_t arena_bytes = 0;
  void* own = nullptr;          // library-owned workspace
  size_t own_bytes = 0;
  bse::Lane lane;               // the caller's stream and host mirrors
  bse::Server* server = nullptr;   // request server, made on first use
};
