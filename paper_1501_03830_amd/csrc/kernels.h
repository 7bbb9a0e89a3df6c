// Host-side launchers of the gfx950 kernels.  Every launcher returns 0 or a
// BSE_* error code and enqueues work on the given stream only.
#pragma once

#include "common.h"

namespace bse {

// ---------------------------------------------------------------- gemm.hip
// Scratch buffer for split-K products issued from this host thread (set by
// the driver before a solve; NULL disables splitting).
void gemm_set_scratch(double* scratch, size_t bytes);
int gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
             long lda, const double* B, long ldb, double beta, double* C, long ldc, int c_uplo,
             int a_tri, int b_tri);

// ---------------------------------------------------------------- chol.hip
// M (N x N, ld) from the lower triangles of complex A, B (eq. embedding);
// zeros above the diagonal.
int launch_build_M(hipStream_t s, int n, const double* A, long lda, const double* B, long ldb,
                   double* M, long ldm);
// Blocked right-looking Cholesky of the lower triangle of M in place.  The
// first failing leading minor is written to *info_dev (0 = success).
// linv: 64 x 64 doubles of scratch for the inverted diagonal blocks.
int potrf_f64(hipStream_t s, int N, double* M, long ldm, int* info_dev, double* linv, bool reset_info = true);
// Inverse of the lower-triangular diagonal block (b0, b0) of size nbk <= 64
// into Linv (64 x 64, ld 64).  Skipped when *info_dev != 0.
int trtri_diag64(hipStream_t s, const double* L, long ld, int b0, int nbk, double* Linv, const int* info_dev);
// W = L^T J L (lower triangle and the W22 = 0 block only; full=true also
// fills the strict upper triangle with -W^T).
int form_W(hipStream_t s, int N, const double* L, long ldl, double* W, long ldw, bool full);
// copy an m x n column-major block
int copy_matrix(hipStream_t s, int m, int n, const double* src, long lds, double* dst, long ldd);
// set the strict upper triangle of an N x N matrix to zero
int zero_upper(hipStream_t s, int N, double* A, long lda);

// ---------------------------------------------------------------- sktrd.hip
struct SktrdWork {
  double* Y1;        // ld x 2*nb  (v_l, p_l interleaved)
  double* Y2;        // ld x 2*nb  (p_l, -v_l interleaved)
  double* Yrow;      // symv partial row sums, one per 64 x 64 tile
  double* Ycol;      // symv partial column sums, one per strip chunk
  double* dotpart;   // per-block partial dot products
  double* normpart;  // per-block partial squared norms
  void* ctrl;        // device control block
  int nb;
};
size_t sktrd_work_bytes(long N, long ld, int nb);
int sktrd_bind_work(void* base, long N, long ld, int nb, SktrdWork* w);
// Optional per-launch timing of the skew matvec (event pairs from a pool).
struct KernelTimer {
  hipEvent_t* ev = nullptr;
  int cap = 0;    // number of events in the pool
  int used = 0;   // events recorded so far (pairs)
  double bytes = 0.0;
};
int sktrd_f64(hipStream_t s, int N, double* W, long ldw, double* alpha, double* tau, const SktrdWork& w,
              KernelTimer* timer = nullptr);

// ---------------------------------------------------------------- stein.hip
// positive eigenvalues of tridiag(alpha, 0, alpha) by bisection
int tridiag_bisect(hipStream_t s, int N, const double* alpha, double* e2, double* scal, double* lam);
// eigenvectors by inverse iteration; Vt is n x N column-major (ld n):
// Vt[j + k n] = k-th component of the j-th eigenvector
int tridiag_invit(hipStream_t s, int N, const double* alpha, const double* scal, const double* lam,
                  double* shift, double* work, double* Vt);
// Gram-Schmidt inside clusters (Cholesky QR of the cluster-masked Gram matrix)
int tridiag_reorth(hipStream_t s, int N, const double* lam, const double* scal, double* Vt, double* G,
                   int* cid, int* info_dev, double* linv);
// transpose Vt (n x N) into V (N x n, ldv)
int transpose_to(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst, long ldd);

// ---------------------------------------------------------------- backtr.hip
struct BacktrWork {
  double* Vb;   // ld x nbq explicit reflector block
  double* S;    // nbq x nbq Gram / T factor
  double* T;    // nbq x nbq
  double* W1;   // nbq x ld
  double* W2;   // nbq x ld
  int nbq;
};
size_t backtr_work_bytes(long N, long ld, int nbq);
int backtr_bind_work(void* base, long N, long ld, int nbq, BacktrWork* w);
// Z (N x N, ld) = [Re(D V_+) | Im(D V_+)] from Vt
int scatter_DV(hipStream_t s, int N, const double* Vt, double* Z, long ldz);
// Z <- U Z with U = H_0 ... H_{N-3} stored below the subdiagonal of W
int apply_U(hipStream_t s, int N, const double* W, long ldw, const double* tau, double* Z, long ldz,
            int ncols, const BacktrWork& w);
// X = S Q G Lambda^{-1/2} from G = L U D V_+ stored as [Re | Im]
int finish_X(hipStream_t s, int n, const double* G, long ldg, const double* lam, double* X, long ldx);
// canonical phase of each column of X and, when dr != NULL, the weights
int phase_and_weights(hipStream_t s, int n, double* X, long ldx, const double* dr, const double* dl,
                      double* w);

}  // namespace bse
