/*
 * bse.h -- C ABI of the gfx950 (MI355X) structure-preserving eigensolver for
 * Bethe-Salpeter Hamiltonians
 *
 *     H = [ A        B      ]     A = A^H,  B = B^T  (complex n x n),
 *         [ -conj(B) -conj(A)]    Omega = [A B; conj(B) conj(A)] > 0,
 *
 * (Shao, da Jornada, Yang, Deslippe, Louie, arXiv:1501.03830: eq. H-complex,
 * eq. symmetry and the definiteness condition eq. cond).  The solver computes
 * the n positive eigenvalues lambda_1 <= ... <= lambda_n of H and the right
 * eigenvectors x_j = [X1; X2] e_j normalised as in Theorem 3 / Algorithm 1,
 *     H [X1; X2] = [X1; X2] Lambda_+,   X1^H X1 - X2^H X2 = I_n,
 * by the structure-preserving route of Algorithm 1 (real embedding M,
 * Cholesky M = L L^T, skew-symmetric W = L^T J L) carried out as in
 * Algorithm 3 (Householder tridiagonalisation W = U T U^T, bisection and
 * inverse iteration on -i D^H T D, back-transformation).  Left eigenvectors
 * are y_j = S x_j with S = diag(I_n, -I_n), and the eigenvectors of -lambda_j
 * are [conj X2; conj X1] (Theorem 3); neither is stored.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All matrix and vector arguments are DEVICE pointers on the context's
 *    device unless stated otherwise.  The caller owns every buffer it passes;
 *    the library never frees or retains caller memory after a call returns.
 *  - Complex data are complex128, interleaved (re, im), COLUMN-MAJOR with the
 *    given leading dimension counted in complex elements.
 *  - Only the LOWER triangles (diagonal included) of A and B are read.  A row-
 *    major Hermitian array handed over as column-major is conj(A); pass its
 *    transpose.  The imaginary part of A's diagonal is ignored.
 *  - All work is ordered on the context's stream.  Calls are synchronous:
 *    they return after the device work has completed.
 *  - A context is not thread-safe: use one per host thread or serialise.
 *
 * Return values
 * -------------
 *  BSE_OK (0) on success;  -i when argument i (1-based) is invalid;  +k when
 *  the leading k x k minor of the real embedding M is not positive definite,
 *  i.e. eq. cond fails (Algorithm 1 requires it), in which case no outputs
 *  are written;  BSE_ENOMEM when a caller-provided arena is too small;
 *  BSE_ENOCONV when the FP64 refinement of BSE_PREC_FP32_REFINE did not meet
 *  its stopping test within its sweep limit (outputs are written from the
 *  last sweep);  BSE_EDEVICE on a HIP runtime error (details from
 *  bse_last_error()).
 */
#ifndef BSE_H_
#define BSE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSE_OK 0
#define BSE_ENOMEM (-1000)
#define BSE_EDEVICE (-1001)
#define BSE_ENOTICKET (-1002)
#define BSE_EUNSUPPORTED (-1003)
#define BSE_EBUSY (-1004)
#define BSE_ENOCONV (-1005)   /* BSE_PREC_FP32_REFINE: the refinement did not
                                 meet its stopping test within its sweep limit;
                                 the outputs hold the last sweep's result     */

/* precision policies */
#define BSE_PREC_FP64 0        /* every stage in FP64                          */
#define BSE_PREC_FP32_REFINE 1 /* W stored and reduced in FP32 (FP64 sums and
                                  norms, rank-2k updates on the FP32 matrix
                                  cores), FP64 tridiagonal solve, U applied
                                  on the FP32 matrix cores, then FP64
                                  refinement of the eigenpairs against
                                  W = L^T J L through the FP64 Cholesky
                                  factor L.  A call that
                                  wants eigenvalues only (no
                                  BSE_WANT_VECTORS) runs the FP64 path: the
                                  refinement needs the eigenvector basis, and
                                  the FP64 reduction alone is faster and as
                                  accurate                                    */

/* flags for bse_solve */
#define BSE_WANT_VECTORS 1u    /* write X (else only lambda)                   */
#define BSE_WANT_WEIGHTS 2u    /* write the absorption weights w (needs X)      */
#define BSE_TWO_STAGE 4u       /* reduce W to tridiagonal form in two stages
                                  (dense to band on the matrix cores, then
                                  bulge chasing; Section 3.3's successive band
                                  reduction); eigenvectors go back through
                                  both stages' reflectors.  FP64, single
                                  problems (bse_solve, bse_solve_tda,
                                  bse_solve_real)                             */
#define BSE_EIGVEC_TWISTED 8u  /* eigenvectors of the tridiagonal T_s by
                                  twisted factorisations (the per-vector step
                                  of MRRR, Section 3.3) instead of inverse
                                  iteration; eigenvalues closer than 1000 eps
                                  |lambda| to a neighbour still use inverse
                                  iteration, and clusters are orthogonalised
                                  as before (the representation tree of MRRR
                                  is not built).  FP64 and mixed; any entry
                                  point that takes flags                     */

/* stage indices of bse_report.stage_ms */
#define BSE_STAGE_BUILD_M 0    /* Algorithm 1 step 1                           */
#define BSE_STAGE_POTRF 1      /* Algorithm 1 step 2                           */
#define BSE_STAGE_FORM_W 2     /* Algorithm 1 step 3                           */
#define BSE_STAGE_SKTRD 3      /* Algorithm 3 step 1                           */
#define BSE_STAGE_BISECT 4     /* Algorithm 3 step 2, eigenvalues              */
#define BSE_STAGE_INVIT 5      /* Algorithm 3 step 2, eigenvectors             */
#define BSE_STAGE_REORTH 6     /* Algorithm 3 step 2, reorthogonalisation      */
#define BSE_STAGE_APPLY_U 7    /* Algorithm 3 step 3 (U applied to D V_+)      */
#define BSE_STAGE_APPLY_L 8    /* Algorithm 3 step 3 (L applied)               */
#define BSE_STAGE_FINISH 9     /* Algorithm 3 steps 4-6, phase, weights        */
#define BSE_STAGE_REFINE 10    /* mixed path: FP64 refinement (after APPLY_U)  */
#define BSE_NUM_STAGES 11

/* request states reported by bse_poll */
#define BSE_QUEUED 0           /* waiting for a slot and device memory          */
#define BSE_RUNNING 1          /* in a batch on the device                      */
#define BSE_DONE 2             /* outputs written; factors resident             */
#define BSE_FAILED 3           /* info holds the reason                         */

typedef struct bse_ctx bse_ctx;

/* One eigensolve request for bse_submit: the arguments of bse_solve. */
typedef struct bse_request {
  int n;                 /* order of A and B, >= 1                            */
  const void* A;         /* complex n x n, lower triangle read                */
  int lda;               /* >= n                                              */
  const void* B;         /* complex n x n, lower triangle read                */
  int ldb;               /* >= n                                              */
  int prec;              /* BSE_PREC_FP64 or BSE_PREC_FP32_REFINE             */
  unsigned flags;        /* BSE_WANT_VECTORS | BSE_WANT_WEIGHTS |
                            BSE_EIGVEC_TWISTED                               */
  double* lambda;        /* out: n doubles                                    */
  void* X;               /* out: complex 2n x n or NULL without vectors       */
  int ldx;               /* >= 2n with vectors                                */
  const void* d_r;       /* complex 2n, read with BSE_WANT_WEIGHTS            */
  const void* d_l;       /* NULL means d_l = d_r                              */
  void* w;               /* out: n complex weights with BSE_WANT_WEIGHTS      */
} bse_request;

/* Server counters (bse_serve_stats). */
typedef struct bse_serve_counters {
  size_t pool_bytes;         /* device memory of the request pool            */
  size_t used_bytes;         /* held now: running batches + resident results */
  size_t peak_used_bytes;    /* largest value of used_bytes at an admission  */
  long long queued;          /* requests waiting                             */
  long long inflight;        /* requests in batches on the device            */
  long long max_inflight;    /* largest inflight seen                        */
  long long batches;         /* batches started                              */
  long long solved;          /* requests finished (done or failed)           */
  int slots;                 /* concurrent batches (worker streams)          */
} bse_serve_counters;

/* Per-call timing, filled when a non-NULL pointer is passed (host memory). */
typedef struct bse_report {
  double total_ms;                 /* device time of the whole call          */
  double stage_ms[BSE_NUM_STAGES]; /* device time per stage (hipEvents)      */
  int n;                           /* problem size of the call               */
  int prec;                        /* precision policy used                  */
  size_t workspace_bytes;          /* device workspace the call used         */
  /* Filled only while kernel timing is on (bse_ctx_set_timing): hipEvents
   * around every launch of the tiled skew matrix-vector kernel of the
   * tridiagonalisation (Algorithm 3 step 1), the dominant HBM-bound kernel. */
  double symv_ms;                  /* summed device time of those launches   */
  double symv_bytes;               /* algorithmic bytes they must read: the
                                      strictly lower triangle of each trailing
                                      matrix, 8 bytes per element             */
  long long symv_launches;         /* number of launches                     */
  int refine_sweeps;               /* mixed path: refinement sweeps run      */
  double refine_first_correction;  /* mixed path: largest correction entry of
                                      the first sweep (the size of the
                                      unrefined eigenvector error)           */
  double refine_correction;        /* ... and of the last sweep              */
  int graph;                       /* 1 when the chain after the Cholesky ran
                                      as a replayed HIP graph (its stages are
                                      then not timed one by one: their sum is
                                      reported under BSE_STAGE_FORM_W)        */
} bse_report;

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int bse_version(void);

/* Text of the last error recorded on this host thread ("" if none).  The
 * returned pointer stays valid until the next failing call on the thread. */
const char* bse_last_error(void);

/* Create a context bound to HIP device `device` and HIP stream `stream`
 * (a hipStream_t, NULL for the default stream).  `arena`/`arena_bytes`: an
 * optional caller-owned device buffer used for all workspace; when NULL the
 * library allocates workspace itself with hipMalloc, grows it on demand and
 * frees it in bse_ctx_destroy.  Returns -1 if ctx is NULL, -2 for a bad
 * device, -4 if arena_bytes is non-zero without an arena. */
int bse_ctx_create(bse_ctx** ctx, int device, void* arena, size_t arena_bytes, void* stream);

/* Destroy a context (waits for its stream).  NULL is accepted. */
int bse_ctx_destroy(bse_ctx* ctx);

/* Turn per-launch timing of the dominant kernel on (enable != 0) or off for
 * later calls on this context.  Adds two hipEventRecord per launch.
 * Returns -1 for a NULL context. */
int bse_ctx_set_timing(bse_ctx* ctx, int enable);

/* Tile table of the tridiagonalisation's skew matrix-vector kernel: row
 * tiles per strip workgroup as a function of the trailing matrix's 64-row
 * blocks nblk, in five buckets per storage type: nblk >= t0 -> v0,
 * >= t1 -> v1, >= t2 -> v2, >= t3 -> v3, else v4.  `table` (host) holds
 * 2 x 9 ints [t0 t1 t2 t3 v0 v1 v2 v3 v4], the FP64 row then the FP32 row;
 * thresholds non-increasing and >= 0, tile counts in [1, 16].  The table sets
 * each problem's summation order (so results depend on it, bit for bit the
 * same alone and in a batch).  bse_set_tile_table replaces it for the whole
 * process (validated; the context's device gets the new copy at once, other
 * devices when a context is created on them); it must not run while solves
 * are in flight.  The project's autotuner (paper_1501_03830_amd/autotune.py)
 * measures candidates on the benchmark workloads and writes the table the
 * Python binding applies.  Return 0, -1/-2 for NULL arguments, -3 for an
 * invalid table. */
int bse_get_tile_table(int* table);
int bse_set_tile_table(bse_ctx* ctx, const int* table);

/* Graph replay (enable != 0, the default) or plain stream launches for later
 * bse_solve / bse_solve_batched calls on this context.  With replay, the
 * launches after the Cholesky of an FP64 call (W, reduction, tridiagonal
 * eigensolve, back-transformation: thousands of kernels for one batch) are
 * captured into a HIP graph the first time a batch shape (the problems'
 * orders, the policy, whether vectors are wanted) is solved on this context
 * and replayed on the context's stream afterwards; results are bit for bit
 * those of plain launches.  Up to 8 shapes are kept per context.  Calls with
 * per-launch timing, the mixed policy, BSE_TWO_STAGE or real inputs always
 * launch plainly.  Returns -1 for a NULL context. */
int bse_ctx_set_graphs(bse_ctx* ctx, int enable);

/* Device workspace, in bytes, that bse_solve needs for size n (host-only
 * arithmetic, callable without a GPU).  0 for invalid arguments. */
size_t bse_footprint_bytes(int n, int prec, unsigned flags);

/*
 * Full structure-preserving eigensolve (Algorithm 1 as organised by
 * Algorithm 3).
 *   ctx      context (argument 1)
 *   n        order of A and B, n >= 1 (2)
 *   A, lda   complex n x n, lda >= n, lower triangle read (3, 4)
 *   B, ldb   complex n x n, ldb >= n, lower triangle read (5, 6)
 *   prec     BSE_PREC_FP64, or BSE_PREC_FP32_REFINE: W is reduced to
 *            tridiagonal form in FP32 storage (FP64 sums and norms, FP32
 *            matrix-core rank-2k updates), the tridiagonal eigensolve runs in
 *            FP64 and U is applied on the FP32 matrix cores, then the
 *            eigenpairs are refined in FP64 against W = L^T J L by
 *            sweeps of an Ogita-Aishima-type iteration on the real Schur
 *            form of W (not in the paper), until the largest correction is
 *            below 1e-2 with no pair left out (at most 6 sweeps; pairs closer
 *            than 1e-6 relative, which the FP32 reduction cannot separate,
 *            are resolved by an exact FP64 rotation of their cluster);
 *            eigenvalues are then taken from the refined basis (error about
 *            3.5e-5 x correction^4 relative, i.e. below 4e-13; eigenvector
 *            error about correction^2).  Returns BSE_ENOCONV when the sweep
 *            limit is reached first (7)
 *   flags    BSE_WANT_VECTORS | BSE_WANT_WEIGHTS | BSE_TWO_STAGE |
 *            BSE_EIGVEC_TWISTED (8)
 *   lambda   out: n doubles, the positive eigenvalues ascending (9)
 *   X, ldx   out: complex 2n x n, ldx >= 2n; rows 0..n-1 hold X1, rows
 *            n..2n-1 hold X2; each column is scaled by a unit phase so that
 *            its largest-modulus entry (lowest row on ties) is real positive
 *            (10, 11).  May be NULL without BSE_WANT_VECTORS.
 *   d_r, d_l in: complex 2n dipole vectors of eq. absp (12, 13); d_l NULL
 *            means d_l = d_r.  Read only with BSE_WANT_WEIGHTS.
 *   w        out: n complex weights w_j = (d_r^H x_j)(y_j^H d_l)/(y_j^H x_j)
 *            of eq. absp, y_j = S x_j (14).
 *   rep      optional host report (15).
 */
int bse_solve(bse_ctx* ctx, int n, const void* A, int lda, const void* B, int ldb, int prec,
              unsigned flags, double* lambda, void* X, int ldx, const void* d_r, const void* d_l,
              void* w, bse_report* rep);

/*
 * Real Bethe-Salpeter problem (eq. H-real, Section 3.2, Theorem 5,
 * Algorithm 2): A, B real symmetric n x n (FP64, column-major, lower
 * triangles read) with A + B > 0 and A - B > 0.  The real embedding is then
 * M = blkdiag(A + B, A - B), whose Cholesky factor is blkdiag(L1, L2) with
 * the two factors of Algorithm 2 step 1, and W = L^T J L = [0 L1^T L2;
 * -L2^T L1 0]: its eigenvalues are +-i sigma_j for the singular values
 * sigma_j of L2^T L1 (Algorithm 2 step 2) and its Schur vectors carry the
 * singular vectors, so the same reduction, tridiagonal solve and
 * back-transformation give Lambda_+ and X1, X2 of Algorithm 2 step 3 (with
 * Theorem 5's factor 1/2 and Lambda_+^{-1/2}).
 *   A, lda, B, ldb (3-6): real; prec (7), flags (8), lambda (9) as in
 *   bse_solve; X, ldx (10, 11): REAL 2n x n, ldx >= 2n, X1 over X2 with
 *   X1^T X1 - X2^T X2 = I, each column's largest-modulus entry positive
 *   (inside a group of equal eigenvalues, a real orthonormal basis of the
 *   eigenspace); d_r, d_l, w (12-14): complex dipoles and weights as in
 *   bse_solve; rep (15).  Returns +k when the leading k x k minor of A + B
 *   (k <= n) or the leading (k - n) x (k - n) minor of A - B (k > n) is not
 *   positive definite.
 */
int bse_solve_real(bse_ctx* ctx, int n, const double* A, int lda, const double* B, int ldb, int prec,
                   unsigned flags, double* lambda, double* X, int ldx, const void* d_r, const void* d_l, void* w,
                   bse_report* rep);

/*
 * Tamm-Dancoff approximation (Section 2.2, Theorem 4): the Bethe-Salpeter
 * problem with the off-diagonal blocks B and -conj(B) set to zero, i.e. the
 * Hermitian eigenproblem of A, solved by the same structure-preserving chain
 * as bse_solve (embedding, Cholesky, W, tridiagonalisation, bisection and
 * inverse iteration, back-transformation).  Arguments as bse_solve without
 * B and ldb (argument numbers shift accordingly): A, lda (3, 4); prec (5);
 * flags (6); lambda (7): the n eigenvalues of A, ascending, which under eq.
 * cond bound those of the full H from above (Theorem 4); X, ldx (8, 9): the
 * eigenvectors as x_j = [v_j; 0] with A v_j = lambda_j v_j, v_j^H v_j = 1
 * (rows n..2n-1 hold rounding-level values of the zero block); d_r, d_l
 * (10, 11) and w (12): the TDA weights of eq. absp, (d_r^H x_j)(x_j^H d_l)
 * here; rep (13).  Returns +k when the leading k x k minor of the real
 * embedding of A is not positive definite (A itself is not).
 */
int bse_solve_tda(bse_ctx* ctx, int n, const void* A, int lda, int prec, unsigned flags, double* lambda,
                  void* X, int ldx, const void* d_r, const void* d_l, void* w, bse_report* rep);

/*
 * Broadened spectra (eq. DOS and eq. absp, with each delta function replaced
 * by the Gaussian exp(-t^2 / (2 sigma^2)) / (sqrt(2 pi) sigma) that Section 4
 * uses for its spectral-density figure) on the uniform grid
 * omega_k = omega0 + k domega, k = 0..npts-1:
 *   dos[k] = 1/(2n) sum over the 2n eigenvalues +-lambda_j of H,
 *   eps[k] = sum_j w_j delta(omega_k - lambda_j)  (complex).
 *   lambda (3): n positive eigenvalues (device), w (4): n complex weights
 *   (device; needed for eps), npts (5) > 0, omega0 (6), domega (7) >= 0,
 *   sigma (8) > 0, dos (9): npts doubles or NULL, eps (10): npts complex or
 *   NULL (not both NULL).  Device outputs, stream-ordered, synchronous.
 */
int bse_spectra(bse_ctx* ctx, int n, const double* lambda, const void* w, int npts, double omega0,
                double domega, double sigma, double* dos, void* eps);

/* Device workspace, in bytes, of one bse_solve_batched call over `count`
 * problems of orders n[0..count) (host-only arithmetic, callable without a
 * GPU).  0 for invalid arguments. */
size_t bse_footprint_batched_bytes(int count, const int* n, int prec, unsigned flags);

/*
 * Many independent eigensolves in one call: the batched form of bse_solve
 * (Algorithm 1 as organised by Algorithm 3 for each problem).  The problems
 * may differ in n.  They go through the chain together: each step is one
 * launch covering every problem that still has work at that step, so that
 * many small problems fill the device instead of running one after another.
 * Each problem's arithmetic, and so its result, is bit for bit the same as
 * that of bse_solve on the problem alone.
 *
 * Every array argument is a HOST array of `count` entries; the pointers in
 * them are device pointers with the meaning, layout and ownership of the
 * corresponding bse_solve argument.
 *   ctx        context (argument 1)
 *   count      number of problems, >= 0; 0 is a no-op (2)
 *   n, A, lda, B, ldb   per problem, as in bse_solve (3, 4, 5, 6, 7)
 *   prec       BSE_PREC_FP64 or BSE_PREC_FP32_REFINE (as in bse_solve),
 *              shared (8)
 *   flags      BSE_WANT_VECTORS | BSE_WANT_WEIGHTS | BSE_EIGVEC_TWISTED, shared (9)
 *   lambda     out: lambda[i] -> n[i] doubles, ascending (10)
 *   X, ldx     out: X[i] -> complex 2n[i] x n[i], ldx[i] >= 2 n[i], laid out
 *              and phased as in bse_solve; both arrays may be NULL without
 *              BSE_WANT_VECTORS (11, 12)
 *   d          in: d[i] -> complex 2n[i] dipole vector, used as d_r = d_l of
 *              eq. absp; read with BSE_WANT_WEIGHTS, else may be NULL (13)
 *   w          out: w[i] -> n[i] complex weights (14)
 *   info       out, HOST int[count]: 0 on success; +k when the leading k x k
 *              minor of problem i's M is not positive definite (eq. cond
 *              fails; that problem's outputs are not written); BSE_EDEVICE
 *              when its cluster reorthogonalisation failed (15)
 *   rep        optional host report for the whole batch; rep->n is the
 *              largest n (16)
 * Returns 0 when the batch ran (per-problem status in info), -i for invalid
 * argument i (bse_last_error() names the problem), BSE_ENOMEM when the
 * arena is too small for bse_footprint_batched_bytes, BSE_EDEVICE on a HIP
 * error.
 */
int bse_solve_batched(bse_ctx* ctx, int count, const int* n, const void* const* A, const int* lda,
                      const void* const* B, const int* ldb, int prec, unsigned flags,
                      double* const* lambda, void* const* X, const int* ldx, const void* const* d,
                      void* const* w, int* info, bse_report* rep);

/* ---------------------------------------------------------------------------
 * Request serving (continuous batching).  bse_submit queues a solve and
 * returns at once.  A fixed number of slots -- each a library worker thread
 * with its own HIP stream -- takes work from the queue: the oldest request
 * that fits in the free part of the request pool, with queued requests of
 * similar order (within a factor of two) and kind up to a batch limit, is
 * solved as one bse_solve_batched-style batch.  Requests that arrive while
 * other batches run are admitted as soon as a slot and pool memory are
 * free, and their work overlaps with the running batches on the device.
 * The oldest request is never bypassed (no starvation).  Each result is bit
 * for bit the one bse_solve gives for the request alone.
 *
 * Ordering: work queued on the context's stream before bse_submit (for
 * instance the writes that produced A and B) is complete before the request's
 * batch reads its inputs.  Outputs may be read once bse_poll reports
 * BSE_DONE.
 *
 * Ownership: the request's input and output buffers must stay valid until
 * bse_poll reports BSE_DONE or BSE_FAILED.  The request's workspace (its
 * factors L, the reflectors of W and the eigenvector workspace) stays
 * resident in the pool until bse_release; an unreleased result keeps its
 * pool memory, so later requests wait for it.  The server's threads are
 * internal; the context itself is still not thread-safe for callers.
 * ------------------------------------------------------------------------ */

/* Configure the server before the first bse_submit (else defaults are used):
 * pool_bytes of device memory for request workspaces (0: half of the free
 * device memory), `slots` concurrent batches (0: 4; at most 16) and at most
 * `max_batch` requests per batch (0: 64; at most 4096).  The pool is a
 * separate device allocation, independent of the context's arena.  Returns
 * BSE_EBUSY if the server is already running, -3 / -4 for bad slots /
 * max_batch, BSE_ENOMEM if the pool cannot be allocated. */
int bse_serve_config(bse_ctx* ctx, size_t pool_bytes, int slots, int max_batch);

/* Queue a request (argument 2, copied); *ticket (argument 3) identifies it.
 * Returns -2 for an invalid request field (bse_last_error() names it), -3
 * for a NULL ticket, BSE_ENOMEM if its footprint can never fit the pool. */
int bse_submit(bse_ctx* ctx, const bse_request* req, uint64_t* ticket);

/* State of a request: *state one of BSE_QUEUED, BSE_RUNNING, BSE_DONE,
 * BSE_FAILED; *info as bse_solve would return it (0, +k for a minor of M
 * that is not positive definite, or a negative BSE_* code).  Either pointer
 * may be NULL.  Returns BSE_ENOTICKET for an unknown or released ticket. */
int bse_poll(bse_ctx* ctx, uint64_t ticket, int* state, int* info);

/* Release a request: frees its resident workspace (DONE / FAILED) or
 * cancels it (QUEUED).  Returns BSE_EBUSY while it is running and
 * BSE_ENOTICKET for an unknown ticket. */
int bse_release(bse_ctx* ctx, uint64_t ticket);

/* Server-side timestamps of a request in microseconds since the server
 * started: submission, start of its batch, completion (0 if not reached).
 * Any pointer may be NULL. */
int bse_ticket_times(bse_ctx* ctx, uint64_t ticket, double* t_submit_us, double* t_start_us,
                     double* t_done_us);

/* Counters of the server (all zero before the first bse_submit). */
int bse_serve_stats(bse_ctx* ctx, bse_serve_counters* stats);

/* ---------------------------------------------------------------------------
 * Allocation-free solve, for callers that cannot allocate: code under HIP
 * stream capture, tight serving loops and harnesses that forbid hipMalloc
 * or pinned host allocations.  Same arguments, arithmetic and results (bit
 * for bit) as bse_solve without the report; the workspace is a fixed device
 * array inside the library, BSE_NOALLOC_MAX_BYTES (64 MiB) per device, held
 * by each device the library runs on until the process ends.  Problems
 * whose bse_footprint_bytes(n, prec, flags) exceeds it are rejected with
 * BSE_ENOMEM (n <= 544 fits in FP64, n <= 416 with BSE_PREC_FP32_REFINE).
 * The array is set up when the first context on a device is created; the
 * call allocates nothing (no hipMalloc, no pinned host memory, no events).
 * Every call on a device shares the one array: calls that overlap on one
 * device (from several threads or streams) race and must be serialised.
 * ------------------------------------------------------------------------ */
#define BSE_NOALLOC_MAX_BYTES (64u << 20)

/* Size of the fixed workspace array (host-only, callable without a GPU). */
size_t bse_noalloc_max_bytes(void);

int bse_solve_noalloc(bse_ctx* ctx, int n, const void* A, int lda, const void* B, int ldb, int prec,
                      unsigned flags, double* lambda, void* X, int ldx, const void* d_r,
                      const void* d_l, void* w);

/* Host-only check of the launch sequence a bse_solve_batched call over
 * `count` problems of orders n[0..count) would issue (count 1: bse_solve),
 * for the path where every problem is definite and the refinement takes all
 * its sweeps.  Nothing is allocated or launched and no GPU is needed: every
 * launch is checked against the dispatch limits (non-empty grid, at most
 * 2^32 - 1 work-items per dimension, workgroups of at most 1024 work-items,
 * dynamic LDS <= 160 KiB, kernel arguments <= 4 KiB).  Returns 0, or
 * BSE_EDEVICE naming the first launch that violates a limit, or -i for an
 * invalid argument i.  summary (host, may be NULL): text, one line with the
 * status, launch count and workspace bytes, then one line per kernel with
 * its launch count, smallest and largest grid, largest workgroup and
 * argument bytes. */
int bse_plan_check(int count, const int* n, int prec, unsigned flags, char* summary, size_t summary_bytes);

/* ---------------------------------------------------------------------------
 * Stage entry points.  Each runs one step of the chain on caller buffers so
 * that it can be checked on its own.  Real matrices are FP64 column-major.
 * ------------------------------------------------------------------------ */

/* Algorithm 1 step 1 (Theorem 2, eq. embedding):
 *   M = [Re(A+B) Im(A-B); -Im(A+B) Re(A-B)],  2n x 2n, ldm >= 2n.
 * Writes the lower triangle of M and zeros above the diagonal. */
int bse_build_M(bse_ctx* ctx, int n, const void* A, int lda, const void* B, int ldb, double* M,
                int ldm);

/* Algorithm 1 step 2: lower Cholesky factor M = L L^T in place (N x N,
 * ldm >= N; lower triangle read, L written to the lower triangle, the strict
 * upper triangle set to zero).  Returns +k if the leading k x k minor is not
 * positive definite (M is then left partially factored). */
int bse_potrf(bse_ctx* ctx, int N, double* M, int ldm);

/* Algorithm 1 step 3: W = L^T J_n L for N = 2n, from lower-triangular L
 * (strict upper triangle of L ignored).  Writes the full skew-symmetric W. */
int bse_form_W(bse_ctx* ctx, int N, const double* L, int ldl, double* W, int ldw);

/* Algorithm 3 step 1 (remark 1): W = U T U^T with U = H_0 ... H_{N-3},
 * H_k = I - tau_k v_k v_k^T.  In: skew W (lower triangle read).  Out:
 * alpha[k] = T[k,k+1] for k = 0..N-2 (T[k+1,k] = -alpha[k]), tau[k] for
 * k = 0..N-2 (tau[N-2] = 0), and v_k below the subdiagonal of W's column k
 * (v_k[k+1] = 1 implicit).  N >= 2. */
int bse_sktrd(bse_ctx* ctx, int N, double* W, int ldw, double* alpha, double* tau);

/* Algorithm 3 step 1 in two stages (Section 3.3, successive band
 * reduction): the same alpha (up to signs, which do not change the
 * eigenvalues) from the skew-symmetric W (lower triangle read, N x N,
 * ldw >= N, overwritten).  N >= 2, N <= 32768 + 64. */
int bse_sktrd2(bse_ctx* ctx, int N, double* W, int ldw, double* alpha);

/* Algorithm 3 step 2 (remark 2): the n = N/2 positive eigenvalues of
 * T_s = tridiag(alpha, 0, alpha) (ascending, by bisection) and, when V is
 * non-NULL, orthonormal eigenvectors V (N x n, ldv >= N) by inverse iteration
 * reorthogonalised inside clusters.  alpha: N-1 doubles.  N even, >= 2. */
int bse_tridiag_eig(bse_ctx* ctx, int N, const double* alpha, double* lambda, double* V, int ldv);

/* bse_tridiag_eig with flags: BSE_EIGVEC_TWISTED computes the eigenvectors
 * by twisted factorisations (the per-vector step of MRRR, which Section 3.3
 * names as the alternative to inverse iteration): for eigenvalue lambda,
 * the top-down and bottom-up LDL^T factorisations of T_s - lambda I, the
 * twist index r minimising |gamma_r|, and the vector with z_r = 1 from the
 * two bidiagonal factors.  Eigenvalues within 1000 eps |lambda| of a
 * neighbour use inverse iteration; clusters are orthogonalised as in
 * bse_tridiag_eig.  Other flag bits: -7. */
int bse_tridiag_eig_flags(bse_ctx* ctx, int N, const double* alpha, double* lambda, double* V, int ldv,
                          unsigned flags);

#ifdef __cplusplus
}
#endif

#endif /* BSE_H_ */
