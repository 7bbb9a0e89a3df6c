// Blocked Householder tridiagonalisation of a real skew-symmetric matrix,
// W = U T U^T (Algorithm 3 step 1; Section 3.3, remark 1).
//
// Reflector k, H_k = I - tau_k v_k v_k^T, acts on rows/columns k+1..N-1 and
// zeroes W[k+2:, k].  For a skew S and p = tau S v one has v^T S v = 0, so
//     H S H = S + v p^T - p v^T
// (no extra rank-one correction as in the symmetric case).  Within a panel of
// nb columns the reflectors are accumulated as in LAPACK's latrd: the
// trailing matrix is not touched, the current one is
//     S~ = S + V P^T - P V^T,
// column i is brought up to date just before its reflector is built, and
//     p_i = tau_i (S v_i + V (P^T v_i) - P (V^T v_i)).
// After the panel, S <- S + V P^T - P V^T is one MFMA product
//     [v_0 p_0 v_1 p_1 ...] [p_0 -v_0 p_1 -v_1 ...]^T  (strictly lower part).
//
// Per column two kernels run:
//   sk_symv   the HBM-bound product S v over the strictly-lower triangle of
//             the trailing matrix.  One 64 x 64 tile per workgroup, each
//             element read once and used twice (row sum for y, column sum for
//             -S^T v).  Partial sums go to a buffer indexed so that every
//             output block has exactly nblk+1 partial slots, summed in a fixed
//             order (deterministic).  Diagonal tiles also store v and the
//             partial dot products V^T v, P^T v.
//   sk_update reduces the partials into p, applies the panel corrections,
//             brings the next column up to date, and the last workgroup to
//             finish computes the next reflector (dlarfg convention).
#include "common.h"
#include "kernels.h"

namespace bse {

namespace {

constexpr int TS = 64;       // symv tile
constexpr int NBMAX = 64;    // panel width bound

struct Ctrl {
  double tau;
  double scale;
  double x0;
  double pad0;
  unsigned int cnt_diag;
  unsigned int cnt_upd;
  unsigned int pad1[2];
  double c[2 * NBMAX];   // c[2l] = v_l . v,  c[2l+1] = p_l . v
};

__device__ inline void larfg(double x0, double xnorm, double& beta, double& tau, double& scale) {
  if (xnorm == 0.0) {
    beta = x0;
    tau = 0.0;
    scale = 0.0;
    return;
  }
  beta = -copysign(hypot(x0, xnorm), x0);
  tau = (beta - x0) / beta;
  scale = 1.0 / (x0 - beta);
}

// Reflector of column j from the (already up to date) column itself.
__global__ __launch_bounds__(256) void sk_start(const double* __restrict__ W, long ld, int N, int j,
                                                Ctrl* __restrict__ ctrl, double* __restrict__ alpha,
                                                double* __restrict__ tau) {
  __shared__ double red[4];
  double ss = 0.0;
  for (long r = j + 2 + threadIdx.x; r < N; r += 256) {
    const double v = W[r + (long)j * ld];
    ss += v * v;
  }
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) {
    const double x0 = W[(long)(j + 1) + (long)j * ld];
    double beta, t, sc;
    larfg(x0, sqrt(ss), beta, t, sc);
    ctrl->tau = t;
    ctrl->scale = sc;
    alpha[j] = -beta;
    tau[j] = t;
  }
}

__global__ __launch_bounds__(256) void sk_symv(const double* __restrict__ W, long ld, int N, int j,
                                               int i, int nblk, int R0, Ctrl* __restrict__ ctrl,
                                               double* __restrict__ Y1, double* __restrict__ Y2,
                                               long ldy, double* __restrict__ Ypart,
                                               double* __restrict__ dotpart) {
  __shared__ double vr[TS], vc[TS];
  __shared__ double red[2][16][TS + 1];
  __shared__ int last_flag;
  int Rl, Cl;
  tri_index(blockIdx.x, Rl, Cl);
  const int R = R0 + Rl, C = R0 + Cl;
  const int s = j + 1;
  const int tid = threadIdx.x;
  const double scale = ctrl->scale;
  if (tid < 2 * TS) {
    const int which = tid >> 6;
    const long r = (long)(which ? C : R) * TS + (tid & 63);
    double v = 0.0;
    if (r == s) v = 1.0;
    else if (r > s && r < N) v = scale * W[r + (long)j * ld];
    if (which) vc[tid & 63] = v;
    else vr[tid & 63] = v;
  }
  __syncthreads();

  const int tx = tid & 15, ty = tid >> 4;
  const long rb = (long)R * TS + 4 * tx;
  const long cb = (long)C * TS + 4 * ty;
  double yr[4] = {0.0, 0.0, 0.0, 0.0}, yc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const long col = cb + c;
    const double* p = W + rb + col * ld;
    const double2 lo = *reinterpret_cast<const double2*>(p);
    const double2 hi = *reinterpret_cast<const double2*>(p + 2);
    const double a4[4] = {lo.x, lo.y, hi.x, hi.y};
    const double vcc = vc[4 * ty + c];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long row = rb + q;
      const bool valid = (row > col) && (col >= s) && (row < N);
      const double a = valid ? a4[q] : 0.0;
      yr[q] += a * vcc;
      yc[c] += a * vr[4 * tx + q];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) red[0][ty][4 * tx + q] = yr[q];
#pragma unroll
  for (int c = 0; c < 4; ++c) red[1][tx][4 * ty + c] = yc[c];
  __syncthreads();
  if (tid < TS) {
    double acc = 0.0;
    for (int k = 0; k < 16; ++k) acc += red[0][k][tid];
    Ypart[((long)Rl * (nblk + 1) + Cl) * TS + tid] = acc;
  } else if (tid < 2 * TS) {
    const int t = tid - TS;
    double acc = 0.0;
    for (int k = 0; k < 16; ++k) acc += red[1][k][t];
    Ypart[((long)Cl * (nblk + 1) + Rl + 1) * TS + t] = -acc;
  }

  if (Rl != Cl) return;  // uniform per workgroup
  // diagonal tile: store v_i and the partial dot products of the panel
  if (tid < TS) {
    const long r = (long)R * TS + tid;
    if (r >= s && r < N) {
      Y1[r + (long)(2 * i) * ldy] = vr[tid];
      Y2[r + (long)(2 * i + 1) * ldy] = -vr[tid];
    }
  }
  if (i == 0) return;
  if (tid < 2 * i) {
    const double* col = Y1 + (long)tid * ldy;
    double acc = 0.0;
    for (int q = 0; q < TS; ++q) {
      const long r = (long)R * TS + q;
      if (r >= s && r < N) acc += col[r] * vr[q];
    }
    dotpart[(long)Rl * (2 * NBMAX) + tid] = acc;
  }
  if (arrive_last(&ctrl->cnt_diag, (unsigned)nblk, &last_flag)) {
    if (tid < 2 * i) {
      double acc = 0.0;
      for (int b = 0; b < nblk; ++b) acc += dotpart[(long)b * (2 * NBMAX) + tid];
      ctrl->c[tid] = acc;
    }
  }
}

__global__ __launch_bounds__(256) void sk_update(double* __restrict__ W, long ld, int N, int j, int i,
                                                 int nbp, int nblk, int R0, Ctrl* __restrict__ ctrl,
                                                 double* __restrict__ Y1, double* __restrict__ Y2,
                                                 long ldy, const double* __restrict__ Ypart,
                                                 double* __restrict__ normpart,
                                                 double* __restrict__ alpha, double* __restrict__ tau_arr) {
  __shared__ double cs[2 * NBMAX];
  __shared__ double red[4][TS];
  __shared__ double pr[TS];
  __shared__ double red4[4];
  __shared__ double sval_s;
  __shared__ int last_flag;
  const int b = blockIdx.x;
  const int R = R0 + b;
  const int s = j + 1;
  const int tid = threadIdx.x;
  const double tau = ctrl->tau;
  if (tid < 2 * i) cs[tid] = ctrl->c[tid];
  const int t = tid & 63, part = tid >> 6;
  {
    double acc = 0.0;
    const double* base = Ypart + (long)b * (nblk + 1) * TS + t;
    for (int x = part; x <= nblk; x += 4) acc += base[(long)x * TS];
    red[part][t] = acc;
  }
  __syncthreads();
  const long r = (long)R * TS + t;
  if (part == 0) {
    double p = 0.0;
    if (r >= s && r < N) {
      const double y = red[0][t] + red[1][t] + red[2][t] + red[3][t];
      double corr = 0.0;
      for (int l = 0; l < i; ++l)
        corr += Y1[r + (long)(2 * l) * ldy] * cs[2 * l + 1] - Y1[r + (long)(2 * l + 1) * ldy] * cs[2 * l];
      p = tau * (y + corr);
      Y1[r + (long)(2 * i + 1) * ldy] = p;
      Y2[r + (long)(2 * i) * ldy] = p;
      if (r > s) W[r + (long)j * ld] = Y1[r + (long)(2 * i) * ldy];  // store v_i in place
    }
    pr[t] = p;
  }
  const bool next_col = (i + 1 < nbp) && (s <= N - 2);
  if (!next_col) return;  // uniform
  // p_i at row s, needed by every block for the update of column s
  {
    double ys = 0.0;
    for (int x = tid; x <= nblk; x += 256) ys += Ypart[(long)x * TS + (s - (long)R0 * TS)];
    ys = block_sum(ys, red4);
    if (tid == 0) {
      double corr = 0.0;
      for (int l = 0; l < i; ++l)
        corr += Y1[s + (long)(2 * l) * ldy] * cs[2 * l + 1] - Y1[s + (long)(2 * l + 1) * ldy] * cs[2 * l];
      sval_s = tau * (ys + corr);
    }
  }
  __syncthreads();
  double nrm = 0.0;
  if (part == 0 && r >= s + 1 && r < N) {
    const double sval = sval_s;
    double upd = W[r + (long)s * ld];
    for (int l = 0; l < i; ++l) {
      const double vrl = Y1[r + (long)(2 * l) * ldy], prl = Y1[r + (long)(2 * l + 1) * ldy];
      const double vsl = Y1[s + (long)(2 * l) * ldy], psl = Y1[s + (long)(2 * l + 1) * ldy];
      upd += vrl * psl - prl * vsl;
    }
    upd += Y1[r + (long)(2 * i) * ldy] * sval - pr[t];
    W[r + (long)s * ld] = upd;
    if (r == s + 1) ctrl->x0 = upd;
    if (r >= s + 2) nrm = upd * upd;
  }
  nrm = block_sum(nrm, red4);
  if (tid == 0) normpart[b] = nrm;
  if (arrive_last(&ctrl->cnt_upd, (unsigned)nblk, &last_flag)) {
    if (tid == 0) {
      double ss = 0.0;
      for (int k = 0; k < nblk; ++k) ss += normpart[k];
      double beta, tn, sc;
      larfg(ctrl->x0, sqrt(ss), beta, tn, sc);
      ctrl->tau = tn;
      ctrl->scale = sc;
      alpha[s] = -beta;
      tau_arr[s] = tn;
    }
  }
}

__global__ void k_zero_ctrl(Ctrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->cnt_diag = 0u;
    ctrl->cnt_upd = 0u;
  }
}

}  // namespace

size_t sktrd_work_bytes(long N, long ld, int nb) {
  (void)N;
  const long nt = ld / TS;
  size_t bytes = 0;
  bytes += 2 * (size_t)ld * 2 * NBMAX * sizeof(double);            // Y1, Y2
  bytes += (size_t)nt * (nt + 1) * TS * sizeof(double);           // Ypart
  bytes += (size_t)nt * 2 * NBMAX * sizeof(double);               // dotpart
  bytes += (size_t)nt * sizeof(double);                           // normpart
  bytes += 4096;                                                  // ctrl
  (void)nb;
  return bytes + 8 * 256;
}

int sktrd_bind_work(void* base, long N, long ld, int nb, SktrdWork* w) {
  (void)N;
  if (nb < 1 || nb > NBMAX) nb = NBMAX;
  const long nt = ld / TS;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += round_up((long)bytes, 256);
    return q;
  };
  w->Y1 = reinterpret_cast<double*>(take((size_t)ld * 2 * NBMAX * sizeof(double)));
  w->Y2 = reinterpret_cast<double*>(take((size_t)ld * 2 * NBMAX * sizeof(double)));
  w->Ypart = reinterpret_cast<double*>(take((size_t)nt * (nt + 1) * TS * sizeof(double)));
  w->dotpart = reinterpret_cast<double*>(take((size_t)nt * 2 * NBMAX * sizeof(double)));
  w->normpart = reinterpret_cast<double*>(take((size_t)nt * sizeof(double)));
  w->ctrl = take(sizeof(Ctrl));
  w->nb = nb;
  return 0;
}

int sktrd_f64(hipStream_t s, int N, double* W, long ld, double* alpha, double* tau, const SktrdWork& w) {
  if (N < 2) return 0;
  Ctrl* ctrl = static_cast<Ctrl*>(w.ctrl);
  const long ldy = ld;
  k_zero_ctrl<<<1, 64, 0, s>>>(ctrl);
  BSE_LAUNCHED();
  const int nb = w.nb;
  for (int k0 = 0; k0 <= N - 2; k0 += nb) {
    const int nbp = (N - 1 - k0 < nb) ? (N - 1 - k0) : nb;
    sk_start<<<1, 256, 0, s>>>(W, ld, N, k0, ctrl, alpha, tau);
    BSE_LAUNCHED();
    for (int i = 0; i < nbp; ++i) {
      const int j = k0 + i;
      if (j >= N - 2) break;  // the last column has no reflector to apply
      const int sidx = j + 1;
      const int R0 = sidx / TS;
      const int nblk = (N - 1) / TS - R0 + 1;
      const unsigned ntiles = (unsigned)((long)nblk * (nblk + 1) / 2);
      sk_symv<<<ntiles, 256, 0, s>>>(W, ld, N, j, i, nblk, R0, ctrl, w.Y1, w.Y2, ldy, w.Ypart, w.dotpart);
      BSE_LAUNCHED();
      sk_update<<<(unsigned)nblk, 256, 0, s>>>(W, ld, N, j, i, nbp, nblk, R0, ctrl, w.Y1, w.Y2, ldy,
                                               w.Ypart, w.normpart, alpha, tau);
      BSE_LAUNCHED();
    }
    const int e = k0 + nbp;
    const int m2 = N - e;
    if (m2 >= 2 && e <= N - 2) {
      BSE_TRY(gemm_f64(s, false, true, m2, m2, 2 * nbp, 1.0, w.Y1 + e, ldy, w.Y2 + e, ldy, 1.0,
                       W + e + (long)e * ld, ld, 2, 0, 0));
    }
  }
  return 0;
}

}  // namespace bse
