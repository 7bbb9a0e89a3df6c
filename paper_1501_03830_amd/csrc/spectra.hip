// Broadened spectra from the eigenpairs: the density of states of eq. DOS
//     phi(omega) = 1/(2n) sum_{j=1}^{2n} delta(omega - lambda_j)
// over all 2n eigenvalues of H (the +lambda_j and their -lambda_j partners
// of Theorem 3), and the absorption spectrum of eq. absp
//     eps+(omega) = sum_{j=1}^{n} w_j delta(omega - lambda_j)
// with the weights w_j of the positive eigenvalues, each delta replaced by
// the Gaussian of standard deviation sigma that Section 4 uses for its
// spectral-density figure,
//     delta(t) ~ exp(-t^2 / (2 sigma^2)) / (sqrt(2 pi) sigma).
//
// One thread per grid point omega_k = omega0 + k domega; the eigenvalues and
// weights are staged through LDS in chunks shared by the workgroup.  The
// work is n exponentials per point (ALU-bound; tiny next to the solve).
#include "driver.h"

namespace bse {

namespace {

constexpr int SP_TB = 256;

__global__ __launch_bounds__(SP_TB) void k_spectra(int n, const double* __restrict__ lam,
                                                   const double* __restrict__ w, int npts, double omega0,
                                                   double domega, double sigma, double* __restrict__ dos,
                                                   double* __restrict__ eps) {
  __shared__ double sl[SP_TB];
  __shared__ double swr[SP_TB];
  __shared__ double swi[SP_TB];
  const int k = blockIdx.x * SP_TB + threadIdx.x;
  const double om = omega0 + (double)k * domega;
  const double inv2s2 = 0.5 / (sigma * sigma);
  const double norm = 1.0 / (sqrt(2.0 * M_PI) * sigma);
  double d = 0.0, er = 0.0, ei = 0.0;
  for (int j0 = 0; j0 < n; j0 += SP_TB) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    sl[threadIdx.x] = (j < n) ? lam[j] : 0.0;
    if (w) {
      swr[threadIdx.x] = (j < n) ? w[2 * j] : 0.0;
      swi[threadIdx.x] = (j < n) ? w[2 * j + 1] : 0.0;
    }
    __syncthreads();
    const int m = min(SP_TB, n - j0);
    for (int q = 0; q < m; ++q) {
      const double l = sl[q];
      const double tp = om - l, tm = om + l;
      const double gp = exp(-tp * tp * inv2s2);
      d += gp + exp(-tm * tm * inv2s2);
      if (w) {
        er += swr[q] * gp;
        ei += swi[q] * gp;
      }
    }
  }
  if (k >= npts) return;
  if (dos) dos[k] = d * norm / (2.0 * (double)n);
  if (eps) {
    eps[2 * k] = er * norm;
    eps[2 * k + 1] = ei * norm;
  }
}

}  // namespace

}  // namespace bse

using namespace bse;

extern "C" int bse_spectra(bse_ctx* ctx, int n, const double* lambda, const void* w, int npts, double omega0,
                           double domega, double sigma, double* dos, void* eps) {
  if (!ctx) return set_error(-1, "ctx is NULL");
  if (n <= 0) return set_error(-2, "n must be positive");
  if (!lambda) return set_error(-3, "lambda is NULL");
  if (npts <= 0) return set_error(-5, "npts must be positive");
  if (!(domega >= 0.0) || !std::isfinite(omega0) || !std::isfinite(domega)) return set_error(-7, "invalid grid");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return set_error(-8, "sigma must be positive");
  if (!dos && !eps) return set_error(-9, "neither dos nor eps requested");
  if (eps && !w) return set_error(-4, "eps needs the weights w");
  BSE_HIP(hipSetDevice(ctx->device));
  const unsigned blocks = (unsigned)((npts + SP_TB - 1) / SP_TB);
  BSE_LAUNCH(k_spectra, dim3(blocks), dim3(SP_TB), 0, ctx->lane.stream, n, lambda,
             eps ? static_cast<const double*>(w) : nullptr, npts, omega0, domega, sigma, dos,
             static_cast<double*>(eps));
  BSE_HIP(hipStreamSynchronize(ctx->lane.stream));
  return 0;
}
