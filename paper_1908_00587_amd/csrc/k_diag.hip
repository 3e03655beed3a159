// Heated-flow diagnostics (section 3: the Nusselt number at the inner
// cylinder -- its heat transfer over that of the basic state at the same
// temperature difference -- and velocity probe time series at fixed points).
//
//   k_diag   one wavefront: the theta-z mean profiles (mode (0,0)) at the
//            two walls through the one-sided nine-point stencils: Nusselt
//            numbers r ln(eta) d<T>/dr and torques -2 pi L_z r^3 d(<u_theta>/r)/dr
//   k_probe  one workgroup per (probe, field): the Fourier sum of the row's
//            modes at (theta, z), reduced across the workgroup
#include <hip/hip_runtime.h>

#include <cmath>

#include "nsc_internal.h"

namespace nsc {
namespace {

constexpr int kProbeThreads = 256;

struct Probes {
  int n;
  int row[kMaxProbes];
  double theta[kMaxProbes], z[kMaxProbes];
};

__global__ void __launch_bounds__(64) k_diag(Dims d, Grid g, const double2 *__restrict__ u,
                                             double log_eta, double *__restrict__ out) {
  const int t = threadIdx.x;
  if (t >= 4) return;
  const int n = d.nr;
  const size_t P = d.nmodes;
  const int wall = t & 1;                      // 0: r_i, 1: r_o
  const int j = wall ? n - 1 : 0;
  const int s0 = wall ? n - kStencil : 0;      // one-sided wall window
  const int f = t < 2 ? 3 : 1;                 // lanes 0, 1: temperature; 2, 3: u_theta
  if (f == 3 && !d.heated) {
    out[t] = 0.0;
    return;
  }
  const double2 *col = u + (size_t)f * n * P + d.kmax;  // mode (0,0)
  double dv = 0.0;
#pragma unroll
  for (int q = 0; q < kStencil; ++q) dv = fma(g.d1[j * kStencil + q], col[(size_t)(s0 + q) * P].x, dv);
  const double r = g.r[j];
  if (f == 3) {
    out[t] = dv * r * log_eta;
  } else {
    const double v = col[(size_t)j * P].x;
    out[t] = -2.0 * M_PI * d.lz * r * r * r * (dv / r - v / (r * r));
  }
}

__global__ void __launch_bounds__(kProbeThreads) k_probe(Dims d, const double2 *__restrict__ u,
                                                         Probes pr, double *__restrict__ out) {
  __shared__ double red[kProbeThreads / 64];
  const int p = blockIdx.x, f = blockIdx.y;
  const int j = pr.row[p];
  const double th = pr.theta[p], zz = pr.z[p];
  const size_t P = d.nmodes;
  const double2 *row = u + ((size_t)f * d.nr + j) * P;
  double acc = 0.0;
  for (int md = threadIdx.x; md < d.nmodes; md += kProbeThreads) {
    const int m = md / d.mz;
    const int k = md - m * d.mz - d.kmax;
    double s, c;
    sincos((double)m * th + (double)k * d.kz * zz, &s, &c);
    const double2 v = row[md];
    acc += (m == 0 ? 1.0 : 2.0) * (v.x * c - v.y * s);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kProbeThreads / 64; ++w) r += red[w];
    out[(size_t)p * d.f + f] = r;
  }
}

}  // namespace
}  // namespace nsc

int nsc_diagnostics(nsc_ctx *c, const double *u_hat, double *out) {
  if (!c || !u_hat || !out) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  hipLaunchKernelGGL(nsc::k_diag, dim3(1), dim3(64), 0, c->stream, c->d, c->g,
                     reinterpret_cast<const double2 *>(u_hat), std::log(c->eta), out);
  return hipGetLastError() == hipSuccess ? NSC_OK : NSC_ERR_DEVICE;
}

int nsc_probe(nsc_ctx *c, const double *u_hat, int n, const int *rows, const double *theta,
              const double *z, double *out) {
  if (!c || !u_hat || !out || !rows || !theta || !z || n < 1 || n > nsc::kMaxProbes)
    return NSC_ERR_ARG;
  nsc::Probes pr{};
  pr.n = n;
  for (int i = 0; i < n; ++i) {
    if (rows[i] < 0 || rows[i] >= c->d.nr || !std::isfinite(theta[i]) || !std::isfinite(z[i]))
      return NSC_ERR_ARG;
    pr.row[i] = rows[i];
    pr.theta[i] = theta[i];
    pr.z[i] = z[i];
  }
  hipLaunchKernelGGL(nsc::k_probe, dim3(n, c->d.f), dim3(nsc::kProbeThreads), 0, c->stream, c->d,
                     reinterpret_cast<const double2 *>(u_hat), pr, out);
  return hipGetLastError() == hipSuccess ? NSC_OK : NSC_ERR_DEVICE;
}
