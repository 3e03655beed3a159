// Host runtime of libnsc.so: argument validation, radial discretisation
// tables, transform plans, device memory, and the orchestration of the
// nonlinear term, the per-mode radial solves and the predictor--corrector
// step (sections 2.1 and 2.2 of the nsCouette paper).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "nsc_internal.h"

using namespace nsc;

namespace {

// ---------------------------------------------------------------------------
// Argument checks (pure host code, no HIP call)
// ---------------------------------------------------------------------------
bool plan_fft(int n, FftPlan *p) {
  if (n < 2 || n > kMaxFFT) return false;
  // power-of-two radices first, so that the accumulated length of every
  // stage up to the radix-3 one is a power of two (mask instead of modulo)
  int rem = n;
  int nst = 0;
  int r[kMaxStages];
  int n3 = 0, n5 = 0, a = 0;
  while (rem % 5 == 0) { rem /= 5; ++n5; }
  while (rem % 3 == 0) { rem /= 3; ++n3; }
  while (rem % 2 == 0) { rem /= 2; ++a; }
  if (rem != 1) return false;
  while (a >= 3 && a != 4) { if (nst >= kMaxStages) return false; r[nst++] = 8; a -= 3; }
  while (a >= 2) { if (nst >= kMaxStages) return false; r[nst++] = 4; a -= 2; }
  if (a == 1) { if (nst >= kMaxStages) return false; r[nst++] = 2; }
  for (int i = 0; i < n3; ++i) { if (nst >= kMaxStages) return false; r[nst++] = 3; }
  for (int i = 0; i < n5; ++i) { if (nst >= kMaxStages) return false; r[nst++] = 5; }
  p->n = n;
  p->nst = nst;
  p->min_radix = 8;
  for (int i = 0; i < nst; ++i) {
    p->radix[i] = r[i];
    if (r[i] < p->min_radix) p->min_radix = r[i];
  }
  // lines that one wavefront can carry through every stage with all of a
  // lane's butterflies (at most kWaveRegs complex values) in registers
  p->wave_lines = 0;
  for (int l = 1; l <= 8; ++l) {
    bool ok = true;
    for (int i = 0; i < nst; ++i) {
      const int per_lane = (l * (n / r[i]) + 63) / 64;
      if (per_lane > kWaveRegs / r[i]) ok = false;
    }
    if (!ok) break;
    p->wave_lines = l;
  }
  return true;
}

int validate(double eta, double Re_i, double Re_o, double Ra, double Pr, int N_r, int M_theta,
             int M_z, double L_z) {
  if (!(eta > 0.0 && eta < 1.0)) return NSC_ERR_ARG;
  if (!std::isfinite(Re_i) || !std::isfinite(Re_o) || !std::isfinite(Ra)) return NSC_ERR_ARG;
  if (Ra < 0.0) return NSC_ERR_ARG;
  if (Ra != 0.0 && !(Pr > 0.0 && std::isfinite(Pr))) return NSC_ERR_ARG;
  if (N_r < kStencil || N_r > 4096) return NSC_ERR_ARG;
  if (M_theta < 1 || M_z < 1 || (M_z % 2) == 0) return NSC_ERR_ARG;
  if (!(L_z > 0.0 && std::isfinite(L_z))) return NSC_ERR_ARG;
  FftPlan pt, pz;
  if (!plan_fft(3 * M_theta, &pt)) return NSC_ERR_ARG;
  if (!plan_fft(3 * ((M_z - 1) / 2 + 1), &pz)) return NSC_ERR_ARG;
  return NSC_OK;
}

// ---------------------------------------------------------------------------
// Radial discretisation (host, FP64)
// ---------------------------------------------------------------------------
// Weights of derivative orders 0..2 at z from the nodes x[0..n-1] by the
// recursive construction of B. Fornberg (Math. Comp. 51, 1988): each new
// node updates the interpolant's derivative weights of all earlier nodes.
void fd_weights(double z, const double *x, int n, double *c /* [n][3] */) {
  for (int i = 0; i < 3 * n; ++i) c[i] = 0.0;
  double c1 = 1.0, c4 = x[0] - z;
  c[0] = 1.0;
  for (int i = 1; i < n; ++i) {
    const int mn = i < 2 ? i : 2;
    double c2 = 1.0;
    const double c5 = c4;
    c4 = x[i] - z;
    for (int j = 0; j < i; ++j) {
      const double c3 = x[i] - x[j];
      c2 *= c3;
      if (j == i - 1) {
        for (int k = mn; k >= 1; --k)
          c[i * 3 + k] = c1 * (k * c[(i - 1) * 3 + k - 1] - c5 * c[(i - 1) * 3 + k]) / c2;
        c[i * 3] = -c1 * c5 * c[(i - 1) * 3] / c2;
      }
      for (int k = mn; k >= 1; --k) c[j * 3 + k] = (c4 * c[j * 3 + k] - k * c[j * 3 + k - 1]) / c3;
      c[j * 3] = c4 * c[j * 3] / c3;
    }
    c1 = c2;
  }
}

// Clenshaw--Curtis weights on x_j = cos(j pi / N), j = 0..N (closed form of
// the interpolatory rule), symmetric so the order of the nodes is irrelevant.
void cc_weights_host(int npts, double *w) {
  const int N = npts - 1;
  for (int j = 0; j <= N; ++j) {
    const double cj = (j == 0 || j == N) ? 1.0 : 2.0;
    long double s = 1.0L;
    for (int k = 1; k <= N / 2; ++k) {
      const long double bk = (2 * k == N) ? 1.0L : 2.0L;
      s -= bk / (4.0L * k * k - 1.0L) * cosl(2.0L * k * j * 3.14159265358979323846264338327950288L / N);
    }
    w[j] = (double)(cj / N * s);
  }
}

// e^{-2 pi i t/n}, t = 0..n-1: FP64 pairs (re, im), and for the FP32
// transforms compensated entries (hi.re, hi.im, lo.re, lo.im), hi the FP32
// rounding of the value and lo the FP32 rounding of what hi leaves out.
void twiddles(int n, double *t64, float *t32) {
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int t = 0; t < n; ++t) {
    const long double a = 2.0L * pi * (long double)t / (long double)n;
    const long double c = cosl(a), s = -sinl(a);
    t64[2 * t] = (double)c;
    t64[2 * t + 1] = (double)s;
    const float hc = (float)c, hs = (float)s;
    t32[4 * t] = hc;
    t32[4 * t + 1] = hs;
    t32[4 * t + 2] = (float)(c - (long double)hc);
    t32[4 * t + 3] = (float)(s - (long double)hs);
  }
}

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) return NSC_ERR_DEVICE;   \
  } while (0)

int dmalloc(void **p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return NSC_ERR_OOM;
  if (e != hipSuccess) return NSC_ERR_DEVICE;
  return NSC_OK;
}

#define TRY(x)                 \
  do {                         \
    int s_ = (x);              \
    if (s_ != NSC_OK) return s_; \
  } while (0)

bool mul_ok(size_t a, size_t b, size_t *out) {
  if (a != 0 && b > SIZE_MAX / a) return false;
  *out = a * b;
  return true;
}

int alloc_factors(Factors *f, int nq, int kp1, int nr, bool packed) {
  f->nq = nq;
  f->nops = nq * kp1;
  TRY(dmalloc((void **)&f->vals, (size_t)nr * kSlots * f->nops * sizeof(double)));
  TRY(dmalloc((void **)&f->edge, (size_t)kEdge * f->nops * sizeof(double)));
  if (packed) TRY(dmalloc((void **)&f->pk, (size_t)nr * 8 * f->nops * sizeof(double)));
  return NSC_OK;
}

// The packed columns of a family with packed rows (the adjoint's transposed
// sweeps), zero where a column entry falls outside the matrix.
int alloc_columns(Factors *f, int nr) {
  if (!f->pk) return NSC_OK;
  const size_t bytes = (size_t)nr * 8 * f->nops * sizeof(double);
  TRY(dmalloc((void **)&f->pc, bytes));
  HIPCHK(hipMemset(f->pc, 0, bytes));
  return NSC_OK;
}

void free_factors(Factors *f) {
  if (f->vals) (void)hipFree(f->vals);
  if (f->edge) (void)hipFree(f->edge);
  if (f->pk) (void)hipFree(f->pk);
  if (f->pc) (void)hipFree(f->pc);
  f->vals = f->edge = f->pk = f->pc = nullptr;
}

int ensure_factors(nsc_ctx *c, double dt, double cc) {
  if (dt == c->fac_dt && cc == c->fac_c) return NSC_OK;
  StageTimer t(c, 10);
  if (c->d.heated)
    HIPCHK(launch_factor2(c, &c->fv, &c->ft, OP_HELMHOLTZ, 1.0 / dt, cc, cc / c->d.pr));
  else
    HIPCHK(launch_factor(c, &c->fv, OP_HELMHOLTZ, 1.0 / dt, cc));
  HIPCHK(launch_influence_setup(c));
  c->fac_dt = dt;
  c->fac_c = cc;
  return NSC_OK;
}

int nonlinear_impl(nsc_ctx *c, const double *u, double *nh, double *cfl_out,
                   double *cfl_host = nullptr) {
  if (!theta_fits(c, c->precision, 0)) return NSC_ERR_STATE;
  {
    StageTimer t(c, 0);
    HIPCHK(launch_zinv(c, c->precision, u));
  }
  {
    StageTimer t(c, 1);
    HIPCHK(launch_theta(c, c->precision, cfl_out != nullptr));
  }
  {
    StageTimer t(c, 2);
    HIPCHK(launch_zfwd(c, c->precision, u, nh, cfl_out, cfl_out ? cfl_host : nullptr));
  }
  return NSC_OK;
}

int solve_impl(nsc_ctx *c, const double *un, const double *nn, const double *nq, double *out,
               double *pout, double dt, double cc, int walls) {
  TRY(ensure_factors(c, dt, cc));
  {
    StageTimer t(c, 4);
    HIPCHK(launch_rhs(c, un, nn, nq, dt, cc));
  }
  const int want_p = pout != nullptr;
  {
    StageTimer t(c, 5);
    HIPCHK(launch_solve_sweeps(c, 0, nn, nq, cc, walls, want_p));
  }
  {
    StageTimer t(c, 6);
    HIPCHK(launch_solve_sweeps(c, 1, nn, nq, cc, walls, want_p));
  }
  {
    StageTimer t(c, 11);
    HIPCHK(launch_solve_sweeps(c, 2, nn, nq, cc, walls, want_p));
  }
  {
    StageTimer t(c, 7);
    HIPCHK(launch_solve_sweeps(c, 3, nn, nq, cc, walls, want_p));
  }
  {
    StageTimer t(c, 8);
    HIPCHK(launch_influence(c));
  }
  {
    StageTimer t(c, 9);
    HIPCHK(launch_finalize(c, out, pout));
  }
  return NSC_OK;
}

// Non-finite check of a fixed-size step: its first nonlinear stage writes the
// CFL bound of the step's input state (NaN if a value was not finite) to the
// host-mapped scalar and records ev_cfl.  At the end of the call the host
// reads it if the stage has finished, without waiting; otherwise the check
// stays pending and the next step call waits for it (by then long done).
int query_nonfinite(nsc_ctx *c) {
  const hipError_t q = hipEventQuery(c->ev_cfl);
  if (q == hipErrorNotReady) {
    (void)hipGetLastError();  // not an error: leave nothing for the next launch check
    c->nan_pending = 1;
    return NSC_OK;
  }
  if (q != hipSuccess) return NSC_ERR_DEVICE;
  c->nan_pending = 0;
  return std::isnan(c->h_pinned[0]) ? NSC_ERR_NONFINITE : NSC_OK;
}

int pending_nonfinite(nsc_ctx *c) {
  if (!c->nan_pending) return NSC_OK;
  c->nan_pending = 0;
  HIPCHK(hipEventSynchronize(c->ev_cfl));
  return std::isnan(c->h_pinned[0]) ? NSC_ERR_NONFINITE : NSC_OK;
}

}  // namespace

// Argument checks of the step VJP (pure host code, before any device work).
int nsc::step_vjp_check(const nsc_ctx *c, const double *u, const double *stages,
                        const double *ubar_next, const double *ubar) {
  if (!c || !u || !stages || !ubar_next || !ubar) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  if ((const void *)ubar == (const void *)u || (const void *)ubar == (const void *)ubar_next)
    return NSC_ERR_ARG;
  const size_t fld = (size_t)c->d.f * c->d.nr * c->d.nmodes * 2;
  const int nc = c->n_corr;
  if (ubar < stages + (size_t)nc * fld && stages < ubar + fld) return NSC_ERR_ARG;
  if (!theta_fits(c, c->precision, 1)) return NSC_ERR_STATE;
  return NSC_OK;
}

// The step VJP's sequence with its four state-sized adjoint workspaces at
// work (caller-provided: the context's own, or the allocation-free entry
// point's static device array).
int nsc::step_vjp_impl(nsc_ctx *c, const double *u, const double *stages,
                       const double *ubar_next, double *ubar, double *work) {
  const size_t fld = (size_t)c->d.f * c->d.nr * c->d.nmodes * 2;
  const int nc = c->n_corr;
  double *abar = work, *bbar = abar + fld, *xa = bbar + fld, *xb = xa + fld;
  TRY(ensure_factors(c, c->dt, c->c));
  // the first solve VJP writes ubar and abar, every one writes bbar; only
  // the nonlinear VJP's output starts from zero
  const double *xbar = ubar_next;
  for (int q = nc; q >= 1; --q) {
    // X^(q+1) = S(u, a, N(X^(q)))
    HIPCHK(launch_solve_vjp(c, xbar, ubar, abar, bbar, c->dt, c->c, q == nc ? 7 : 4));
    double *xn = (xbar == xa) ? xb : xa;
    HIPCHK(launch_fill_zero(c, xn, fld));
    HIPCHK(launch_nonlinear_vjp(c, c->precision, stages + (size_t)(q - 1) * fld, bbar, xn));
    xbar = xn;
  }
  // X^(1) = S(u, a, a)
  HIPCHK(launch_solve_vjp(c, xbar, ubar, abar, bbar, c->dt, c->c, nc >= 1 ? 4 : 7));
  HIPCHK(launch_add(c, abar, bbar, fld));
  HIPCHK(launch_nonlinear_vjp(c, c->precision, u, abar, ubar));
  return NSC_OK;
}

// ---------------------------------------------------------------------------
// Public ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *nsc_strerror(int status) {
  switch (status) {
    case NSC_OK: return "ok";
    case NSC_ERR_ARG: return "invalid argument";
    case NSC_ERR_DEVICE: return "HIP device or runtime error";
    case NSC_ERR_OOM: return "device allocation failed or size overflow";
    case NSC_ERR_NONFINITE: return "non-finite value detected";
    case NSC_ERR_DT: return "time step collapsed below 1e-12";
    case NSC_ERR_STATE: return "call not valid in the current context state";
    case NSC_ERR_IO: return "state file missing, unreadable, truncated or not a state file";
    default: return "unknown status";
  }
}

int nsc_destroy(nsc_ctx *c) {
  if (!c) return NSC_OK;
  void *ptrs[] = {c->tables, c->tw64_t, c->tw64_z, c->tw32_t, c->tw32_z, c->zbuf, c->wbuf,
                  c->cfl_part, c->cfl_val, c->e_part, c->s_f, c->s_g, c->s_p, c->s_x,
                  c->s_lam, c->s_vjp, c->s_u1, c->s_nn, c->s_nq, c->s_adj, c->s_mean, c->inf.resp, c->inf.ainv,
                  c->t_row, c->t_cnt, c->t_wt};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  free_factors(&c->fv);
  free_factors(&c->ft);
  free_factors(&c->fp);
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  if (c->ev_cfl) (void)hipEventDestroy(c->ev_cfl);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete[] c->h_r;
  delete c;
  return NSC_OK;
}

// pipe = 1: the pipe-flow variant (eta, Re_o, Ra, Pr unused; Re_i is the
// centreline speed Re of the laminar flow).
static int init_impl(nsc_ctx *c, double eta, double Re_i, double Re_o, double Ra, double Pr,
                     int N_r, int M_theta, int M_z, double L_z, int pipe = 0) {
  Dims &d = c->d;
  d.nr = N_r;
  d.mt = M_theta;
  d.mz = M_z;
  d.kmax = (M_z - 1) / 2;
  d.nt = 3 * M_theta;
  d.nz = 3 * (d.kmax + 1);
  d.nmodes = M_theta * M_z;
  d.heated = Ra != 0.0 ? 1 : 0;
  d.f = d.heated ? 4 : 3;
  d.kz = 2.0 * M_PI / L_z;
  d.pr = d.heated ? Pr : 1.0;
  d.gr = d.heated ? Ra / Pr : 0.0;
  d.re_i = Re_i;
  d.re_o = Re_o;
  d.r_i = eta / (1.0 - eta);
  d.r_o = 1.0 / (1.0 - eta);
  d.lz = L_z;
  d.a_cou = (Re_o * d.r_o - Re_i * d.r_i) / (d.r_o * d.r_o - d.r_i * d.r_i);
  d.b_cou = d.r_i * (Re_i - d.a_cou * d.r_i);
  d.pipe = pipe;
  d.gp = 0.0;
  if (pipe) {
    // radius 1, no wall motion, driven by -dP/dz = 4 Re (laminar: Re (1 - r^2))
    d.re_i = d.re_o = 0.0;
    d.r_i = 0.0;
    d.r_o = 1.0;
    d.a_cou = d.b_cou = 0.0;
    d.gp = 4.0 * Re_i;
  }
  c->eta = eta;
  c->ra = Ra;
  c->n_in = d.heated ? 9 : 6;
  c->n_out = d.heated ? 4 : 3;
  plan_fft(d.nt, &c->plan_t);
  plan_fft(d.nz, &c->plan_z);

  // size guards
  size_t field, tmp;
  if (!mul_ok((size_t)d.nr, (size_t)d.nmodes, &field) || !mul_ok(field, 16, &field))
    return NSC_ERR_OOM;
  size_t inter;
  if (!mul_ok((size_t)d.nr * d.nz, (size_t)d.mt, &inter) || !mul_ok(inter, 16, &inter))
    return NSC_ERR_OOM;
  (void)tmp;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return NSC_ERR_DEVICE;
  HIPCHK(hipGetDevice(&c->device));
  noalloc_setup(c->device);  // the allocation-free entry point's scratch address
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) ==
            hipSuccess &&
        lds >= 32 * 1024)
      c->lds_max = lds - 1024;  // headroom for the kernels' static LDS
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
        v > 0)
      c->cu_count = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device) ==
            hipSuccess &&
        v >= lds)
      c->lds_cu = v;
  }

  // host tables
  const int n = d.nr;
  c->h_r = new (std::nothrow) double[n];
  if (!c->h_r) return NSC_ERR_OOM;
  // np parity sets of derivative rows: one for the cylinders, two (even,
  // odd) for the pipe
  const int np = pipe ? 2 : 1;
  const int nw = n * kStencil;
  std::vector<double> rinv(n), d1(np * nw), d2(np * nw), dr(n), ccw(n, 0.0);
  std::vector<int> s(n);
  for (int j = 0; j < n; ++j) {
    if (pipe) {  // positive half of the 2 N_r Gauss--Lobatto points of [-1, 1]
      c->h_r[j] = std::cos(M_PI * (double)(n - 1 - j) / (double)(2 * n - 1));
    } else {
      const double x = std::cos(M_PI * (double)(n - 1 - j) / (double)(n - 1));
      c->h_r[j] = 0.5 * (d.r_i + d.r_o) + 0.5 * x;
    }
  }
  for (int j = 0; j < n; ++j) {
    rinv[j] = 1.0 / c->h_r[j];
    int sj = j - kHalf;
    if (sj < 0) sj = 0;
    if (sj > n - kStencil) sj = n - kStencil;
    s[j] = sj;
    double w[kStencil * 3];
    if (!pipe) {
      fd_weights(c->h_r[j], c->h_r + sj, kStencil, w);
      for (int t = 0; t < kStencil; ++t) {
        d1[j * kStencil + t] = w[t * 3 + 1];
        d2[j * kStencil + t] = w[t * 3 + 2];
      }
    } else {
      // the nine points nearest to r_j on the grid extended by the mirror
      // points -r_k (position N_r + j of 2 N_r, ascending); a mirror point's
      // weight goes to column k times the parity (+1 even, -1 odd)
      double x[kStencil];
      const int e0 = n + j;
      int se = e0 - kHalf;
      if (se > 2 * n - kStencil) se = 2 * n - kStencil;
      for (int t = 0; t < kStencil; ++t) {
        const int e = se + t;
        x[t] = e >= n ? c->h_r[e - n] : -c->h_r[n - 1 - e];
      }
      fd_weights(c->h_r[j], x, kStencil, w);
      for (int par = 0; par < 2; ++par) {
        const double sg = par ? -1.0 : 1.0;
        for (int t = 0; t < kStencil; ++t) {
          const int e = se + t;
          const int col = e >= n ? e - n : n - 1 - e;
          const double f = e >= n ? 1.0 : sg;
          d1[par * nw + j * kStencil + col - sj] += f * w[t * 3 + 1];
          d2[par * nw + j * kStencil + col - sj] += f * w[t * 3 + 2];
        }
      }
    }
    double lo = j > 0 ? c->h_r[j] - c->h_r[j - 1] : c->h_r[1] - c->h_r[0];
    if (pipe && j == 0) lo = 2.0 * c->h_r[0];  // the mirror point -r_0
    const double hi = j < n - 1 ? c->h_r[j + 1] - c->h_r[j] : c->h_r[n - 1] - c->h_r[n - 2];
    dr[j] = lo < hi ? lo : hi;
  }
  if (!pipe) {
    cc_weights_host(n, ccw.data());
    for (int j = 0; j < n; ++j) ccw[j] *= 0.5;
  }
  std::vector<double> lw(np * nw);
  for (int par = 0; par < np; ++par)
    for (int j = 0; j < n; ++j)
      for (int t = 0; t < kStencil; ++t) {
        const int i = par * nw + j * kStencil + t;
        lw[i] = std::fma(d1[i], rinv[j], d2[i]);
      }
  // device tables: one allocation
  const size_t nd = (size_t)n * (1 + 1 + 1 + 1) + (size_t)np * nw * 3;
  TRY(dmalloc(&c->tables, nd * sizeof(double) + (size_t)n * sizeof(int) + 256));
  double *base = (double *)c->tables;
  double *p_r = base, *p_rinv = p_r + n, *p_d1 = p_rinv + n, *p_d2 = p_d1 + np * nw,
         *p_dr = p_d2 + np * nw, *p_cc = p_dr + n;
  double *p_lw = p_cc + n;
  int *p_s = (int *)(p_lw + np * nw);
  HIPCHK(hipMemcpy(p_r, c->h_r, n * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p_rinv, rinv.data(), n * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p_d1, d1.data(), np * nw * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p_d2, d2.data(), np * nw * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p_dr, dr.data(), n * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p_cc, ccw.data(), n * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p_lw, lw.data(), np * nw * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p_s, s.data(), n * sizeof(int), hipMemcpyHostToDevice));
  c->g = Grid{p_r, p_rinv, p_d1, p_d2, p_s, p_dr, p_cc, p_lw, pipe ? nw : 0};
  // the adjoint's transposed rows of D2 + D1/r: column j collects the rows
  // whose windows hold it (nine inside, up to thirteen where the one-sided
  // wall windows overlap)
  {
    std::vector<int> trow((size_t)n * kTrans, 0), tcnt(n, 0);
    std::vector<double> twt((size_t)n * kTrans, 0.0);
    for (int i = 0; i < n; ++i)
      for (int t = 0; t < kStencil; ++t) {
        const int j = s[i] + t;
        if (tcnt[j] >= kTrans) return NSC_ERR_ARG;
        trow[(size_t)j * kTrans + tcnt[j]] = i;
        twt[(size_t)j * kTrans + tcnt[j]] = lw[(size_t)i * kStencil + t];
        ++tcnt[j];
      }
    TRY(dmalloc((void **)&c->t_row, trow.size() * sizeof(int)));
    TRY(dmalloc((void **)&c->t_cnt, tcnt.size() * sizeof(int)));
    TRY(dmalloc((void **)&c->t_wt, twt.size() * sizeof(double)));
    HIPCHK(hipMemcpy(c->t_row, trow.data(), trow.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->t_cnt, tcnt.data(), tcnt.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->t_wt, twt.data(), twt.size() * sizeof(double), hipMemcpyHostToDevice));
  }

  // twiddles
  {
    std::vector<double> t64(2 * d.nt);
    std::vector<float> t32(4 * d.nt);
    twiddles(d.nt, t64.data(), t32.data());
    TRY(dmalloc((void **)&c->tw64_t, t64.size() * sizeof(double)));
    TRY(dmalloc((void **)&c->tw32_t, t32.size() * sizeof(float)));
    HIPCHK(hipMemcpy(c->tw64_t, t64.data(), t64.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->tw32_t, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
    std::vector<double> z64(2 * d.nz);
    std::vector<float> z32(4 * d.nz);
    twiddles(d.nz, z64.data(), z32.data());
    TRY(dmalloc((void **)&c->tw64_z, z64.size() * sizeof(double)));
    TRY(dmalloc((void **)&c->tw32_z, z32.size() * sizeof(float)));
    HIPCHK(hipMemcpy(c->tw64_z, z64.data(), z64.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->tw32_z, z32.data(), z32.size() * sizeof(float), hipMemcpyHostToDevice));
  }

  // stencil kernels: rows first once a nine-row window of three fields'
  // whole radial rows exceeds an XCD's L2 (4 MB)
  c->rows_first = (size_t)kStencil * 3 * field / d.nr > ((size_t)4 << 20) ? 1 : 0;

  // workspaces; where the FP64 theta pass cannot run (its line set exceeds
  // the LDS, and the nonlinear calls refuse FP64), the transform
  // intermediates are sized for FP32 only
  if (!theta_fits(c, NSC_FP64, 0)) inter /= 2;
  TRY(dmalloc(&c->zbuf, inter * c->n_in));
  TRY(dmalloc(&c->wbuf, inter * c->n_out));
  c->cfl_nblk = d.nz * d.nr;
  TRY(dmalloc((void **)&c->cfl_part, (size_t)c->cfl_nblk * sizeof(double)));
  TRY(dmalloc((void **)&c->cfl_val, 4 * sizeof(double)));
  c->e_nblk = 1024;
  TRY(dmalloc((void **)&c->e_part, (size_t)c->e_nblk * sizeof(double)));
  TRY(dmalloc((void **)&c->s_f, field * 4));
  TRY(dmalloc((void **)&c->s_g, field));
  TRY(dmalloc((void **)&c->s_p, field));
  TRY(dmalloc((void **)&c->s_x, field * 4));
  TRY(dmalloc((void **)&c->s_lam, (size_t)d.nmodes * 32));
  TRY(dmalloc((void **)&c->s_u1, field * d.f));
  TRY(dmalloc((void **)&c->s_nn, field * d.f));
  TRY(dmalloc((void **)&c->s_nq, field * d.f));
  c->s_tmp = c->s_u1;  // the initial-state scratch: no step runs meanwhile
  TRY(dmalloc((void **)&c->s_adj, field * c->n_in));
  TRY(dmalloc((void **)&c->s_mean, (size_t)8 * n * sizeof(double)));
  HIPCHK(hipHostMalloc((void **)&c->h_pinned, 64, hipHostMallocDefault));
  HIPCHK(hipHostGetDevicePointer((void **)&c->h_pinned_dev, c->h_pinned, 0));
  HIPCHK(hipEventCreateWithFlags(&c->ev_cfl, hipEventDisableTiming));
  HIPCHK(hipEventCreate(&c->ev0));
  HIPCHK(hipEventCreate(&c->ev1));

  // factors
  const int kp1 = d.kmax + 1;
  const bool packed = sweeps_unrolled(d, (d.mt + 1) * kp1);
  TRY(alloc_factors(&c->fv, d.mt + 1, kp1, n, packed));
  TRY(alloc_factors(&c->fp, d.mt, kp1, n, packed));
  if (d.heated) TRY(alloc_factors(&c->ft, d.mt, kp1, n, packed));
  c->inf.nops = d.mt * kp1;
  TRY(dmalloc((void **)&c->inf.resp, (size_t)8 * n * c->inf.nops * sizeof(double)));
  TRY(dmalloc((void **)&c->inf.ainv, (size_t)4 * c->inf.nops * sizeof(double)));
  TRY(alloc_columns(&c->fv, n));
  TRY(alloc_columns(&c->fp, n));
  if (d.heated) TRY(alloc_columns(&c->ft, n));

  // Delta t-independent pressure factors (slot (0,0): the mean pressure head)
  HIPCHK(launch_factor(c, &c->fp, OP_POISSON, 0.0, 0.0));
  HIPCHK(launch_influence_pressure(c));  // pressure responses: independent of the step size
  HIPCHK(hipStreamSynchronize(c->stream));
  return NSC_OK;
}

int nsc_init(double eta, double Re_i, double Re_o, double Ra, double Pr, int N_r, int M_theta,
             int M_z, double L_z, nsc_ctx **out) {
  if (!out) return NSC_ERR_ARG;
  *out = nullptr;
  int st = validate(eta, Re_i, Re_o, Ra, Pr, N_r, M_theta, M_z, L_z);
  if (st != NSC_OK) return st;
  nsc_ctx *c = new (std::nothrow) nsc_ctx();
  if (!c) return NSC_ERR_OOM;
  st = init_impl(c, eta, Re_i, Re_o, Ra, Pr, N_r, M_theta, M_z, L_z);
  if (st != NSC_OK) {
    nsc_destroy(c);
    return st;
  }
  *out = c;
  return NSC_OK;
}

int nsc_init_pipe(double Re, int N_r, int M_theta, int M_z, double L_z, nsc_ctx **out) {
  if (!out) return NSC_ERR_ARG;
  *out = nullptr;
  if (!std::isfinite(Re)) return NSC_ERR_ARG;
  // the cylinder checks with a dummy radius ratio cover the grid sizes
  int st = validate(0.5, Re, 0.0, 0.0, 1.0, N_r, M_theta, M_z, L_z);
  if (st != NSC_OK) return st;
  nsc_ctx *c = new (std::nothrow) nsc_ctx();
  if (!c) return NSC_ERR_OOM;
  st = init_impl(c, 0.5, Re, 0.0, 0.0, 1.0, N_r, M_theta, M_z, L_z, 1);
  if (st != NSC_OK) {
    nsc_destroy(c);
    return st;
  }
  *out = c;
  return NSC_OK;
}

int nsc_set_stream(nsc_ctx *c, void *s) {
  if (!c) return NSC_ERR_ARG;
  c->stream = (hipStream_t)s;
  return NSC_OK;
}

int nsc_set_precision(nsc_ctx *c, int mode) {
  if (!c || (mode != NSC_FP64 && mode != NSC_MIXED)) return NSC_ERR_ARG;
  c->precision = mode;
  return NSC_OK;
}

int nsc_set_timestep(nsc_ctx *c, double dt, int dynamic, double cfl, double dt_max, int n_corr,
                     double c_implicit) {
  if (!c) return NSC_ERR_ARG;
  if (!(dt > 0.0 && std::isfinite(dt)) || !(cfl > 0.0) || !(dt_max > 0.0) || n_corr < 0 ||
      n_corr > 64 || !(c_implicit > 0.0 && c_implicit <= 1.0) || (dynamic != 0 && dynamic != 1))
    return NSC_ERR_ARG;
  c->dt = dt;
  c->dynamic = dynamic;
  c->cfl = cfl;
  c->dt_max = dt_max;
  c->n_corr = n_corr;
  c->c = c_implicit;
  return NSC_OK;
}

int nsc_nonlinear(nsc_ctx *c, const double *u, double *nh, double *cfl_dt_dev) {
  if (!c || !u || !nh || (const void *)u == (const void *)nh) return NSC_ERR_ARG;
  return nonlinear_impl(c, u, nh, cfl_dt_dev);
}

int nsc_radial_solve(nsc_ctx *c, const double *un, const double *nn, const double *nq, double *out,
                     double *pout) {
  if (!c || !un || !nn || !nq || !out) return NSC_ERR_ARG;
  if ((const void *)out == (const void *)un || (const void *)out == (const void *)nn ||
      (const void *)out == (const void *)nq)
    return NSC_ERR_ARG;
  return solve_impl(c, un, nn, nq, out, pout, c->dt, c->c, 1);
}

int nsc_step(nsc_ctx *c, double *u, double *dt_inout) {
  if (!c || !u || !dt_inout) return NSC_ERR_ARG;
  const double dt = *dt_inout;
  if (!(dt > 0.0 && std::isfinite(dt))) return NSC_ERR_ARG;
  const bool dyn = c->dynamic != 0;
  TRY(pending_nonfinite(c));
  // the bound (NaN for a non-finite state) lands in the host-mapped pinned
  // scalar; the event marks it
  TRY(nonlinear_impl(c, u, c->s_nn, c->cfl_val, c->h_pinned_dev));
  HIPCHK(hipEventRecord(c->ev_cfl, c->stream));
  // predictor, then correctors; the last stage writes u in place (the
  // finalising kernel reads only library scratch, never u^n)
  TRY(solve_impl(c, u, c->s_nn, c->s_nn, c->n_corr == 0 ? u : c->s_u1, nullptr, dt, c->c, 1));
  for (int q = 1; q <= c->n_corr; ++q) {
    TRY(nonlinear_impl(c, c->s_u1, c->s_nq, nullptr));
    TRY(solve_impl(c, u, c->s_nn, c->s_nq, q == c->n_corr ? u : c->s_u1, nullptr, dt, c->c, 1));
  }
  if (!dyn) return query_nonfinite(c);
  HIPCHK(hipEventSynchronize(c->ev_cfl));
  const double dtc = c->h_pinned[0];
  if (std::isnan(dtc)) return NSC_ERR_NONFINITE;
  // hysteresis: shrink to 0.9 of the bound when exceeded, grow (to 0.9 of
  // the bound, capped by dt_max) only past +20 %
  const double b = c->cfl * dtc;
  double next = dt;
  if (b < dt) next = 0.9 * b;
  else if ((b < c->dt_max ? b : c->dt_max) > 1.2 * dt) next = (0.9 * b < c->dt_max ? 0.9 * b : c->dt_max);
  if (!(next >= 1e-12)) return NSC_ERR_DT;
  *dt_inout = next;
  return NSC_OK;
}

int nsc_energy(nsc_ctx *c, const double *u, double *e_dev) {
  if (!c || !u || !e_dev) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  HIPCHK(launch_energy(c, u, e_dev));
  return NSC_OK;
}

int nsc_initial_state(nsc_ctx *c, const double *amps, double *out) {
  if (!c || !amps || !out) return NSC_ERR_ARG;
  HIPCHK(launch_seed(c, amps, c->s_tmp));
  TRY(solve_impl(c, c->s_tmp, nullptr, nullptr, out, nullptr, 1e-3, 1.0, 0));
  HIPCHK(launch_add_base(c, c->s_tmp, out));
  return NSC_OK;
}

int nsc_nonlinear_vjp(nsc_ctx *c, const double *u, const double *nbar, double *ubar) {
  if (!c || !u || !nbar || !ubar) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  if ((const void *)ubar == (const void *)u || (const void *)ubar == (const void *)nbar)
    return NSC_ERR_ARG;
  if (!theta_fits(c, c->precision, 1)) return NSC_ERR_STATE;
  HIPCHK(launch_nonlinear_vjp(c, c->precision, u, nbar, ubar));
  return NSC_OK;
}

int nsc_radial_solve_vjp(nsc_ctx *c, const double *ubar_out, double *ubar_n, double *nbar_n,
                         double *nbar_q) {
  if (!c || !ubar_out || !ubar_n || !nbar_n || !nbar_q) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  const void *o = ubar_out;
  if (o == ubar_n || o == nbar_n || o == nbar_q || (void *)ubar_n == (void *)nbar_n ||
      (void *)ubar_n == (void *)nbar_q || (void *)nbar_n == (void *)nbar_q)
    return NSC_ERR_ARG;
  TRY(ensure_factors(c, c->dt, c->c));
  HIPCHK(launch_solve_vjp(c, ubar_out, ubar_n, nbar_n, nbar_q, c->dt, c->c));
  return NSC_OK;
}

int nsc_step_stages(nsc_ctx *c, const double *u, double *stages, double *u_next) {
  if (!c || !u || !stages || !u_next) return NSC_ERR_ARG;
  const size_t fld = (size_t)c->d.f * c->d.nr * c->d.nmodes * 2;  // doubles per state
  const int nc = c->n_corr;
  if ((const void *)u_next == (const void *)u) return NSC_ERR_ARG;
  if (nc > 0 && (u_next < stages + nc * fld && stages < u_next + fld)) return NSC_ERR_ARG;
  if (nc > 0 && (u < stages + nc * fld && stages < u + fld)) return NSC_ERR_ARG;
  double *xs = const_cast<double *>(u);
  TRY(pending_nonfinite(c));
  // same sequence as nsc_step: N(u); X^(1) = S(u, N, N); X^(q+1) = S(u, N, N(X^(q)));
  // the first nonlinear stage's bound serves the non-finite check
  TRY(nonlinear_impl(c, xs, c->s_nn, c->cfl_val, c->h_pinned_dev));
  HIPCHK(hipEventRecord(c->ev_cfl, c->stream));
  TRY(solve_impl(c, xs, c->s_nn, c->s_nn, nc == 0 ? u_next : stages, nullptr, c->dt, c->c, 1));
  for (int q = 1; q <= nc; ++q) {
    TRY(nonlinear_impl(c, stages + (size_t)(q - 1) * fld, c->s_nq, nullptr));
    TRY(solve_impl(c, xs, c->s_nn, c->s_nq, q == nc ? u_next : stages + (size_t)q * fld, nullptr,
                   c->dt, c->c, 1));
  }
  return query_nonfinite(c);
}

int nsc_step_vjp(nsc_ctx *c, const double *u, const double *stages, const double *ubar_next,
                 double *ubar) {
  TRY(step_vjp_check(c, u, stages, ubar_next, ubar));
  const size_t fld = (size_t)c->d.f * c->d.nr * c->d.nmodes * 2;
  if (!c->s_vjp) TRY(dmalloc((void **)&c->s_vjp, 4 * fld * sizeof(double)));
  return step_vjp_impl(c, u, stages, ubar_next, ubar, c->s_vjp);
}

int nsc_energy_grad(nsc_ctx *c, const double *u, double *g) {
  if (!c || !u || !g || (const void *)u == (const void *)g) return NSC_ERR_ARG;
  if (c->d.pipe) return NSC_ERR_STATE;
  HIPCHK(launch_energy_grad(c, u, g));
  return NSC_OK;
}

int nsc_get_grid(nsc_ctx *c, double *r, int n) {
  if (!c || !r || n < c->d.nr) return NSC_ERR_ARG;
  std::memcpy(r, c->h_r, sizeof(double) * c->d.nr);
  return NSC_OK;
}

int nsc_set_profiling(nsc_ctx *c, int on) {
  if (!c) return NSC_ERR_ARG;
  c->profiling = on ? 1 : 0;
  return NSC_OK;
}

int nsc_get_timings(nsc_ctx *c, double *ms, int n) {
  if (!c || !ms || n < 0) return NSC_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (i < kNumStages) ms[i] = c->stage_ms[i];
    else if (i < 2 * kNumStages) ms[i] = c->stage_cnt[i - kNumStages];
    else ms[i] = 0.0;
  }
  for (int i = 0; i < kNumStages; ++i) c->stage_ms[i] = c->stage_cnt[i] = 0.0;
  return NSC_OK;
}

}  // extern "C"
