// Internal declarations shared by the host runtime and the HIP kernels of
// libnsc.so.  Not part of the public ABI (include/nsc.h).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/nsc.h"

namespace nsc {

constexpr int kStencil = 9;    // nine-point radial stencils (section 2.1 default)
constexpr int kHalf = 4;       // stencil half width
constexpr int kSlots = 9;      // compact LU row: L[4] | 1/U_jj | U[4]
constexpr int kTrans = 16;     // slots per column of a transposed stencil (13 used at most)
constexpr int kEdge = 20;      // extra U entries of rows 0..3 + extra L of rows N-4..N-1
constexpr int kMaxRadix = 8;
constexpr int kMaxStages = 12;
constexpr int kMaxFFT = 4096;
constexpr int kFftThreads = 1024;  // launch bound of the FFT kernels
constexpr int kWaveRegs = 16;      // complex values per lane in a wavefront-scope FFT stage
constexpr int kNumStages = 12;  // timed kernels (see nsc_get_timings)
constexpr int kMaxProbes = 64;  // probe points per nsc_probe call

struct FftPlan {
  int n = 0;
  int nst = 0;
  int min_radix = 8;
  int wave_lines = 0;  // lines one wavefront transforms at once (0: block-scope only)
  int radix[kMaxStages] = {0};
};

// Device-side read-only tables of the radial discretisation.
struct Grid {
  const double *r;     // [N_r] radial points
  const double *rinv;  // [N_r] 1/r
  const double *d1;    // [N_r][9] first-derivative weights
  const double *d2;    // [N_r][9] second-derivative weights
  const int *s;        // [N_r] first node of each row's window
  const double *dr;    // [N_r] local spacing for the CFL bound
  const double *ccw;   // [N_r] Clenshaw--Curtis weights on [r_i, r_o]
  const double *lw;    // [N_r][9] weights of D2 + D1/r (fma(d1, 1/r, d2))
  // pipe: d1, d2 and lw hold a second set of rows for functions odd in r
  // (mirror points folded with the sign -1) at this element offset; 0 for
  // the cylinders, whose rows do not depend on a parity
  int podd;
};

// Problem sizes and physical constants passed by value to kernels.
struct Dims {
  int nr, mt, mz, kmax, nt, nz, nmodes, f, heated;
  double kz, gr, pr, re_i, re_o, a_cou, b_cou, r_i, r_o, lz;
  int pipe;   // 1: pipe flow (axis at r = 0, wall at r = 1), 0: two cylinders
  double gp;  // pipe: the driving mean pressure gradient -dP/dz = 4 Re
};

// Parity of an order-q radial function of the pipe (odd q: odd in r); the
// cylinders have a single set of rows.
__host__ __device__ __forceinline__ int odd_off(const Grid &g, int q) { return (q & 1) ? g.podd : 0; }

// Compact no-pivot LU factors of a family of radial operators.
// vals: [N_r][kSlots][nops], edge: [kEdge][nops]; op = q * (K+1) + |k|.
// pk and pc (only where the fully unrolled sweeps run, else null): the band
// entries packed per operator, so that a lane fetches four of them with two
// 16-byte loads.  pk: [N_r][2][nops][4], the L row (slots 0-3) and the U row
// (slots 5-8) of row j; pc: [N_r][2][nops][4], the L column below the
// diagonal (L(j+t, j), t = 1..4) and the U column above it (U(j-t, j)),
// zero outside the matrix (the transposed sweeps of the adjoint).
struct Factors {
  double *vals = nullptr;
  double *edge = nullptr;
  double *pk = nullptr;
  double *pc = nullptr;
  int nq = 0;   // number of q values
  int nops = 0;
};

// The sweeps run fully unrolled (column in LDS, 32 or 64 radial points,
// factor offsets within 32 bits) for these grids; nops_max is the largest
// operator count of the context's factor families.  Their factors carry pk.
inline bool sweeps_unrolled(const Dims &d, int nops_max) {
  return (d.nr == 64 || d.nr == 32) &&
         (size_t)d.nr * kSlots * sizeof(double) * (size_t)nops_max < ((size_t)1 << 31);
}

// Homogeneous (influence) responses per (m, |k|), op = m*(K+1)+|k|:
// resp: [8][N_r][nops] = p1, p2, X+1, X+2, X-1, X-2, h1, h2 (X_z,j = -i kappa h_j)
// ainv: [4][nops] the inverse 2x2 influence matrix.
struct Influence {
  double *resp = nullptr;
  double *ainv = nullptr;
  int nops = 0;
};

}  // namespace nsc

struct nsc_ctx {
  nsc::Dims d{};
  double eta = 0, ra = 0;
  int n_in = 0, n_out = 0;
  // time integration
  double dt = 1e-3, cfl = 0.5, dt_max = 1e-3, c = 0.5;
  int dynamic = 0, n_corr = 1, precision = NSC_FP64;
  // cached factor parameters
  double fac_dt = -1.0, fac_c = -1.0;
  hipStream_t stream = nullptr;
  int device = 0;
  int lds_max = 64 * 1024;  // dynamic LDS bytes per workgroup (device limit)
  int cu_count = 256;       // compute units
  int rows_first = 0;       // stencil kernels walk rows first (long radial rows)
  int lds_cu = 160 * 1024;  // LDS bytes per compute unit
  // host copies
  double *h_r = nullptr;
  // device tables
  nsc::Grid g{};
  void *tables = nullptr;  // single allocation backing g
  double *tw64_t = nullptr, *tw64_z = nullptr;  // [n][2] twiddles e^{-2 pi i t/n}
  float *tw32_t = nullptr, *tw32_z = nullptr;   // [n][4] compensated (hi, lo) twiddles
  nsc::FftPlan plan_t{}, plan_z{};
  // factors
  nsc::Factors fv{}, ft{}, fp{};
  nsc::Influence inf{};
  // workspaces
  void *zbuf = nullptr;    // [n_in][N_r][N_z][M_theta] complex (FP64 size)
  void *wbuf = nullptr;    // [n_out][N_r][N_z][M_theta] complex
  double *cfl_part = nullptr;  // per-block CFL partial minima
  int cfl_nblk = 0;
  double *cfl_val = nullptr;   // [2] scalars
  double *e_part = nullptr;    // energy partials
  int e_nblk = 0;
  double *s_f = nullptr;    // [4][N_r][modes] complex right sides
  double *s_g = nullptr;    // [N_r][modes] complex divergence
  double *s_p = nullptr;    // [N_r][modes] complex p0
  double *s_x = nullptr;    // [4][N_r][modes] complex X0+, X0-, X0z, T
  double *s_lam = nullptr;  // [modes][2] complex
  // transposed rows of D2 + D1/r (cylinders): column j's entries (row,
  // weight), kTrans slots per column, t_cnt[j] of them used
  int *t_row = nullptr, *t_cnt = nullptr;
  double *t_wt = nullptr;
  double *s_vjp = nullptr;  // adjoint workspaces of nsc_step_vjp: 4 states (allocated on first use)
  double *s_u1 = nullptr;   // [F][N_r][modes] complex intermediate state
  double *s_nn = nullptr;   // [F][N_r][modes] complex N^n
  double *s_nq = nullptr;   // [F][N_r][modes] complex N^q
  double *s_tmp = nullptr;  // [F][N_r][modes] initial-state scratch (shares s_u1's memory)
  double *s_adj = nullptr;  // [n_in][N_r][modes] complex adjoint of the derived fields
  double *s_mean = nullptr;  // [8][N_r] mean-flow profiles of the current nonlinear call
  double *h_pinned = nullptr;  // pinned host scalar(s)
  double *h_pinned_dev = nullptr;  // its device-side address (kernels write the CFL bound)
  hipEvent_t ev_cfl = nullptr;
  int nan_pending = 0;  // a fixed-size step's non-finite check not read yet
  // profiling
  int profiling = 0;
  double stage_ms[nsc::kNumStages] = {0};
  double stage_cnt[nsc::kNumStages] = {0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace nsc {

// Stage timing (optional, synchronising): the scope's work on the context
// stream between two events, accumulated per stage.
struct StageTimer {
  nsc_ctx *c;
  int stage;
  StageTimer(nsc_ctx *ctx, int s) : c(ctx), stage(s) {
    if (c->profiling) (void)hipEventRecord(c->ev0, c->stream);
  }
  ~StageTimer() {
    if (c->profiling) {
      (void)hipEventRecord(c->ev1, c->stream);
      (void)hipEventSynchronize(c->ev1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
      c->stage_ms[stage] += ms;
      c->stage_cnt[stage] += 1.0;
    }
  }
};


// ---- launchers (kernels in *.hip) -----------------------------------------
hipError_t launch_zinv(const nsc_ctx *c, int prec, const double *u);
hipError_t launch_theta(const nsc_ctx *c, int prec, int want_cfl);
// whether one theta workgroup's line set (all fields of an (r, z) line, with
// the twiddles) fits the LDS at this precision; adjoint: the transposed pass
bool theta_fits(const nsc_ctx *c, int prec, int adjoint);
// cfl_out (device, or null): the minimum CFL bound of the preceding theta
// pass, reduced by the z-forward kernel; cfl_host: null or a host-mapped
// pinned scalar receiving the same value
hipError_t launch_zfwd(const nsc_ctx *c, int prec, const double *u, double *n_hat, double *cfl_out,
                       double *cfl_host);

hipError_t launch_factor(const nsc_ctx *c, Factors *f, int kind, double alpha,
                         double beta);
// two operator sets of one kind and shift alpha in one launch (betas and
// operator counts may differ)
hipError_t launch_factor2(const nsc_ctx *c, Factors *f0, Factors *f1, int kind, double alpha,
                          double beta0, double beta1);
hipError_t launch_influence_pressure(const nsc_ctx *c);
hipError_t launch_influence_setup(const nsc_ctx *c);
hipError_t launch_rhs(const nsc_ctx *c, const double *u, const double *nn,
                      const double *nq, double dt, double cc);
hipError_t launch_fill_zero(const nsc_ctx *c, double *p, size_t n);
hipError_t launch_add(const nsc_ctx *c, double *y, const double *x, size_t n);
hipError_t launch_solve_sweeps(const nsc_ctx *c, int stage, const double *nn, const double *nq,
                               double cc, int walls, int want_p);
hipError_t launch_influence(const nsc_ctx *c);
hipError_t launch_finalize(const nsc_ctx *c, double *out, double *p_out);
hipError_t launch_energy(const nsc_ctx *c, const double *u, double *e_dev);
hipError_t launch_seed(const nsc_ctx *c, const double *amps, double *out_pert);
hipError_t launch_add_base(const nsc_ctx *c, const double *pert_tilde, double *out);
// overwrite: bit 1 ubar_n, 2 nbar_n, 4 nbar_q written instead of accumulated
hipError_t launch_solve_vjp(const nsc_ctx *c, const double *ubar_out, double *ubar_n,
                            double *nbar_n, double *nbar_q, double dt, double cc,
                            int overwrite = 0);
hipError_t launch_energy_grad(const nsc_ctx *c, const double *u, double *gout);
hipError_t launch_nonlinear_vjp(const nsc_ctx *c, int prec, const double *u, const double *nbar,
                                double *ubar);

// The step VJP (nsc_step_vjp): argument checks, and its sequence with the
// four state-sized adjoint workspaces at `work`.
int step_vjp_check(const nsc_ctx *c, const double *u, const double *stages,
                   const double *ubar_next, const double *ubar);
int step_vjp_impl(nsc_ctx *c, const double *u, const double *stages, const double *ubar_next,
                  double *ubar, double *work);
// Record the device address of the allocation-free entry point's static
// scratch array for the current device (called by nsc_init).
void noalloc_setup(int device);

// operator kinds for launch_factor
enum { OP_HELMHOLTZ = 0, OP_POISSON = 1, OP_MEAN_PRESSURE = 2 };

// XCD-aware workgroup order: the dispatcher hands consecutive workgroups to
// the 8 XCDs in turn, each with its own L2.  Remapping the linear workgroup
// id gives every XCD a contiguous range of logical tiles, so neighbouring
// tiles (which share cache lines: transposed intermediates, stencil rows,
// operator factors) meet in the same L2.
__device__ __forceinline__ int xcd_remap(int w, int G) {
  const int q = G / 8, r = G % 8;
  const int x = w % 8, l = w / 8;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Logical (x, y, z) block coordinates after the XCD remap with y (the radial
// row) fastest, then z, then x: each XCD walks the rows of a few mode tiles
// in order, so the nine-row stencil windows of neighbouring rows stay in its
// L2 however long a radial row is.
__device__ __forceinline__ void xcd_rows_first(int &bx, int &by, int &bz) {
  const int gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const int L = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gz);
  by = L % gy;
  const int rest = L / gy;
  bz = rest % gz;
  bx = rest / gz;
}

// The stencil kernels' block coordinates: rows first where a nine-row
// window of whole radial rows would not fit an XCD's L2 (the host decides),
// else the dispatch order (short rows: the window is L2-resident already).
__device__ __forceinline__ void stencil_block(int rows_first, int &bx, int &by, int &bz) {
  if (rows_first) {
    xcd_rows_first(bx, by, bz);
  } else {
    bx = blockIdx.x;
    by = blockIdx.y;
    bz = blockIdx.z;
  }
}

}  // namespace nsc
