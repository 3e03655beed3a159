/*
 * nsc.h -- C ABI of the MI355X Taylor--Couette time-step library (libnsc.so).
 *
 * The library advances the incompressible Navier--Stokes equations (and,
 * optionally, a Boussinesq temperature equation) for the flow between two
 * independently rotating, differentially heated concentric cylinders, with
 * the discretisation described in the nsCouette paper (section 2.1,
 * "Functionality"): Fourier--Galerkin in the azimuthal (theta) and axial (z)
 * directions with pseudospectral, 3/2-rule dealiased nonlinear terms;
 * nine-point finite differences in r; a predictor--corrector integrator with
 * dynamic time-step control; linear terms solved independently per Fourier
 * mode (section 2.2).  The equations themselves are not printed in the paper;
 * the library's conventions are:
 *
 *   units: gap d = 1, time d^2/nu, velocity nu/d; r_i = eta/(1-eta),
 *          r_o = 1/(1-eta); Re_i, Re_o = azimuthal wall speeds;
 *   du/dt = -grad P + lap u + u x omega + Gr T e_z,  Gr = Ra/Pr,
 *   dT/dt = -u . grad T + lap T / Pr,  T(r_i) = +1/2, T(r_o) = -1/2,
 *   div u = 0, no slip at both walls, periodic in theta and z.
 *
 * ARRAY CONVENTION.  Every spectral array is interleaved complex FP64
 * (re, im pairs; torch.complex128), contiguous [F][N_r][M_theta][M_z],
 * F = 3 (u_r, u_theta, u_z) or 4 (+ T) when Ra != 0.  Mode (m, k) has
 * m = 0..M_theta-1 and k = -K..K, K = (M_z-1)/2, stored at index k+K;
 * the physical field is f = sum_k f_0k e^{i k kz z}
 *   + 2 Re sum_{m>=1} sum_k f_mk e^{i(m theta + k kz z)}, kz = 2 pi / L_z,
 * so the m = 0 column must be Hermitian (f_0,-k = conj f_0,k).  Outputs
 * are re-symmetrised.  Radial index j = 0..N_r-1 runs from r_i to r_o on
 * Chebyshev--Gauss--Lobatto points (wall points included).
 *
 * OWNERSHIP.  Unless stated otherwise every array pointer is a DEVICE
 * pointer owned by the caller, at least 16-byte aligned; the library never
 * frees it nor keeps it after the call returns.  The library owns the
 * context and all of its workspaces, freed by nsc_destroy.  All device work
 * is enqueued on the context's stream (nsc_set_stream; default the null
 * stream) and is asynchronous, except where a call says it synchronises.
 * A context is not thread-safe: use one context per host thread.
 *
 * ERRORS.  Every call returns an int status: NSC_OK or a negative code
 * (nsc_strerror gives a message).  Arguments are validated before any device
 * work; a failing call leaves caller arrays untouched when the failure is
 * detected before launch.
 */
#ifndef NSC_H
#define NSC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nsc_ctx nsc_ctx;

enum {
  NSC_OK = 0,
  NSC_ERR_ARG = -1,       /* invalid argument (checked before device work)   */
  NSC_ERR_DEVICE = -2,    /* HIP runtime error or no device                  */
  NSC_ERR_OOM = -3,       /* device allocation failed or size overflow       */
  NSC_ERR_NONFINITE = -4, /* NaN/Inf detected in a reduction                 */
  NSC_ERR_DT = -5,        /* time step collapsed below 1e-12                 */
  NSC_ERR_STATE = -6,     /* call not valid in the context's current state:
                           * also the nonlinear term (and its VJP) at a
                           * precision whose theta line set (all fields of
                           * one (r, z) line, padded, with the twiddles) does
                           * not fit one workgroup's LDS -- FP64 with
                           * N_theta = 1536; the mixed precision fits */
  NSC_ERR_IO = -7         /* state file missing, unreadable, truncated or
                           * not a state file                                */
};

enum { NSC_FP64 = 0, NSC_MIXED = 1 };

/* Create a context for one problem (section 1, the flow between two
 * independently rotating cylinders; section 2.1, where every parameter of a
 * run is read once when the run starts, so that these arguments are the
 * whole description of the problem).  eta in (0,1); Re_i, Re_o wall speeds; Ra >= 0 (0 = isothermal) and Pr > 0
 * if Ra != 0; N_r >= 9 radial points; M_theta >= 1 azimuthal modes with
 * N_theta = 3 M_theta, M_z odd axial modes with N_z = 3 (M_z+1)/2, both
 * padded lengths of the form 2^a 3^b 5^c and <= 4096; L_z > 0 axial period.
 * Computes the grid, the finite-difference weights, transform tables and
 * the Delta t-independent pressure factors, and allocates workspaces.
 * *out receives the context (NULL on failure).  Errors: NSC_ERR_ARG,
 * NSC_ERR_DEVICE, NSC_ERR_OOM. */
int nsc_init(double eta, double Re_i, double Re_o, double Ra, double Pr,
             int N_r, int M_theta, int M_z, double L_z, nsc_ctx **out);

/* Create a context for the pipe-flow variant (abstract and section 4: the
 * method, applied to flows in straight pipes).  Conventions (the paper does
 * not print the pipe formulation; these are this library's): a pipe of
 * radius 1, periodic in z with period L_z, time in R^2/nu, velocity in nu/R;
 * du/dt = -grad P + lap u + u x omega + 4 Re e_z, div u = 0, u = 0 at r = 1:
 * the flow is driven by the constant mean pressure gradient 4 Re, whose
 * laminar solution is u_z = Re (1 - r^2).  Isothermal, F = 3.  Radial points
 * r_j = cos(pi (N_r - 1 - j) / (2 N_r - 1)), j = 0..N_r-1 (the positive half
 * of the 2 N_r Gauss--Lobatto points of [-1, 1]: r = 1 included, the axis
 * not a point).  At the axis an order-m coefficient is even or odd in r as
 * (-1)^m (u_z, pressure) or (-1)^(m+1) (u_r, u_theta): the nine-point rows
 * reach across the axis onto the mirror points -r_k, whose weights are
 * folded onto r_k with that sign.  One wall: the pressure correction has one
 * influence condition, div u = 0 at r = 1.  Mode (0,0): u_r = 0; pressure
 * head p(1) = 0.  nsc_nonlinear, nsc_radial_solve, nsc_step,
 * nsc_set_timestep/precision/stream, nsc_initial_state (perturbation
 * (a_r +- i a_theta) g_{m+-1}(r) for u_r +- i u_theta and a_z g_m(r) for
 * u_z, g_q = r^q (1 - r^2)^2 at peak one, projected as for the cylinders,
 * on Hagen--Poiseuille flow), nsc_get_grid, nsc_probe and the timing calls
 * apply; the energy, adjoint, diagnostics and state-file calls return
 * NSC_ERR_STATE.  Re finite; N_r, M_theta, M_z, L_z as for nsc_init.
 * Errors: NSC_ERR_ARG, NSC_ERR_DEVICE, NSC_ERR_OOM. */
int nsc_init_pipe(double Re, int N_r, int M_theta, int M_z, double L_z, nsc_ctx **out);

/* Release the context and every device buffer it owns.  NULL is a no-op. */
int nsc_destroy(nsc_ctx *ctx);

/* Enqueue all later work on hip_stream (a hipStream_t; NULL = null stream). */
int nsc_set_stream(nsc_ctx *ctx, void *hip_stream);

/* Precision policy: NSC_FP64 (everything FP64) or NSC_MIXED (transforms and
 * pointwise products in FP32 with FP32 accumulation; radial solves,
 * influence correction and reductions stay FP64).  The ABI stays FP64. */
int nsc_set_precision(nsc_ctx *ctx, int mode);

/* Time integration (section 2.1, predictor--corrector with variable step).
 * dt > 0 the (initial) step; dynamic = 1 enables CFL control: with the
 * bound b = cfl * dt_cfl(u^n) evaluated during step n, the next step is
 * 0.9 b if b < dt, min(dt_max, 0.9 b) if min(dt_max, b) > 1.2 dt, else dt
 * (the radial operators are refactorised only on such changes); n_corr >= 0 corrector
 * stages; c_implicit in (0,1] the implicit weight of the viscous term
 * (0.5 = Crank--Nicolson type).  Defaults: dt = 1e-3, dynamic = 0, cfl = 0.5,
 * dt_max = 1e-3, n_corr = 1, c = 0.5.  Radial factors are rebuilt lazily
 * when dt or c changes. */
int nsc_set_timestep(nsc_ctx *ctx, double dt, int dynamic, double cfl,
                     double dt_max, int n_corr, double c_implicit);

/* Nonlinear term N(u) (section 2.1 pseudospectral method): curl and
 * temperature gradient in spectral space, inverse z and theta FFTs onto the
 * 3/2-padded grid, pointwise u x omega and -u . grad T, forward FFTs,
 * truncation, buoyancy N_z += Gr T.  u_hat, n_hat: [F][N_r][M_theta][M_z]
 * (must not alias).  cfl_dt_dev: NULL or one device double receiving
 * dt_cfl = min over grid points of (dr_j/|u_r|, r_j dtheta/|u_theta|,
 * dz/|u_z|) (NaN if a non-finite value was met). */
int nsc_nonlinear(nsc_ctx *ctx, const double *u_hat, double *n_hat,
                  double *cfl_dt_dev);

/* Implicit stage of the step, per Fourier mode (section 2.2: linear terms
 * treated independently per mode): with X+- = u_r +- i u_theta,
 *   f = X^n/dt + (1-c) L X^n + c N^q + (1-c) N^n,
 *   pressure Poisson with Neumann rows, Helmholtz solves (I/dt - c L) X,
 *   influence-matrix correction making div u = 0 at both walls,
 * using the step set by nsc_set_timestep.  u_hat_n, n_hat_n, n_hat_q,
 * u_hat_out: [F][N_r][M_theta][M_z]; u_hat_out must not alias the inputs.
 * p_hat_out: NULL or [N_r][M_theta][M_z] pressure head (mode (0,0): the
 * solution of dp/dr = F_r = c N^q_r + (1-c) N^n_r in divergence form,
 * (D2 + D1/r) p = (D1 + 1/r) F_r, with p(r_i) = 0 and D1 p = F_r at r_o). */
int nsc_radial_solve(nsc_ctx *ctx, const double *u_hat_n,
                     const double *n_hat_n, const double *n_hat_q,
                     double *u_hat_out, double *p_hat_out);

/* One full time step in place: N^n = N(u^n), predictor X^(1) =
 * Solve(u^n, N^n, N^n), then n_corr correctors X^(q+1) = Solve(u^n, N^n,
 * N(X^(q))) (section 2.1).  *dt_inout (HOST pointer): on entry the step
 * size; on return the size for the next step (changed only if dynamic).
 * With dynamic control the call waits for the first nonlinear stage's CFL
 * scalar (the rest of the step stays queued).  Errors: NSC_ERR_NONFINITE
 * when u^n holds a NaN or infinite value (the first nonlinear stage finds
 * it) -- with dynamic control in this call; with a fixed step in this call
 * if that stage has finished when the call returns (the call does not wait
 * for it), else in the next nsc_step or nsc_step_stages call, which waits
 * for it first; NSC_ERR_DT. */
int nsc_step(nsc_ctx *ctx, double *u_hat, double *dt_inout);

/* Perturbation kinetic energy about the basic state (section 3: the flow
 * whose azimuthal velocity and temperature depend on r only and are known in
 * closed form; for the velocity that is circular Couette flow),
 * E = 1/2 int |u - U_b|^2 dV, U_b = (0, A r + B/r, 0), with Clenshaw--Curtis
 * weights in r and Parseval in theta, z; deterministic FP64 reduction.
 * e_dev: one device double. */
int nsc_energy(nsc_ctx *ctx, const double *u_hat, double *e_dev);

/* Divergence-free initial condition exciting selected modes (section 2.1):
 * amps_dev: [F][M_theta][M_z] complex mode amplitudes (m = 0 column made
 * Hermitian, mode (0,0) ignored); the perturbation amps * g(r),
 * g = 16 (r-r_i)^2 (r_o-r)^2, is projected by one backward-Euler Stokes
 * stage (dt = 1e-3, zero wall data) and added to the basic state (Couette
 * flow; conduction profile plus the unprojected temperature amplitudes).
 * Leaves the time-step settings unchanged.  u_hat_out: [F][N_r][M_theta][M_z]. */
int nsc_initial_state(nsc_ctx *ctx, const double *amps_dev, double *u_hat_out);

/* ---- Discrete adjoint (vector--Jacobian products, FP64 inner product
 * <a, b> = sum over every stored entry of Re(conj(a) b); the gradient of a
 * real function w.r.t. a complex entry is dF/dRe + i dF/dIm).  Used for
 * gradients of flow functionals with respect to initial perturbations
 * (optimal-perturbation search) by checkpoint-and-recompute over steps. */

/* u_bar += (dN/du at u_hat)^T n_bar for the nonlinear term of nsc_nonlinear
 * (same precision policy).  u_hat, n_bar, u_bar: [F][N_r][M_theta][M_z];
 * u_bar must not alias the inputs.  Uses the context workspaces. */
int nsc_nonlinear_vjp(nsc_ctx *ctx, const double *u_hat, const double *n_bar,
                      double *u_bar);

/* Transpose of the implicit stage of nsc_radial_solve (same step size and
 * implicit weight; wall data are constants and drop out): with u_bar_out the
 * adjoint of the stage output, accumulates u_bar_n += dS/du_n^T u_bar_out,
 * n_bar_n += dS/dN^n^T u_bar_out, n_bar_q += dS/dN^q^T u_bar_out.  All
 * [F][N_r][M_theta][M_z], pairwise distinct. */
int nsc_radial_solve_vjp(nsc_ctx *ctx, const double *u_bar_out,
                         double *u_bar_n, double *n_bar_n, double *n_bar_q);

/* One predictor--corrector step of the size set by nsc_set_timestep (fixed;
 * no step-size update; NSC_ERR_NONFINITE as for a fixed nsc_step) from
 * u_hat, keeping the stage states the
 * adjoint needs: stages = X^(1..n_corr) (n_corr consecutive state-sized
 * arrays, written), u_next = u^{n+1} (written).  Same kernels and arithmetic
 * as nsc_step, so the states agree with it bit for bit.  DEVICE arrays;
 * u_next and stages must not alias u_hat or each other. */
int nsc_step_stages(nsc_ctx *ctx, const double *u_hat, double *stages, double *u_next);

/* Vector--Jacobian product of one step (the adjoint of nsc_step_stages at
 * u_hat with its stage states): u_bar = (d u^{n+1} / d u^n)^T u_bar_next,
 * written.  Chains the transposed stages: for q = n_corr..1 the transposed
 * implicit stage, then the nonlinear VJP at X^(q); finally the predictor's
 * transposed stage and the nonlinear VJP at u_hat.  DEVICE arrays; u_bar
 * distinct from the inputs.  The first call allocates four state-sized
 * adjoint workspaces (kept until nsc_destroy); NSC_ERR_OOM if that fails. */
int nsc_step_vjp(nsc_ctx *ctx, const double *u_hat, const double *stages,
                 const double *u_bar_next, double *u_bar);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same product as nsc_step_vjp, by the same kernels in the same order, with
 * its four state-sized adjoint workspaces taken from a static device array
 * of 128 MiB that the library holds on every device it runs on until the
 * process ends.  Allocates nothing.  States up to 32 MiB
 * (F * N_r * M_theta * M_z * 16 bytes) -- larger ones return NSC_ERR_ARG
 * before any device work.  Every context on a device shares that array, so
 * calls that overlap on one device (any contexts, any streams) race; the
 * array keeps the last call's contents and each call clears what it needs.
 * Same arguments and other errors as nsc_step_vjp; NSC_ERR_DEVICE if the
 * array's address could not be obtained when the context was created. */
int nsc_step_vjp_noalloc(nsc_ctx *ctx, const double *u_hat, const double *stages,
                         const double *u_bar_next, double *u_bar);

/* Gradient of nsc_energy (the perturbation energy about the section 3 basic
 * state) with respect to the state: g = 2 pi L_z w_j r_j c_m (u - U_b) for the
 * velocity fields, 0 for T (c_0 = 1, c_m = 2).  g is written, not added. */
int nsc_energy_grad(nsc_ctx *ctx, const double *u_hat, double *g);

/* Radial grid points r_j (HOST array of n >= N_r doubles). */
int nsc_get_grid(nsc_ctx *ctx, double *r_host, int n);

/* Per-kernel device time accumulated since the last call, in ms (HOST array
 * of n doubles), one entry per kernel: [0] z-inverse (mean profiles, curl,
 * inverse z FFT), [1] theta FFTs + products, [2] forward z FFT (with the
 * CFL reduction when a bound is asked for), [3] restart remap
 * (nsc_remap_state, and nsc_load_state at another resolution), [4]
 * right sides, [5] Poisson right side (and temperature wall
 * rows), [6] pressure/temperature sweeps, [7] velocity sweeps, [8] influence
 * coefficients, [9] finalisation, [10] factorisation, [11] velocity right
 * sides (f - grad p); entries [12..23] the launch counts of the same
 * kernels.  Counters are reset by the call.  Timing is enabled by
 * nsc_set_profiling(ctx, 1): each kernel is then bracketed by HIP events on
 * the context stream and the host waits for the second event. */
int nsc_get_timings(nsc_ctx *ctx, double *ms, int n);
int nsc_set_profiling(nsc_ctx *ctx, int on);

/* Heated-flow diagnostics (section 3: the Nusselt number at the inner
 * cylinder, the heat transfer there over that of the basic state at the same
 * temperature difference).  Writes 4 DEVICE doubles to out: Nu_i, Nu_o (the
 * theta-z mean temperature's radial derivative at r_i, r_o times r ln(eta),
 * one-sided nine-point stencils; 1 for the conduction profile; 0 without
 * temperature), then G_i, G_o, the torques -2 pi L_z r^3 d(<u_theta>/r)/dr at
 * the two walls (4 pi L_z B for Couette flow).  Queued on the context
 * stream, no synchronisation.  Errors: NSC_ERR_ARG, NSC_ERR_DEVICE. */
int nsc_diagnostics(nsc_ctx *ctx, const double *u_hat, double *out);

/* Every field at n <= 64 physical points (section 3: probe time series at
 * fixed points): point i at radial grid row rows[i], azimuth theta[i], axial
 * position z[i] (HOST arrays, read before the call returns).  out: DEVICE
 * [n][F] doubles, the Fourier sums sum_k u_0k e^{i k kz z} + 2 Re sum_{m>=1,k}
 * u_mk e^{i (m theta + k kz z)}, kz = 2 pi / L_z.  Queued on the context
 * stream.  Errors: NSC_ERR_ARG (n, a row out of range, a non-finite
 * position), NSC_ERR_DEVICE. */
int nsc_probe(nsc_ctx *ctx, const double *u_hat, int n, const int *rows, const double *theta,
              const double *z, double *out);

/* Checkpoint-restart on the spectral coefficients, with a change of
 * resolution at the restart (section 2.1: the resolution may change at every
 * restart through interpolation and mode padding; section 2.4: the restart
 * works on the coefficients).
 *
 * State file (little endian): a 128-byte header -- char magic[8] =
 * "NSCSTATE"; uint32 version = 1; uint32 F (3 or 4); int32 N_r, M_theta,
 * M_z; uint32 zero; FP64 eta, Re_i, Re_o, Ra, Pr, L_z, time; 40 zero bytes --
 * then the state [F][N_r][M_theta][M_z] as (re, im) FP64 pairs, the layout
 * of u_hat everywhere in this interface. */

/* Write the DEVICE state u_hat of the context's shape, with the context's
 * parameters and the given time, to the file at path (created or replaced;
 * staged through pinned host memory on the context stream, which is
 * synchronised; on an error the partial file is removed).  Errors:
 * NSC_ERR_ARG, NSC_ERR_IO, NSC_ERR_DEVICE, NSC_ERR_OOM. */
int nsc_save_state(nsc_ctx *ctx, const double *u_hat, double time, const char *path);

/* Host only (no device, no context): the header of a state file.  dims: HOST
 * int[4] = F, N_r, M_theta, M_z; params: HOST double[7] = eta, Re_i, Re_o, Ra,
 * Pr, L_z, time.  Errors: NSC_ERR_ARG, NSC_ERR_IO (also for a payload whose
 * size does not match the header). */
int nsc_read_state_header(const char *path, int *dims, double *params);

/* Read a state file into the DEVICE array u_hat of the context's shape.  The
 * file's geometry must be the context's (same F, eta and L_z to 1e-12
 * relative, else NSC_ERR_ARG); its flow parameters may differ (the context's
 * apply from here on).  At another resolution the state is carried over as
 * nsc_remap_state does, through a temporary device copy of the file's state.
 * time_out: NULL or a HOST double receiving the file's time.  Errors:
 * NSC_ERR_ARG, NSC_ERR_IO, NSC_ERR_DEVICE, NSC_ERR_OOM. */
int nsc_load_state(nsc_ctx *ctx, const char *path, double *u_hat, double *time_out);

/* Carry a DEVICE state src [F][N_r_src][M_theta_src][M_z_src] of the same
 * geometry to the context's resolution, into the DEVICE array dst (context
 * shape; the two must not overlap).  Modes (m, k) present at both
 * resolutions keep their coefficients, new modes are zero, modes past the
 * new truncation are dropped; each mode's radial profile is then the value
 * on the context's grid of the polynomial through the old grid's points
 * (both grids Chebyshev--Gauss--Lobatto between the walls, whose values are
 * kept).  N_r_src >= 9, M_theta_src >= 1, M_z_src odd.  Synchronises the
 * context stream.  Errors: NSC_ERR_ARG, NSC_ERR_DEVICE, NSC_ERR_OOM. */
int nsc_remap_state(nsc_ctx *ctx, const double *src, int N_r_src, int M_theta_src,
                    int M_z_src, double *dst);

/* Static description of the status code. */
const char *nsc_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* NSC_H */
