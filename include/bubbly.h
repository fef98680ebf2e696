/*
 * bubbly.h -- C ABI of libbubbly.so, the MI355X (gfx950) hot path of the
 * phase-averaged cavitating bubbly-flow solver of Vaca-Revelo, Wilfong,
 * Bryngelson and Gnanaskandan, "Hardware-Accelerated Phase-Averaging for
 * Cavitating Bubbly Flows" (arXiv:2511.21031).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Every function returns int: BUB_OK (0) or a negative BUB_E* code.  No
 *    exception crosses the ABI.  Argument errors are reported synchronously,
 *    before anything is enqueued.
 *  * Array arguments are caller-owned DEVICE pointers (for instance
 *    torch.Tensor.data_ptr() of a CUDA/HIP tensor) unless marked "host".
 *    They must stay valid until the enqueued work has finished.
 *  * `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued on it; nothing synchronises the host except
 *    bub_last_error and the functions documented as synchronous.
 *  * Units are SI.  Fields are structure-of-arrays, [var][z][y][x] with x
 *    fastest, N = nx*ny*nz cells per field, FP64.
 *  * Conserved state q[nvar][N], nvar = ndim + 3 + 2*nb (Sec. 2 eq.
 *    euler_transport, Sec. 2.2 eqs. e:alpha and the bin-variable equation):
 *        rho, rho*u_1..ndim, E, alpha, (n R)_1..nb, (n Rdot)_1..nb
 *    with rho the mixture density (1-alpha) rho_l, E the mixture total energy
 *    (1-alpha)(p_l + gamma pi_inf)/(gamma-1) + rho|u|^2/2, n the bubble number
 *    density and R, Rdot the radius and wall velocity of each equilibrium-radius
 *    bin.  n is not stored: alpha = (4 pi/3) n mean(R^3) (eq. e:ndf) gives
 *    n = sqrt((4 pi/3) sum_i w_i (nR_i)^3 / alpha).
 *  * A context owns only its own small device buffers (bin table, one
 *    primitive scratch field set, scalars for the time step and the error
 *    word) and is not thread-safe: calls on one context must be serialised by
 *    the caller (one stream per context is the intended use).
 *  * Numerical failures found on the device (non-finite state, non-positive
 *    radius, void fraction outside [0,1), p_l + pi_inf <= 0, sub-step budget
 *    exhausted) set a sticky error word read by bub_last_error.
 */
#ifndef BUBBLY_H
#define BUBBLY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BUB_OK = 0,
    BUB_EINVAL = -1,        /* invalid argument (null pointer, bad size, bad option) */
    BUB_ENOMEM = -2,        /* device or host allocation failed */
    BUB_EHIP = -3,          /* HIP runtime error (launch, copy, no device) */
    BUB_ENONFINITE = -4,    /* device: NaN/Inf or inadmissible state (rho, alpha, p_l) */
    BUB_ENEGR = -5,         /* device: non-positive bubble radius */
    BUB_ESUBSTEP = -6,      /* device: adaptive bubble sub-step budget exhausted */
    BUB_EUNSUPPORTED = -7   /* valid request the library does not support */
};

enum { BUB_BC_PERIODIC = 0, BUB_BC_REFLECTIVE = 1 };
enum { BUB_PREC_FP64 = 0, BUB_PREC_MIXED = 1 };
enum { BUB_BUBBLES_UNSPLIT = 0, BUB_BUBBLES_SPLIT = 1 };

/* Cartesian grid.  ndim in {1,2,3}; n[d] = 1 and dx[d] ignored for d >= ndim.
 * bc[d][0/1] = low/high boundary of direction d, both ends alike: 0 periodic,
 * 1 reflective (mirror ghost cells, normal velocity negated; needs n[d] >= 3)
 * or 2 non-reflective (Sec. 5.1, after Thompson: every ghost cell takes the
 * boundary cell's state, so the Riemann problem at the boundary face has no
 * jump and no wave enters through it; an outgoing plane wave at normal
 * incidence leaves with a reflection of order 1e-5 of its amplitude at 12
 * cells per pulse width).  The Lagrangian calls take 0 and 1 only. */
typedef struct { int ndim; int n[3]; double dx[3]; int bc[3][2]; } bub_grid;

/* Stiffened-gas liquid, eq. eos_liquid: p_l = (gamma-1) rho_l e_l - gamma pi_inf.
 * rho0, p0: reference state (equilibrium bubble pressure p_g0 = p0 + 2 sigma/R0 - pv). */
typedef struct { double gamma, pi_inf, rho0, p0; } bub_liquid;

/* Bubble contents and interface: polytropic exponent kappa (p_b = p_g0 (R0/R)^(3 kappa)),
 * surface tension sigma, liquid viscosity mu (inside Keller--Miksis only), vapour pressure pv. */
typedef struct { double kappa, sigma, mu, pv; } bub_gas;

/* Log-normal equilibrium radii (Sec. 2.2): nb odd bins over ln(R0/r0_median) in
 * [-3 sigma_ln, 3 sigma_ln], composite Simpson weights of the normal pdf, normalised. */
typedef struct { int nb; double r0_median, sigma_ln; } bub_bins;

/* Bubble contents (Sec. 2).  BUB_CONTENTS_POLYTROPIC: gas with p_b = p_g0 (R0/R)^(3 kappa),
 * p_g0 = p0 + 2 sigma/R0 - pv.  BUB_CONTENTS_TRANSFER: gas and vapour with heat and vapour transfer
 * at the wall through constant transfer coefficients (eq. massVaporRate and the contents-pressure
 * equation that follows it).  The state then carries, after (n Rdot)_i, (n p_b)_i and (n m_v)_i per
 * bin (nvar = ndim + 3 + 4 nb; p_b the contents' pressure, m_v the vapour mass of one bubble),
 * gas.kappa is not used and gas.pv is the vapour's saturation pressure at T0 (0 <= pv < p0).  Per
 * bubble: Tbar = p_b V/(m_g Rg + m_v Rv) with the bin's gas mass m_g = (p_b0 - pv) V0/(Rg T0);
 * the wall stays at T0 with its vapour saturated; wall gradients dT/dr = beta_T (T0 - Tbar)/R and
 * dchi/dr = beta_c (chi_w - m_v/(m_v + m_g))/R; dm_v/dt = 4 pi R^2 D_v rho_w/(1 - chi_w) dchi/dr;
 * dp_b/dt = 3 gam_b/R (-Rdot p_b + Rv T0 dm_v/dt/(4 pi R^2) + (gam_b - 1)/gam_b k_b dT/dr).  At
 * equilibrium p_b0 = p0 + 2 sigma/R0 and m_v0 = pv V0/(Rv T0).  The paper does not give the
 * coefficients: the caller does.  Ensemble-averaged model only (the Lagrangian calls return
 * BUB_EUNSUPPORTED); stage shape 0 with the separate primitive pass.  gam_b: specific-heat ratio of
 * the contents; Rg, Rv: gas constants of gas and vapour (J/(kg K)); T0: liquid temperature (K);
 * k_b: thermal conductivity of the contents (W/(m K)); D_v: vapour-gas diffusion coefficient
 * (m^2/s); beta_T, beta_c: the transfer coefficients (>= 0). */
enum { BUB_CONTENTS_POLYTROPIC = 0, BUB_CONTENTS_TRANSFER = 1 };
typedef struct { double gam_b, Rg, Rv, T0, k_b, D_v, beta_T, beta_c; } bub_transfer;

/* Options.  cfl: time step fraction for dt <= 0 requests.  precision:
 * BUB_PREC_FP64 or BUB_PREC_MIXED (FP32 reconstruction/Riemann/flux differences,
 * FP64 primitives, moments, Keller--Miksis, sources and RK accumulation).
 * bubble_mode: BUB_BUBBLES_UNSPLIT (bubble sources inside every RK stage) or
 * BUB_BUBBLES_SPLIT (Strang splitting with adaptive embedded RK3/RK2 bubble
 * sub-steps, Sec. 3; sub_rtol and max_substeps apply).  viscous: 0 for an
 * inviscid carrier (the liquid viscosity gas.mu enters Keller--Miksis only), 1
 * to add the liquid's viscous stress T = mu (grad u + grad u^T - 2/3 div(u) I)
 * (eq. stressTensor) to the mixture fluxes: -T in the momentum flux and -T.u in
 * the energy flux of eq. euler_transport, by second-order central differences
 * at each face (normal derivatives from the two cells, transverse derivatives
 * averaged over the two cells' central differences, face velocity their mean).
 * The stress is added by a pass after each stage kernel (so the stages of a
 * viscous problem take a separate primitive pass).  The time step stays the
 * acoustic CFL step (the viscous limit dx^2/(2 ndim nu) is far larger at
 * bubbly-flow scales).  contents: BUB_CONTENTS_POLYTROPIC or BUB_CONTENTS_TRANSFER
 * (below); transfer: its constants (ignored for polytropic contents). */
typedef struct {
    double cfl;
    int precision;
    int bubble_mode;
    double sub_rtol;
    int max_substeps;
    int viscous;
    int contents;
    bub_transfer transfer;
} bub_opts;

typedef struct bub_ctx bub_ctx;

/* Create a context for one problem on the current HIP device.  Computes the bin
 * table on the host and allocates the context's device buffers
 * (about (ndim+6)*N*8 bytes).  *out receives the context (caller destroys it). */
int bub_ctx_create(const bub_grid *grid, const bub_liquid *liq, const bub_gas *gas,
                   const bub_bins *bins, const bub_opts *opts, bub_ctx **out);

/* Free a context.  A context from bub_ctx_create waits for the device and
 * frees its buffers; one from bub_ctx_create_on only frees host memory (the
 * caller keeps the device buffer alive until work that uses it has finished). */
int bub_ctx_destroy(bub_ctx *ctx);

/* Device bytes a context needs (bin table, primitive scratch, scalars). */
int bub_ctx_buffer_bytes(const bub_grid *grid, const bub_bins *bins, size_t *bytes);

/* As bub_ctx_create, but the context lives in `buffer` (caller-owned device
 * memory of at least bub_ctx_buffer_bytes, 256-byte aligned) and is initialised
 * by a kernel enqueued on `stream`: no device allocation and no host
 * synchronisation, so problems can be admitted while others run. */
int bub_ctx_create_on(const bub_grid *grid, const bub_liquid *liq, const bub_gas *gas, const bub_bins *bins,
                      const bub_opts *opts, void *buffer, size_t bytes, void *stream, bub_ctx **out);

/* Sizes: nvar conserved variables, nprim primitive scratch fields, ncells = N,
 * state_bytes = nvar*N*8, work_bytes = the `work` buffer bub_rk3_step needs.
 * Any output pointer may be NULL. */
int bub_layout(const bub_ctx *ctx, int *nvar, int *nprim, int64_t *ncells,
               size_t *state_bytes, size_t *work_bytes);

/* Copy the bin table to host arrays r0[nb], w[nb] (host pointers). */
int bub_bins_get(const bub_ctx *ctx, double *r0, double *w);

/* Conserved state from primitives (Sec. 4: initial conditions, then device
 * residency).  prim[ndim+3][N] = rho_l, u_1..ndim, p_l, alpha (device);
 * every bubble starts at its equilibrium radius with zero wall velocity:
 * n = alpha / ((4 pi/3) sum w R0^3), (nR)_i = n R0_i, (nRdot)_i = 0.
 * q[nvar][N] (device) is written. */
int bub_init_state(bub_ctx *ctx, const double *prim, double *q, void *stream);

/* Right-hand side of the semi-discrete system (Sec. 3, finite-volume form):
 * rhs = sum_d (F_{-1/2} - F_{+1/2}) / dx_d + s, with WENO5 reconstruction
 * (Sec. 3) of rho, u, p_l, alpha, n, B = mean(R^3 p_bw)/mean(R^3) -
 * rho mean(R^3 Rdot^2)/mean(R^3), R_i, Rdot_i; HLLC fluxes with face pressure
 * p = (1-alpha) p_l + alpha B (eq. e:pressure); sources 3 alpha
 * mean(R^2 Rdot)/mean(R^3) (eq. e:alpha), n Rdot_i and n Rddot_i with Rddot_i
 * from Keller--Miksis (eq. keller_miksis) driven by the cell's p_l.
 * q (device, read) and rhs (device, written) are [nvar][N] and must not alias.
 * In split mode the bubble source terms are left out (they belong to the
 * bubble sub-steps). */
int bub_rhs_stage(bub_ctx *ctx, const double *q, double *rhs, void *stream);

/* One SSP-RK3 step (Sec. 3, third-order TVD Runge--Kutta), in place on q.
 * work: device buffer of work_bytes (two state copies).  dt > 0: fixed step;
 * dt <= 0: dt = cfl * min over cells and directions of dx_d/(|u_d| + c),
 * computed on the device from q (no host synchronisation).  dt_dev (device
 * double, may be NULL) receives the step used.  In split mode the step is
 * S_b(dt/2) S_f(dt) S_b(dt/2) (Strang splitting, Sec. 3). */
int bub_rk3_step(bub_ctx *ctx, double *q, double *work, double dt, double *dt_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): bub_rhs_stage without
 * a context.  The problem is described as for bub_ctx_create; the context's device
 * buffers (bin table, scalars, one primitive scratch of (ndim+6)*N doubles) live in
 * one static device array of BUB_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends, and nothing is allocated (no hipMalloc, no host heap).  q (device,
 * read) and rhs (device, written) are [nvar][N] as for bub_rhs_stage, and the
 * result is bitwise that of bub_rhs_stage on a context of the same problem.  err
 * (device int64[3], may be NULL) receives the device error word (code, first
 * failing cell or -1, failing bin or -1) after the call's kernels.
 * BUB_ENOMEM if the problem's buffers, 11520 + 8*(ndim+6)*N bytes, exceed the
 * static array (2D grids up to 723^2 cells fit, 3D up to 77^3); the argument
 * errors of bub_ctx_create and
 * bub_rhs_stage.  Every call on one GPU uses that GPU's array: calls whose work
 * overlaps on one GPU (other streams, other threads) race and must be ordered
 * by the caller. */
#define BUB_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int bub_rhs_stage_noalloc(const bub_grid *grid, const bub_liquid *liq, const bub_gas *gas, const bub_bins *bins,
                          const bub_opts *opts, const double *q, double *rhs, int64_t *err, void *stream);

/* One-way planar acoustic source (Sec. 2: forcing of the mass, momentum and
 * energy equations on a source plane; the Sec. 5.1 set-ups are driven this
 * way).  The plane is normal to axis `dir` (< ndim) at coordinate x (cell i has
 * its centre at (i + 1/2) dx[dir]); sign = +1 emits toward +dir, -1 toward
 * -dir.  The emitted pressure wave is amp sin(2 pi freq (t - t0)) for t0 <= t <=
 * t0 + ncycles/freq (ncycles = 0: from t0 on), delayed by the travel time from
 * the plane, with nothing emitted upstream.  Forcing, about the reference
 * liquid state (c0 = sqrt(gamma (p0 + pi_inf) / rho0)): S_p = c0 A(t) g(s),
 * S_rho = S_p / c0^2, S_m = sign S_p / c0 along dir, S_E = (1 - alpha) S_p /
 * (gamma - 1) + u.S_m - |u|^2 S_rho / 2, with g the normal pdf of standard
 * deviation `width` (cut at 6 widths) of the distance s from the plane, and A
 * the sine with its amplitude raised by exp((2 pi freq width / c0)^2 / 2),
 * the factor the Gaussian's smoothing takes off it.  RK stages evaluate the
 * source at the time of their input state (t, t + dt, t + dt/2). */
typedef struct { int dir; int sign; double x, width, amp, freq, t0, ncycles; } bub_source;

/* Set (src non-NULL) or clear (NULL) the context's source.  BUB_EINVAL if dir >=
 * ndim, sign is not +-1, width <= 0, freq <= 0, ncycles < 0 or amp is not
 * finite.  The source is added by a pass after each stage kernel (so the
 * stages take a separate primitive pass while one is set). */
int bub_set_source(bub_ctx *ctx, const bub_source *src);

/* The context's clock: the time of the state.  Every RK step advances it by
 * its dt on the device; bub_set_time sets it (ordered on `stream`), and
 * bub_get_time reads it (waits for the device).  A new context starts at 0.
 * bub_rhs_stage evaluates the source at the clock's time. */
int bub_set_time(bub_ctx *ctx, double t, void *stream);
int bub_get_time(bub_ctx *ctx, double *t);

/* nsteps calls of bub_rk3_step in one (same arguments; dt_dev receives the last
 * step's dt).  Results are bitwise those of nsteps separate calls.  In unsplit
 * mode on grids of 2^19 cells or more, the last stage of each step but the
 * final one also computes the primitives and wave speeds of the state it
 * writes, so later steps start without a primitive pass of their own.
 * BUB_EINVAL for nsteps < 0 or the argument errors of bub_rk3_step. */
int bub_rk3_steps(bub_ctx *ctx, double *q, double *work, int nsteps, double dt, double *dt_dev, void *stream);

/* Per-cell diagnostics out[8][N] (device): n, alpha, M3 = mean(R^3),
 * M2d = mean(R^2 Rdot), Mp = mean(R^3 p_bw), Mk = mean(R^3 Rdot^2), the mixture
 * pressure of eq. e:pressure and the liquid pressure p_l.  Means are the bin
 * quadrature sum_i w_i (.)_i. */
int bub_moments(bub_ctx *ctx, const double *q, double *out, void *stream);

/* Bubble half of the Strang splitting (Sec. 3), in place on q: every (cell, bin)
 * advances (R, Rdot) over `tau` by the Keller--Miksis equation with the cell's
 * p_l, rho_l and c frozen at entry, using adaptive embedded SSP-RK3 / Heun-RK2
 * sub-steps (relative error of R and Rdot below opts.sub_rtol, Rdot floored at
 * 1e-3 sqrt(p0/rho0); step factor 0.9 (rtol/err)^(1/3) clamped to [1/4, 4],
 * first sub-step = tau; at most opts.max_substeps attempts, else BUB_ESUBSTEP on
 * the error word).  n is held fixed: (nR)_i = n R_i, (nRdot)_i = n Rdot_i, and
 * alpha is rescaled by mean(R^3)_new / mean(R^3)_old.  tau > 0 (seconds).
 * nsub (device int32 [nb][N], may be NULL) receives the accepted sub-step count
 * of every (cell, bin).  Valid in either bubble mode. */
int bub_bubble_advance(bub_ctx *ctx, double *q, double tau, int32_t *nsub, void *stream);

/* Sub-step counts of split-mode steps (diagnostics of the adaptive bubble
 * sub-steps of Sec. 3).  While set, every bub_rk3_step of this context in split
 * mode writes the accepted sub-step count of each (cell, bin) of its first and
 * of its second bubble half-step into nsub[2][nb][N] (device int32, caller-owned,
 * valid until the steps that use it have finished); NULL stops the recording.
 * Results of the steps do not change. */
int bub_substep_counts(bub_ctx *ctx, int32_t *nsub);

/* ---- Volume-averaged (Euler--Lagrange) variant, Sec. 2.1 --------------------
 * Needs a 3D context with equal spacing in all directions; its bins are not
 * used.  Liquid state ql[5][N] = rho_l, rho_l u, rho_l v, rho_l w, E_l (device)
 * with E_l = (p_l + gamma pi_inf)/(gamma-1) + rho_l |u|^2 / 2.  Bubbles are a
 * device structure-of-arrays bubbles[8][nbub] = x, y, z, R0, R, Rdot, p_g0,
 * h_sub (h_sub: last sub-step, carried between calls; 0 = none yet).  Bubbles
 * are fixed in space (Sec. 2.1).  alpha_D[2][N] (device) holds the smeared void
 * fraction alpha = sum V_n delta_n and its rate D = sum 4 pi R_n^2 Rdot_n delta_n,
 * delta the Gaussian of eq. kernel3D with width h = max(dx, R_n) truncated at
 * 3h (eq. model_inequality and the width rule after it), evaluated at cell
 * centres; cells beyond a reflective wall are skipped, periodic ones wrap. */

/* Bytes of the `work` buffer bub_lagrangian_step needs for nbub bubbles. */
int bub_lagrangian_layout(const bub_ctx *ctx, int64_t nbub, size_t *work_bytes);

/* Bubble records at rest at their equilibrium radius from xyzr0[4][nbub] =
 * x, y, z, R0 (device): R = R0, Rdot = 0, p_g0 = p0 + 2 sigma/R0 - pv, h_sub = 0. */
int bub_lagrangian_bubbles(bub_ctx *ctx, const double *xyzr0, double *bubbles, int64_t nbub, void *stream);

/* Liquid conserved state from primitives prim[5][N] = rho_l, u, v, w, p_l (device). */
int bub_lagrangian_init(bub_ctx *ctx, const double *prim, double *ql, void *stream);

/* alpha_D <- smear of the bubbles (FP64 atomic adds: the summation order, and so
 * the last bits, may differ between runs). */
int bub_lagrangian_smear(bub_ctx *ctx, const double *bubbles, int64_t nbub, double *alpha_D, void *stream);

/* Forcing of each bubble, out[3][nbub] (device): kernel-weighted liquid pressure
 * sum(delta p_l)/sum(delta) over the support, and rho_l, c of the host cell. */
int bub_lagrangian_gather(bub_ctx *ctx, const double *ql, const double *bubbles, int64_t nbub, double *out,
                          void *stream);

/* Liquid right-hand side (Sec. 2.1 liquid equations, inviscid) for frozen
 * alpha_D: WENO5 + HLLC fluxes of the stiffened-gas liquid plus the sources
 * rho_l D/(1-alpha), rho_l u D/(1-alpha) - alpha grad p_l/(1-alpha),
 * E_l D/(1-alpha) - alpha div(p_l u)/(1-alpha), with grad p_l and div(p_l u)
 * from face averages of the reconstructed states.  rhs[5][N] (device). */
int bub_lagrangian_rhs(bub_ctx *ctx, const double *ql, const double *alpha_D, double *rhs, void *stream);

/* One Strang-split step (lagrangian_step): bubbles over dt/2 (Keller--Miksis per
 * bubble with adaptive Dormand--Prince 5(4), relative tolerance opts.sub_rtol,
 * forcing gathered at the start and frozen), smear, liquid SSP-RK3 over dt with
 * alpha_D frozen, bubbles over dt/2, smear.  dt <= 0: CFL step of the liquid.
 * work: device buffer of bub_lagrangian_layout bytes.  dt_dev (device, may be
 * NULL) receives the step; nsub (device int32 [nbub], may be NULL) the accepted
 * sub-steps of each bubble over the step. */
int bub_lagrangian_step(bub_ctx *ctx, double *ql, double *bubbles, int64_t nbub, double *alpha_D, double *work,
                        double dt, double *dt_dev, int32_t *nsub, void *stream);

/* nsteps Lagrangian steps in one call (same arguments; dt_dev receives the
 * last step's dt, nsub the last step's sub-step counts).  A step's closing
 * smear is overwritten by the next step's smear before anything reads it (the
 * bubbles' half-step gathers the liquid alone), so only the last step makes
 * it: ql and the bubbles are those of nsteps separate calls, up to the order
 * of the smears' atomic adds.  The last liquid stage of each step but the
 * final one also computes the primitives and wave speeds of the state it
 * writes, so later steps start without a primitive pass of their own.
 * BUB_EINVAL for nsteps < 0 or the argument errors of bub_lagrangian_step. */
int bub_lagrangian_steps(bub_ctx *ctx, double *ql, double *bubbles, int64_t nbub, double *alpha_D, double *work,
                         int nsteps, double dt, double *dt_dev, int32_t *nsub, void *stream);

/* ---- Batches: many resident problems advanced together ----
 * A batch holds up to max_cases problems (contexts of any dimensionality, bin
 * count, size and bubble mode, all of the batch's precision) with their state q
 * and work buffer (caller-owned device memory, as for bub_rk3_step).  Every
 * step of a member is a CFL-limited SSP-RK3 step with its own step size, and a
 * member's result is bitwise the one bub_rk3_step gives it alone, whatever the
 * other members are.  Two ways to advance the members:
 *
 *  * bub_batch_run: a chunk of steps for the members that still have steps to
 *    take.  Members are added with the number of steps they need; completion is
 *    reported by bub_batch_poll from flags in pinned host memory.  The chunk is
 *    stepped as in the lanes form.  (The library also holds a grouped form of
 *    the chunk -- every phase of a step one kernel launch per kernel class over
 *    a device table of the members -- which is switched off in this build: on
 *    the GPU it has corrupted member states, for a cause not yet found.)
 *  * bub_batch_step (lanes): each member's bub_rk3_step, dealt largest first
 *    over a few internal streams (default priority) so that small problems'
 *    kernels overlap.
 *
 * Members keep their own error word (bub_last_error or bub_error_copy on the
 * member's context).  A context may be in one batch slot at a time and must not
 * be destroyed, nor its buffers freed, while it is a member or while a step
 * that included it may still be running.  All calls on one batch must be made
 * from one thread with one stream.  This replaces the void* batch of a plain
 * pointer-and-size interface; the call names and roles are kept. */
typedef struct bub_batch bub_batch;

/* hbm_budget: device bytes the members may hold together (state, work and the
 * context's buffers of each; 0 = no budget); bub_batch_add refuses a member
 * that does not fit.  max_cases in 1..256.  BUB_ENOMEM if the batch's device
 * table or its pinned flags cannot be allocated, BUB_EHIP if its internal
 * streams or events cannot be created. */
int bub_batch_create(int precision, int max_cases, size_t hbm_budget, bub_batch **out);
/* Waits for the device, then releases the batch's streams, graphs, table and flags. */
int bub_batch_destroy(bub_batch *batch);

/* Add a member that needs `steps` more steps from bub_batch_run (0: open-ended,
 * stepped by every run and never reported done); *slot receives its handle.
 * BUB_ENOMEM if its bytes (3 state copies + bub_ctx_buffer_bytes) exceed what
 * the budget has left; BUB_EINVAL if the batch is full, steps < 0, the precision
 * differs, the context is already a member, or q and work overlap.  A member
 * whose (ndim, nb) class was autotuned gets that class's stage tile shape. */
int bub_batch_add(bub_batch *batch, bub_ctx *ctx, double *q, double *work, int steps, int *slot);
/* Remove a member (its bytes return to the budget).  Its buffers must stay
 * valid until the work already enqueued for it has finished. */
int bub_batch_remove(bub_batch *batch, int slot);

/* Advance every member that still has steps to take (and every open-ended
 * one) by n = min(max_steps, fewest steps left among them) steps, ordered on
 * `stream` (no host synchronisation; the members' steps run on the batch's
 * lanes between a fork from and a join back into `stream`).  *steps_taken (may
 * be NULL) receives n (0 when nothing is left).  Members that reach their last
 * step get a completion flag written on `stream` after the chunk. */
int bub_batch_run(bub_batch *batch, int max_steps, int *steps_taken, void *stream);
/* Slots whose last step has completed on the device since the last poll
 * (read from the pinned flags, no synchronisation).  done_slots: host array of
 * max_cases entries; *ndone receives how many were written.  A reported member
 * stays in its slot until removed and is not stepped again. */
int bub_batch_poll(bub_batch *batch, int *done_slots, int *ndone);
/* Steps a member still has to take in bub_batch_run (-1 for an open-ended one). */
int bub_batch_remaining(const bub_batch *batch, int slot, int *steps);

/* Lanes form: nsteps steps of every member, ordered on `stream` (no host
 * synchronisation).  The internal streams start after the work already queued
 * on `stream`, and `stream` continues only after all of them. */
int bub_batch_step(bub_batch *batch, int nsteps, void *stream);

/* Number of internal streams ("lanes", 1..16, default 4) the members are dealt
 * over.  Kernels of different lanes run concurrently only as far as the
 * process has hardware queues (HIP's GPU_MAX_HW_QUEUES, 4 by default), so more
 * lanes pay only with more queues.  BUB_EINVAL outside 1..16. */
int bub_batch_lanes(bub_batch *batch, int lanes);

/* Graph mode (on by default).  Lanes form: each member's step is captured once
 * as a HIP graph (its kernels only) and replayed with one graph launch per
 * step, which cuts the host's launch work about tenfold; a member is captured
 * again when its tile shape or bin grouping changes, and profiled members
 * launch directly.  enable = 0 launches every kernel directly.  Results are
 * the same either way. */
int bub_batch_graphs(bub_batch *batch, int enable);

/* Members, total cells and total cell-bins of the current members. */
int bub_batch_info(const bub_batch *batch, int *ncases, int64_t *cells, int64_t *cell_bins);

/* Autotuner of the stage kernel's tile shape per (ndim, nb) class: for every
 * member whose class has no tuned shape yet, bub_autotune on that member (its
 * work buffer receives right-hand sides; its state is not changed) picks the
 * fastest shape, which then applies to every member of the class, present and
 * later.  *classes (may be NULL) receives the number of tuned classes.
 * Synchronises `stream`; results do not depend on the tile shape. */
int bub_batch_autotune(bub_batch *batch, int reps, int *classes, void *stream);

/* Tile-shape cache file of the class autotuner (NULL or "": none): a class
 * found there takes the cached shape without timing, a class tuned here is
 * appended (bub_autotune_cached). */
int bub_batch_tune_cache(bub_batch *batch, const char *cache_path);

/* Synchronises `stream`, then reports and clears the sticky device error word:
 * *code (BUB_OK or a device BUB_E* code), *cell (first failing cell or -1),
 * *bin (failing bin or -1).  Any output pointer may be NULL. */
int bub_last_error(bub_ctx *ctx, int *code, int64_t *cell, int *bin, void *stream);

/* Non-blocking form of bub_last_error for callers that must not synchronise:
 * enqueues on `stream` a copy of the error word into dst (device-accessible
 * int64 [3]: code, first failing cell or -1, failing bin or -1) and returns.
 * The word is not cleared. */
int bub_error_copy(const bub_ctx *ctx, int64_t *dst, void *stream);

/* Human-readable name of a BUB_* code (static string). */
const char *bub_strerror(int code);

/* Tile shapes of the fused stage kernel.  Each dimensionality has a fixed list
 * of compiled shapes (tile extent tx*ty*tz cells, `block` threads); a context
 * starts on shape 0.  Results do not depend on the shape (each face flux is
 * computed by the same arithmetic whichever tile owns it); only speed does.
 * bub_tile_info: shape idx of this context's dimensionality (host outputs).
 * bub_tile_set / bub_tile_get: select / query the shape used by later calls. */
int bub_tile_count(const bub_ctx *ctx, int *count);
int bub_tile_info(const bub_ctx *ctx, int idx, int *tx, int *ty, int *tz, int *block);
int bub_tile_set(bub_ctx *ctx, int idx);
int bub_tile_get(const bub_ctx *ctx, int *idx);

/* Bin groups of the fused stage kernel: `groups` workgroups share each tile,
 * each taking a contiguous range of bins (the mixture faces are computed by
 * every group and written by the first).  0 (the default) chooses per launch:
 * one group when the grid has at least 1024 tiles, else enough groups to give
 * about 1024 workgroups, with at least two bins per group.  Results do not
 * depend on the grouping; only the latency of small problems does.  BUB_EINVAL
 * for groups < 0; values above nb act as nb. */
int bub_bin_groups(bub_ctx *ctx, int groups);

/* Autotuner: times `reps` launches of the fused stage kernel (right-hand-side
 * form) for every tile shape on the caller's state q (device, read) with
 * `scratch` (device, state_bytes, overwritten) as output, selects the fastest
 * for this context and returns it in *best (may be NULL).  ms_out (host,
 * bub_tile_count entries, may be NULL) receives the mean time per launch of
 * each shape.  Synchronises `stream`. */
int bub_autotune(bub_ctx *ctx, const double *q, double *scratch, int reps, double *ms_out, int *best,
                 void *stream);

/* The autotuner with a cache of its choices that persists across processes:
 * a text file (created on the first store) of lines
 * "<arch> <ndim> <nb> <precision> <size class> <tile>", keyed by the GPU's
 * architecture name (e.g. gfx950), the context's dimensionality, bin count
 * and precision, and floor(log2 N).  With an entry for the context's key the
 * context takes that tile shape at once (*hit = 1; no launch, no
 * synchronisation, q and scratch unused); otherwise bub_autotune runs and its
 * choice is appended to the file (*hit = 0).  Lines that do not parse or name
 * no valid shape are ignored; the last matching line wins.  best and hit may
 * be NULL.  BUB_EINVAL if the file cannot be appended to. */
int bub_autotune_cached(bub_ctx *ctx, const char *cache_path, const double *q, double *scratch, int reps,
                        int *best, int *hit, void *stream);

/* Kernel timing for benchmarks.  bub_profile(ctx, 1) starts recording a HIP
 * event pair around every kernel the context launches afterwards (on the
 * stream of that call), bub_profile(ctx, 0) stops recording and discards
 * nothing.  bub_profile_read synchronises the device, then returns the summed
 * elapsed time in milliseconds and the launch count of one kernel kind
 * (BUB_K_STAGE: the fused RK-stage kernel; BUB_K_PRIM: the primitive/moment
 * pass; BUB_K_OTHER: everything else) and clears that record.  At most 65536
 * launches are recorded between reads; later launches are not timed. */
enum { BUB_K_STAGE = 0, BUB_K_PRIM = 1, BUB_K_OTHER = 2 };
int bub_profile(bub_ctx *ctx, int enable);
int bub_profile_read(bub_ctx *ctx, int kind, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* BUBBLY_H */
