/*
 * Plain FP64 CPU oracle of the phase-averaged bubbly-flow hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the
 * smoke check and the CPU-baseline leg of the benchmark can check the GPU
 * path against a slow, obviously correct implementation written from the
 * paper.  Nothing in the product path may link, load or call it.
 *
 * It shares no code, header, table or constant generator with the GPU
 * library: every formula below is written again here, in the order the
 * paper (and the readings listed in the design notes) state it.
 *
 * Units are SI.  State arrays are structure-of-arrays [var][z][y][x], x
 * fastest.  Conserved slots (nvar = ndim + 3 + 2 nb):
 *   rho, rho*u_1..ndim, E, alpha, (n R)_1..nb, (n Rdot)_1..nb
 * (mixture conservation laws, Sec. 2 eq. euler_transport; void fraction
 * and bin transport, Sec. 2.2 eqs. e:alpha and the bin-variable equation).
 * With transfer contents (contents = 1) nvar = ndim + 3 + 4 nb: the slots
 * above, then (n p_b)_1..nb and (n m_v)_1..nb (Sec. 2.2 lists p_b and m_v
 * among the bin variables).
 *
 * Parity status per function is given in the header comment of oracle.c.
 */
#ifndef BUBBLY_ORACLE_H
#define BUBBLY_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int ndim;            /* 1, 2 or 3 */
    int n[3];            /* cells per direction, unused directions are 1 */
    double dx[3];        /* spacing per direction (m) */
    int bc[3][2];        /* 0 periodic, 1 reflective, 2 non-reflective, per direction low/high */
    double gamma, pi_inf, rho0, p0;   /* stiffened-gas liquid */
    double kappa, sigma, mu, pv;      /* polytropic gas, surface tension, viscosity, vapour */
    int nb;              /* bins (odd) */
    double r0_median, sigma_ln;       /* lognormal equilibrium-radius distribution */
    double cfl;
    int split;           /* 0: sources inside RK3; 1: Strang-split adaptive bubble sub-steps */
    double sub_rtol;     /* relative tolerance of the bubble sub-stepper */
    int max_substeps;
    int viscous;         /* 1: the liquid's viscous stress (eq. stressTensor) in the mixture fluxes */
    /* One-way planar acoustic source (Sec. 2, source-term forcing; Sec. 5.1 set-ups). */
    double t;            /* time of the state handed in (the source waveform's clock) */
    int src_on;          /* 1: source active */
    int src_dir;         /* axis of the plane's normal (0, 1, 2) */
    int src_sign;        /* +1: the wave travels toward +axis, -1: toward -axis */
    double src_x;        /* plane position along the axis; cell i has its centre at (i + 1/2) dx */
    double src_width;    /* standard deviation of the Gaussian support (m) */
    double src_amp;      /* pressure amplitude of the emitted wave (Pa) */
    double src_freq;     /* frequency (Hz) */
    double src_t0;       /* start time of the sine */
    double src_ncyc;     /* cycles emitted (0: continuous) */
    /* Bubble contents (Sec. 2).  0: polytropic gas, p_b = p_g0 (R0/R)^(3 kappa).  1: gas and vapour
     * with heat and vapour transfer at the wall through constant transfer coefficients (the reduced
     * model the paper adopts: eq. massVaporRate and the contents-pressure equation after it); the
     * state then carries (n p_b)_i and (n m_v)_i per bin as well. */
    int contents;
    double gam_b;        /* specific-heat ratio of the contents */
    double Rg, Rv;       /* gas constants of the non-condensable gas and of the vapour (J/(kg K)) */
    double T0;           /* liquid temperature, which the bubble wall keeps (K) */
    double k_b;          /* thermal conductivity of the contents (W/(m K)) */
    double D_v;          /* binary diffusion coefficient of vapour in the gas (m^2/s) */
    double beta_T;       /* heat transfer coefficient: dT/dr at the wall = beta_T (T0 - Tbar) / R */
    double beta_c;       /* mass transfer coefficient: dchi/dr at the wall = beta_c (chi_w - chibar) / R */
} orc_problem;

/* Bins: ln(R0/R_med) on [-3 sigma, 3 sigma], composite Simpson weights of the
 * normal pdf, normalised to sum 1 (Sec. 2.2, log-normal bins + Simpson). */
int orc_bins(int nb, double r0_median, double sigma_ln, double *r0, double *w);

/* Conserved state from primitives prim[ndim+3][N] = rho_l, u.., p_l, alpha,
 * with every bubble at its equilibrium radius and at rest. */
int orc_init_state(const orc_problem *pb, const double *prim, double *q);

/* Per-cell diagnostics out[8][N]: n, alpha, M3, M2d, Mp, Mk, p_mix, p_l. */
int orc_moments(const orc_problem *pb, const double *q, double *out);

/* Right-hand side L(q) of the semi-discrete system (Sec. 3), acoustic source at time pb->t. */
int orc_rhs(const orc_problem *pb, const double *q, double *rhs);

/* L(q) at k listed cells only; out[k][nvar] (cell-major). */
int orc_rhs_cells(const orc_problem *pb, const double *q, const int64_t *cells, int64_t k, double *out);

/* Same as orc_rhs but with the bubble source terms left out (split mode flux part). */
int orc_rhs_flux_only(const orc_problem *pb, const double *q, double *rhs);

/* CFL time step: cfl * min over cells and directions of dx_d / (|u_d| + c). */
double orc_cfl_dt(const orc_problem *pb, const double *q);

/* One SSP-RK3 step in place from time pb->t (the stages see the source at t, t + dt and
 * t + dt/2).  dt <= 0 selects the CFL step.  Returns the step used in *dt_used.  With
 * pb->split = 1 the step is Strang-split. */
int orc_rk3_step(const orc_problem *pb, double *q, double dt, double *dt_used);

/* Adaptive bubble half-step of split mode on the whole grid (exposed for tests).
 * nsub_out (may be NULL) receives per-(cell,bin) accepted sub-step counts [nb][N]. */
int orc_bubble_advance(const orc_problem *pb, double *q, double dt, int32_t *nsub_out);

/* Pressure amplitude A(t) the acoustic source emits at time t (0 outside its burst). */
double orc_source_amplitude(const orc_problem *pb, double t);

/* OpenMP threads used by the parallel loops (1 without OpenMP). */
int orc_num_threads(void);

/* Threads of the oracle's later parallel loops (n > 0). */
void orc_set_threads(int n);

/* ---- scalar building blocks, exposed for the pins ---- */

/* Keller--Miksis wall acceleration with polytropic contents (Sec. 2 eq. keller_miksis). */
double orc_km_rddot(const orc_problem *pb, double R, double Rdot, double R0, double pg0,
                    double p_inf, double rho, double c);

/* Keller--Miksis wall acceleration for contents of pressure p_b changing at the rate pdot_b
 * (Sec. 2 eq. keller_miksis with p_bw from p_b). */
double orc_km_rddot_pb(const orc_problem *pb, double R, double Rdot, double p_b, double pdot_b,
                       double p_inf, double rho, double c);

/* Transfer contents of one bubble (gas mass mg, radius R, wall velocity Rdot, pressure p_b, vapour
 * mass m_v): the rates dp_b/dt and dm_v/dt (Sec. 2, eq. massVaporRate and the contents-pressure
 * equation).  The bin's equilibrium: p_b = p0 + 2 sigma/R0, m_v = p_v V0/(R_v T0),
 * mg = (p_b - p_v) V0/(R_g T0) with V0 = 4/3 pi R0^3. */
void orc_contents_rates(const orc_problem *pb, double R, double Rdot, double p_b, double m_v, double mg,
                        double *pdot_b, double *mdot_v);

/* WENO5-JS value at the right face of the centre cell from v[0..4] = cells i-2..i+2. */
double orc_weno5(const double *v);

/* HLLC flux at a face from left/right reconstructed primitive vectors
 * W = [rho, u_1..ndim, p_l, alpha, n, B, R_1..nb, Rdot_1..nb] (length nW).
 * dir is the face normal.  F has nvar entries in conserved-slot order. */
int orc_hllc(const orc_problem *pb, int dir, const double *WL, const double *WR, double *F);

/* Single-bubble Keller--Miksis integration with adaptive Dormand--Prince 5(4).
 * y = (R, Rdot) at t=0.  Samples R, Rdot at the nt increasing times t_out.
 * If r_stop > 0 the run ends when R first reaches r_stop; the crossing time is
 * returned in *t_stop (else *t_stop = -1).  Returns the accepted step count. */
int64_t orc_km_integrate(const orc_problem *pb, double R0, double pg0, double p_inf, double rho,
                         double c, double R_init, double Rdot_init, double rtol, double atol_r,
                         double atol_v, int nt, const double *t_out, double *R_out, double *V_out,
                         double r_stop, double *t_stop);

/* One Dormand--Prince 5(4) step of the single-bubble KM system from y = (R, Rdot). */
void orc_km_dp54_step(const orc_problem *pb, double R0, double pg0, double p_inf, double rho, double c,
                      const double *y, double h, double *y5, double *y4);

/* ---- volume-averaged (Euler--Lagrange) variant, Sec. 2.1 ---- */

/* Three-dimensional only.  Liquid conserved state ql[5][N] = rho_l, rho_l u,
 * rho_l v, rho_l w, E_l (liquid-phase variables of Sec. 2.1).  Bubbles are
 * structure-of-arrays bub[8][nbub] = x, y, z, R0, R, Rdot, pg0, h_sub, where
 * h_sub is the last accepted sub-step (carried from one half-step to the next). */

/* Truncated Gaussian regularisation kernel, eq. kernel3D. */
double orc_el_kernel(double d, double h);

/* Void fraction alpha = sum V_n delta and its material rate
 * dalpha = sum 4 pi R_n^2 Rdot_n delta, at cell centres. */
int orc_el_smear(const orc_problem *pb, const double *bub, int64_t nbub, double *alpha, double *dalpha);

/* Kernel-weighted liquid pressure around each bubble (normalised), and the
 * liquid density and sound speed of the host cell. */
int orc_el_gather(const orc_problem *pb, const double *ql, const double *bub, int64_t nbub,
                  double *p_inf, double *rho_l, double *c_l);

/* Liquid right-hand side with the bubble source terms for frozen alpha, dalpha. */
int orc_el_rhs(const orc_problem *pb, const double *ql, const double *alpha, const double *dalpha,
               double *rhs);

/* One Strang-split step: bubbles dt/2 (adaptive DP5(4)), smear, liquid SSP-RK3
 * over dt with alpha and dalpha frozen, bubbles dt/2, smear.  dt <= 0 selects
 * the CFL step of the liquid; the step used is returned in *dt_used.
 * nsub_out (may be NULL) receives accepted sub-steps per bubble (both halves). */
int orc_el_step(const orc_problem *pb, double *ql, double *bub, int64_t nbub, double dt,
                double *alpha, double *dalpha, int32_t *nsub_out, double *dt_used);

#ifdef __cplusplus
}
#endif
#endif
