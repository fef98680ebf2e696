/*
 * Plain FP64 CPU oracle of the phase-averaged bubbly-flow hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  The product path never links or calls
 * it, and it shares no code with the GPU library.
 *
 * Written from the paper, step by step, in plain C99 with IEEE double
 * arithmetic (no fast-math, no FMA contraction on the default x86-64 target),
 * OpenMP only over independent cells or faces (deterministic).
 *
 * What each part follows, and what pins it (tests/test_oracle_*.py):
 *   bins            Sec. 2.2 (log-normal PDF, Simpson's rule) -- pinned by
 *                   Simpson pattern/exactness and lognormal moments.
 *   primitives      Sec. 2 (mixture closures), eq. eos_liquid, eq. e:ndf,
 *                   eq. e:pressure -- pinned by equilibrium p = p0, n recovery
 *                   and the low-frequency sound speed of the bubbly mixture
 *                   (linear part of the bin moment of R^3 p_bw, the alpha
 *                   source).  The R^3 Rdot^2 moment (quadratic in Rdot) is
 *                   parity unpinned.
 *   Keller--Miksis  eq. keller_miksis with polytropic contents -- pinned by the
 *                   Rayleigh collapse time, the linearised oscillator and
 *                   equilibrium.  Its terms of second and higher order in
 *                   Rdot/c are parity unpinned.
 *   WENO5           Sec. 3 (fifth-order WENO) -- pinned by quadratic exactness,
 *                   5th-order convergence, mirror symmetry.
 *   HLLC            Sec. 3 (HLLC Riemann solver) -- pinned by consistency,
 *                   contact at rest, the exact Sod solution, passive fluxes
 *                   = upwind specific value times mass flux, and a trace void
 *                   fraction following the exact contact.
 *   viscous stress  eq. stressTensor in eq. euler_transport (optional) --
 *                   pinned by the analytic divergence of T and T.u for a 2D
 *                   field at second order, and the decay of a shear wave.
 *   semi-discrete   Sec. 3 eq. (finite-volume form) -- pinned by free-stream
 *                   preservation, discrete conservation, symmetry, 1D = 2D.
 *   SSP-RK3         Sec. 3 (third-order TVD RK) -- pinned by order >= 2.8 on the
 *                   0D uniform-state reduction.
 *   split sub-steps Sec. 3 (Strang splitting, RK3/RK2 pair, tolerance 1e-4)
 *                   -- pinned by the Rayleigh time, equilibrium and the
 *                   composition's observed order (2 at a trace void
 *                   fraction; 1 where the void fraction feeds back on p_l,
 *                   which the bin-by-bin sub-steps hold fixed).
 *   transfer        Sec. 2 (gas and vapour contents with constant heat and
 *   contents        mass transfer coefficients, eq. massVaporRate and the
 *                   contents-pressure equation) -- pinned by equilibrium, the
 *                   reduction to the polytropic model without transfer, the
 *                   isothermal limit, the first law with vapour transfer, the
 *                   hand-linearised heat-transfer oscillator at two radii,
 *                   fixed-radius vapour relaxation, and the passive fluxes of
 *                   n p_b and n m_v.  The coefficients are inputs (the paper
 *                   does not give them); the sub-steps' error norm on p_b and
 *                   m_v is parity unpinned.
 *   Lagrangian      Sec. 2.1 (kernel eq. kernel3D, smear, gather) -- pinned by
 *                   the kernel mass lattice sum, uniform gather, bubble at rest;
 *                   its liquid sources by exponential growth under a frozen
 *                   uniform D and the wave speed c_l/sqrt(1-alpha) under a
 *                   frozen uniform alpha.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define NBMAX 64
#define NWMAX (3 + 5 + 4 * NBMAX)
#define NVMAX (3 + 3 + 4 * NBMAX)

typedef struct {
    const orc_problem *pb;
    int nd, nb, nvar, nW;
    int nf;                             /* fields per bin: 2 (R, Rdot) or 4 (and p_b, m_v) */
    int64_t N;
    int iE, iA, iNR, iNV, iNP, iNM;     /* conserved slots */
    int wPL, wA, wN, wB, wR, wV, wP, wM; /* primitive slots */
    double r0[NBMAX], w[NBMAX], pg0[NBMAX];
    double pb0[NBMAX], mv0[NBMAX], mg[NBMAX];  /* transfer contents at equilibrium; gas mass */
} setup_t;

typedef struct {
    double c, rhol, M3, M2d, Mp, Mk, pmix;
} aux_t;

static double sq(double x) { return x * x; }

/* ------------------------------------------------------------------------ */
/* Bins: log-normal distribution of R0, Simpson's rule (Sec. 2.2).          */
/* ------------------------------------------------------------------------ */
int orc_bins(int nb, double rmed, double sig, double *r0, double *w)
{
    if (nb < 1 || nb % 2 == 0 || nb > NBMAX || !(rmed > 0.0)) return -1;
    if (nb == 1) {
        r0[0] = rmed;
        w[0] = 1.0;
        return 0;
    }
    if (!(sig > 0.0)) return -1;
    double h = 6.0 * sig / (nb - 1);
    double sum = 0.0;
    for (int i = 0; i < nb; ++i) {
        double phi = -3.0 * sig + h * i;
        r0[i] = rmed * exp(phi);
        double s = (i == 0 || i == nb - 1) ? 1.0 : ((i % 2) ? 4.0 : 2.0);
        double f = exp(-phi * phi / (2.0 * sig * sig)) / (sig * sqrt(2.0 * ORC_PI));
        w[i] = h / 3.0 * s * f;
        sum += w[i];
    }
    for (int i = 0; i < nb; ++i) w[i] /= sum;
    return 0;
}

static int setup(const orc_problem *pb, setup_t *s)
{
    memset(s, 0, sizeof(*s));
    s->pb = pb;
    if (pb->ndim < 1 || pb->ndim > 3) return -1;
    for (int d = 0; d < 3; ++d) {
        if (pb->n[d] < 1) return -1;
        if (d >= pb->ndim && pb->n[d] != 1) return -1;
        if (d < pb->ndim) {
            if (!(pb->dx[d] > 0.0)) return -1;
            for (int e = 0; e < 2; ++e) {
                if (pb->bc[d][e] < 0 || pb->bc[d][e] > 2) return -1;
                if (pb->bc[d][e] == 1 && pb->n[d] < 3) return -1;
            }
            if (pb->bc[d][0] != pb->bc[d][1] && (pb->bc[d][0] == 0 || pb->bc[d][1] == 0)) return -1;
        }
    }
    if (pb->src_on) {
        if (pb->src_dir < 0 || pb->src_dir >= pb->ndim || (pb->src_sign != 1 && pb->src_sign != -1)) return -1;
        if (!(pb->src_width > 0.0) || !(pb->src_freq > 0.0) || !(pb->src_ncyc >= 0.0) || !isfinite(pb->src_amp))
            return -1;
    }
    if (pb->contents < 0 || pb->contents > 1) return -1;
    if (pb->contents == 1) {
        if (!(pb->gam_b > 1.0) || !(pb->Rg > 0.0) || !(pb->Rv > 0.0) || !(pb->T0 > 0.0) || !(pb->k_b >= 0.0) ||
            !(pb->D_v >= 0.0) || !(pb->beta_T >= 0.0) || !(pb->beta_c >= 0.0) || !(pb->pv >= 0.0) ||
            !(pb->pv < pb->p0))
            return -1;
    }
    s->nd = pb->ndim;
    s->nb = pb->nb;
    s->nf = pb->contents == 1 ? 4 : 2;
    if (orc_bins(pb->nb, pb->r0_median, pb->sigma_ln, s->r0, s->w) != 0) return -1;
    for (int i = 0; i < s->nb; ++i) {
        s->pg0[i] = pb->p0 + 2.0 * pb->sigma / s->r0[i] - pb->pv;
        if (s->nf == 4) {
            /* equilibrium: contents at the Laplace pressure, vapour at its saturation pressure p_v and the
             * liquid temperature T0, the rest non-condensable gas at T0 */
            double V0 = 4.0 * ORC_PI / 3.0 * s->r0[i] * s->r0[i] * s->r0[i];
            s->pb0[i] = pb->p0 + 2.0 * pb->sigma / s->r0[i];
            s->mv0[i] = pb->pv * V0 / (pb->Rv * pb->T0);
            s->mg[i] = (s->pb0[i] - pb->pv) * V0 / (pb->Rg * pb->T0);
        }
    }
    s->nvar = s->nd + 3 + s->nf * s->nb;
    s->nW = s->nd + 5 + s->nf * s->nb;
    s->N = (int64_t)pb->n[0] * pb->n[1] * pb->n[2];
    s->iE = s->nd + 1;
    s->iA = s->nd + 2;
    s->iNR = s->nd + 3;
    s->iNV = s->nd + 3 + s->nb;
    s->iNP = s->nd + 3 + 2 * s->nb;
    s->iNM = s->nd + 3 + 3 * s->nb;
    s->wPL = s->nd + 1;
    s->wA = s->nd + 2;
    s->wN = s->nd + 3;
    s->wB = s->nd + 4;
    s->wR = s->nd + 5;
    s->wV = s->nd + 5 + s->nb;
    s->wP = s->nd + 5 + 2 * s->nb;
    s->wM = s->nd + 5 + 3 * s->nb;
    return 0;
}

static int64_t lin(const orc_problem *pb, int i, int j, int k)
{
    return (int64_t)i + (int64_t)pb->n[0] * ((int64_t)j + (int64_t)pb->n[1] * k);
}

/* Ghost-cell index map along one direction: periodic wrap, mirror for a
 * reflective wall (the normal velocity of the mirrored cell changes sign), or
 * the boundary cell itself for a non-reflective boundary (Sec. 5.1, after
 * Thompson): with every ghost state equal to the boundary cell, the Riemann
 * problem at the boundary face has no jump, so no wave enters from outside --
 * the time derivative of each incoming characteristic at the boundary cell
 * comes from the interior face alone. */
static int map_index(const orc_problem *pb, int dir, int i, int *flip)
{
    int n = pb->n[dir];
    if (i < 0) {
        if (pb->bc[dir][0] == 0) return ((i % n) + n) % n;
        if (pb->bc[dir][0] == 2) return 0;
        *flip = !*flip;
        return -1 - i;
    }
    if (i >= n) {
        if (pb->bc[dir][1] == 0) return i % n;
        if (pb->bc[dir][1] == 2) return n - 1;
        *flip = !*flip;
        return 2 * n - 1 - i;
    }
    return i;
}

/* ------------------------------------------------------------------------ */
/* One-way planar acoustic source (Sec. 2, source-term forcing of the mass,  */
/* momentum and energy equations on a source plane).                         */
/*                                                                          */
/* Written from linear acoustics about the reference liquid state (c0 =      */
/* sqrt(gamma (p0 + pi_inf) / rho0)): forcing the pressure rate with         */
/* S_p = c0 A(t) g(s), the momentum along the emission direction n with      */
/* S_p / c0 and the mass with the isentropic S_p / c0^2 drives only the      */
/* characteristic p' + rho0 c0 (u'.n), so the plane emits                    */
/* p' = A(t - s/c0) (smoothed by g) downstream and nothing upstream, and no  */
/* entropy spot.  s = x - x_s along the axis; g is the normal pdf of         */
/* standard deviation `width`, cut at 6 widths.  A is a sine burst; its      */
/* amplitude is raised by exp((k width)^2 / 2), k = 2 pi f / c0, the factor  */
/* by which the Gaussian's smoothing lowers a sinusoid, so the emitted wave  */
/* has amplitude src_amp.  The energy forcing is the change of E that S_p,   */
/* S_m and S_rho make at fixed alpha:                                        */
/*   S_E = (1 - alpha) S_p / (gamma - 1) + u.S_m - |u|^2 S_rho / 2.          */
/* ------------------------------------------------------------------------ */
static double ref_sound_speed(const orc_problem *pb)
{
    return sqrt(pb->gamma * (pb->p0 + pb->pi_inf) / pb->rho0);
}

double orc_source_amplitude(const orc_problem *pb, double t)
{
    if (!pb->src_on) return 0.0;
    double tau = t - pb->src_t0;
    if (tau < 0.0) return 0.0;
    if (pb->src_ncyc > 0.0 && tau > pb->src_ncyc / pb->src_freq) return 0.0;
    double k = 2.0 * ORC_PI * pb->src_freq / ref_sound_speed(pb);
    return pb->src_amp * exp(0.5 * sq(k * pb->src_width)) * sin(2.0 * ORC_PI * pb->src_freq * tau);
}

/* Spatial support g at the centre of cell index i along the source axis. */
static double source_shape(const orc_problem *pb, int i)
{
    double s = (i + 0.5) * pb->dx[pb->src_dir] - pb->src_x;
    double w = pb->src_width;
    if (fabs(s) > 6.0 * w) return 0.0;
    return exp(-0.5 * sq(s / w)) / (sqrt(2.0 * ORC_PI) * w);
}

/* Adds the source at time t to the right-hand side L (nvar entries) of the cell at
 * coordinates co, whose primitive vector is W. */
static void acoustic_source(const setup_t *s, const double *W, const int co[3], double t, double *L)
{
    const orc_problem *pb = s->pb;
    double g = source_shape(pb, co[pb->src_dir]);
    if (g == 0.0) return;
    double c0 = ref_sound_speed(pb);
    double Sp = c0 * orc_source_amplitude(pb, t) * g;
    double Srho = Sp / (c0 * c0);
    double Sm = pb->src_sign * Sp / c0;
    double u2 = 0.0;
    for (int d = 0; d < s->nd; ++d) u2 += sq(W[1 + d]);
    L[0] += Srho;
    L[1 + pb->src_dir] += Sm;
    L[s->iE] += (1.0 - W[s->wA]) * Sp / (pb->gamma - 1.0) + W[1 + pb->src_dir] * Sm - 0.5 * u2 * Srho;
}

static void gather(const setup_t *s, const double *q, int64_t c, double *qc)
{
    for (int v = 0; v < s->nvar; ++v) qc[v] = q[(int64_t)v * s->N + c];
}

/* ------------------------------------------------------------------------ */
/* Keller--Miksis (eq. keller_miksis), polytropic contents p_b = p_g0 (R0/R)^(3 kappa).
 * The R-ddot part of d(p_bw)/dt (from the viscous term) is moved to the left. */
/* ------------------------------------------------------------------------ */
double orc_km_rddot(const orc_problem *pb, double R, double V, double R0, double pg0,
                    double pinf, double rho, double c)
{
    double pb_ = pg0 * pow(R0 / R, 3.0 * pb->kappa);
    double pbw = pb_ - 4.0 * pb->mu * V / R - 2.0 * pb->sigma / R;
    double dpbw = -3.0 * pb->kappa * pb_ * V / R + 4.0 * pb->mu * V * V / (R * R)
                  + 2.0 * pb->sigma * V / (R * R);
    double num = (1.0 + V / c) * (pbw - pinf) / rho + R * dpbw / (rho * c)
                 - 1.5 * V * V * (1.0 - V / (3.0 * c));
    double den = R * (1.0 - V / c) + 4.0 * pb->mu / (rho * c);
    return num / den;
}

/* Keller--Miksis with the contents' pressure p_b and its rate given (transfer contents). */
double orc_km_rddot_pb(const orc_problem *pb, double R, double V, double p_b, double pdot_b,
                       double pinf, double rho, double c)
{
    double pbw = p_b - 4.0 * pb->mu * V / R - 2.0 * pb->sigma / R;
    double dpbw = pdot_b + 4.0 * pb->mu * V * V / (R * R) + 2.0 * pb->sigma * V / (R * R);
    double num = (1.0 + V / c) * (pbw - pinf) / rho + R * dpbw / (rho * c)
                 - 1.5 * V * V * (1.0 - V / (3.0 * c));
    double den = R * (1.0 - V / c) + 4.0 * pb->mu / (rho * c);
    return num / den;
}

/* ------------------------------------------------------------------------ */
/* Transfer contents (Sec. 2: constant heat and mass transfer coefficients at */
/* the wall, eq. massVaporRate, and the contents-pressure equation).        */
/* The contents are an ideal-gas mixture of gas (fixed mass mg) and vapour  */
/* (mass m) at uniform pressure p; its mean temperature follows from        */
/* p V = (mg Rg + m Rv) Tbar.  The wall stays at the liquid temperature T0  */
/* with the vapour at its saturation pressure p_v there, which fixes the    */
/* wall's vapour mass fraction chi_w and mixture density rho_w.  The wall   */
/* gradients of T and of the vapour mass fraction are the transfer          */
/* coefficients times (wall value - bubble mean) / R.                       */
/* ------------------------------------------------------------------------ */
void orc_contents_rates(const orc_problem *pb, double R, double V, double p, double m, double mg,
                        double *pdot, double *mdot)
{
    double vol = 4.0 * ORC_PI / 3.0 * R * R * R;
    double Tbar = p * vol / (mg * pb->Rg + m * pb->Rv);
    double chibar = m / (m + mg);
    double chiw = pb->pv * pb->Rg / (pb->pv * pb->Rg + (p - pb->pv) * pb->Rv);
    double Rw = chiw * pb->Rv + (1.0 - chiw) * pb->Rg;
    double rhow = p / (Rw * pb->T0);
    double dTdr = pb->beta_T * (pb->T0 - Tbar) / R;
    double dchidr = pb->beta_c * (chiw - chibar) / R;
    double flux = pb->D_v * rhow / (1.0 - chiw) * dchidr;   /* vapour mass into the bubble per wall area */
    *pdot = 3.0 * pb->gam_b / R
            * (-V * p + pb->Rv * pb->T0 * flux + (pb->gam_b - 1.0) / pb->gam_b * pb->k_b * dTdr);
    *mdot = 4.0 * ORC_PI * R * R * flux;
}

/* ------------------------------------------------------------------------ */
/* Conserved -> primitive, bin moments and mixture pressure (Sec. 2, 2.2).  */
/* ------------------------------------------------------------------------ */
static void primitives(const setup_t *s, const double *qc, double *W, aux_t *ax)
{
    const orc_problem *pb = s->pb;
    double rho = qc[0];
    double ke = 0.0;
    W[0] = rho;
    for (int d = 0; d < s->nd; ++d) {
        W[1 + d] = qc[1 + d] / rho;
        ke += 0.5 * rho * W[1 + d] * W[1 + d];
    }
    double E = qc[s->iE];
    double a = qc[s->iA];
    double pl = (pb->gamma - 1.0) * (E - ke) / (1.0 - a) - pb->gamma * pb->pi_inf;
    double rhol = rho / (1.0 - a);
    double c = sqrt(pb->gamma * (pl + pb->pi_inf) / rhol);
    W[s->wPL] = pl;
    W[s->wA] = a;
    double n = 0.0, B = 0.0, M3 = 0.0, M2d = 0.0, Mp = 0.0, Mk = 0.0;
    if (a > 0.0) {
        double sum = 0.0;
        for (int i = 0; i < s->nb; ++i) sum += s->w[i] * pow(qc[s->iNR + i], 3.0);
        n = sqrt(4.0 * ORC_PI / 3.0 * sum / a);
        for (int i = 0; i < s->nb; ++i) {
            double R = qc[s->iNR + i] / n;
            double V = qc[s->iNV + i] / n;
            W[s->wR + i] = R;
            W[s->wV + i] = V;
            double pbub;
            if (s->nf == 4) {
                pbub = qc[s->iNP + i] / n;
                W[s->wP + i] = pbub;
                W[s->wM + i] = qc[s->iNM + i] / n;
            } else {
                pbub = s->pg0[i] * pow(s->r0[i] / R, 3.0 * pb->kappa);
            }
            double pbw = pbub - 4.0 * pb->mu * V / R - 2.0 * pb->sigma / R;
            double R3 = R * R * R;
            M3 += s->w[i] * R3;
            M2d += s->w[i] * R * R * V;
            Mp += s->w[i] * R3 * pbw;
            Mk += s->w[i] * R3 * V * V;
        }
        B = (Mp - rho * Mk) / M3;
    } else {
        for (int i = 0; i < s->nb; ++i) {
            W[s->wR + i] = s->r0[i];
            W[s->wV + i] = 0.0;
            if (s->nf == 4) {
                W[s->wP + i] = s->pb0[i];
                W[s->wM + i] = s->mv0[i];
            }
            M3 += s->w[i] * pow(s->r0[i], 3.0);
        }
    }
    W[s->wN] = n;
    W[s->wB] = B;
    if (ax) {
        ax->c = c;
        ax->rhol = rhol;
        ax->M3 = M3;
        ax->M2d = M2d;
        ax->Mp = Mp;
        ax->Mk = Mk;
        ax->pmix = (1.0 - a) * pl + a * B;
    }
}

/* ------------------------------------------------------------------------ */
/* WENO5-JS (Jiang & Shu 1996): face value at i+1/2 from cells i-2..i+2.    */
/* ------------------------------------------------------------------------ */
double orc_weno5(const double *v)
{
    const double eps = 1e-16;
    double q0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    double q1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
    double b0 = 13.0 / 12.0 * sq(v[0] - 2.0 * v[1] + v[2]) + 0.25 * sq(v[0] - 4.0 * v[1] + 3.0 * v[2]);
    double b1 = 13.0 / 12.0 * sq(v[1] - 2.0 * v[2] + v[3]) + 0.25 * sq(v[1] - v[3]);
    double b2 = 13.0 / 12.0 * sq(v[2] - 2.0 * v[3] + v[4]) + 0.25 * sq(3.0 * v[2] - 4.0 * v[3] + v[4]);
    double a0 = 0.1 / sq(eps + b0);
    double a1 = 0.6 / sq(eps + b1);
    double a2 = 0.3 / sq(eps + b2);
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* ------------------------------------------------------------------------ */
/* HLLC (Toro): Davis wave speeds, contact speed, difference-form star flux. */
/* ------------------------------------------------------------------------ */
typedef struct {
    double rho, u[3], pl, a, n, B, p, E, c;
} face_core_t;

static void face_core(const setup_t *s, const double *W, face_core_t *f)
{
    const orc_problem *pb = s->pb;
    f->rho = W[0];
    f->u[0] = f->u[1] = f->u[2] = 0.0;
    for (int d = 0; d < s->nd; ++d) f->u[d] = W[1 + d];
    f->pl = W[s->wPL];
    f->a = W[s->wA];
    f->n = W[s->wN];
    f->B = W[s->wB];
    f->p = (1.0 - f->a) * f->pl + f->a * f->B;
    f->E = (1.0 - f->a) * (f->pl + pb->gamma * pb->pi_inf) / (pb->gamma - 1.0)
           + 0.5 * f->rho * (f->u[0] * f->u[0] + f->u[1] * f->u[1] + f->u[2] * f->u[2]);
    f->c = sqrt(pb->gamma * (f->pl + pb->pi_inf) * (1.0 - f->a) / f->rho);
}

/* side: 0 = left state, 1 = right state; star: 1 for the star-region flux */
static void hllc_select(const face_core_t *L, const face_core_t *R, int dir, double *SL, double *SR,
                        double *Ss, int *side, int *star)
{
    double uL = L->u[dir], uR = R->u[dir];
    *SL = fmin(uL - L->c, uR - R->c);
    *SR = fmax(uL + L->c, uR + R->c);
    *Ss = (R->p - L->p + L->rho * uL * (*SL - uL) - R->rho * uR * (*SR - uR))
          / (L->rho * (*SL - uL) - R->rho * (*SR - uR));
    if (*SL >= 0.0) { *side = 0; *star = 0; }
    else if (*Ss >= 0.0) { *side = 0; *star = 1; }
    else if (*SR > 0.0) { *side = 1; *star = 1; }
    else { *side = 1; *star = 0; }
}

int orc_hllc(const orc_problem *pb, int dir, const double *WL, const double *WR, double *F)
{
    setup_t s;
    if (setup(pb, &s) != 0) return -1;
    face_core_t L, R;
    face_core(&s, WL, &L);
    face_core(&s, WR, &R);
    double SL, SR, Ss;
    int side, star;
    hllc_select(&L, &R, dir, &SL, &SR, &Ss, &side, &star);
    const face_core_t *K = side ? &R : &L;
    const double *WK = side ? WR : WL;
    double SK = side ? SR : SL;
    double un = K->u[dir];
    F[0] = K->rho * un;
    for (int j = 0; j < s.nd; ++j) F[1 + j] = K->rho * un * K->u[j] + (j == dir ? K->p : 0.0);
    F[s.iE] = (K->E + K->p) * un;
    F[s.iA] = K->a * un;
    for (int i = 0; i < s.nb; ++i) {
        F[s.iNR + i] = K->n * WK[s.wR + i] * un;
        F[s.iNV + i] = K->n * WK[s.wV + i] * un;
        if (s.nf == 4) {
            F[s.iNP + i] = K->n * WK[s.wP + i] * un;
            F[s.iNM + i] = K->n * WK[s.wM + i] * un;
        }
    }
    if (star) {
        double fac = SK * (Ss - un) / (SK - Ss);
        F[0] += fac * K->rho;
        for (int j = 0; j < s.nd; ++j) F[1 + j] += fac * (j == dir ? K->rho * SK : K->rho * K->u[j]);
        F[s.iE] += fac * (K->E + K->p + K->rho * Ss * (SK - un));
        F[s.iA] += fac * K->a;
        for (int i = 0; i < s.nb; ++i) {
            F[s.iNR + i] += fac * K->n * WK[s.wR + i];
            F[s.iNV + i] += fac * K->n * WK[s.wV + i];
            if (s.nf == 4) {
                F[s.iNP + i] += fac * K->n * WK[s.wP + i];
                F[s.iNM + i] += fac * K->n * WK[s.wM + i];
            }
        }
    }
    return 0;
}

/* Face flux from the six cells i-3..i+2 around face i-1/2 (Wst[2] is the left
 * cell, Wst[3] the right cell).  Reconstruction of every primitive on both
 * sides, then the admissibility fallbacks, then HLLC. */
static void face_flux(const setup_t *s, int dir, double (*Wst)[NWMAX], double *F)
{
    const orc_problem *pb = s->pb;
    double WL[NWMAX], WR[NWMAX], v[5];
    for (int k = 0; k < s->nW; ++k) {
        for (int o = 0; o < 5; ++o) v[o] = Wst[o][k];
        WL[k] = orc_weno5(v);
        for (int o = 0; o < 5; ++o) v[o] = Wst[5 - o][k];
        WR[k] = orc_weno5(v);
    }
    /* Core admissibility on both sides; failure -> first order for the whole face. */
    int ok = 1;
    const double *sides[2] = {WL, WR};
    for (int t = 0; t < 2; ++t) {
        const double *Wk = sides[t];
        if (!(Wk[0] > 0.0)) ok = 0;
        if (!(Wk[s->wA] >= 0.0 && Wk[s->wA] < 1.0)) ok = 0;
        if (!(Wk[s->wN] >= 0.0)) ok = 0;
        if (!(Wk[s->wPL] + pb->pi_inf > 0.0)) ok = 0;
    }
    if (!ok) {
        memcpy(WL, Wst[2], sizeof(double) * s->nW);
        memcpy(WR, Wst[3], sizeof(double) * s->nW);
    } else {
        /* Bin radii entering the flux come from the upwind (selected) side only;
         * a non-positive radius there falls back to that side's cell values. */
        face_core_t L, R;
        face_core(s, WL, &L);
        face_core(s, WR, &R);
        double SL, SR, Ss;
        int side, star;
        hllc_select(&L, &R, dir, &SL, &SR, &Ss, &side, &star);
        double *WK = side ? WR : WL;
        const double *Wc = side ? Wst[3] : Wst[2];
        for (int i = 0; i < s->nb; ++i) {
            if (!(WK[s->wR + i] > 0.0)) {
                WK[s->wR + i] = Wc[s->wR + i];
                WK[s->wV + i] = Wc[s->wV + i];
                if (s->nf == 4) {
                    WK[s->wP + i] = Wc[s->wP + i];
                    WK[s->wM + i] = Wc[s->wM + i];
                }
            }
        }
    }
    orc_hllc(pb, dir, WL, WR, F);
}

/* Primitive vector of the cell at (possibly ghost) coordinates, via the BC map. */
static void stencil_prim(const setup_t *s, const double *q, int dir, const int coord[3], int off,
                         double *W)
{
    const orc_problem *pb = s->pb;
    int flip = 0;
    int cc[3] = {coord[0], coord[1], coord[2]};
    cc[dir] = map_index(pb, dir, coord[dir] + off, &flip);
    double qc[NVMAX];
    gather(s, q, lin(pb, cc[0], cc[1], cc[2]), qc);
    primitives(s, qc, W, NULL);
    if (flip) W[1 + dir] = -W[1 + dir];
}

/* ------------------------------------------------------------------------ */
/* Viscous stress of the liquid, eq. stressTensor:                          */
/*   T = mu (grad u + grad u^T - 2/3 (div u) I),                             */
/* carried by the momentum flux as -T and by the energy flux as -T.u        */
/* (eq. euler_transport).  Second-order central differences at the face.    */
/* ------------------------------------------------------------------------ */

/* Velocity of the cell at co + oa e_a (+ ob e_b when b >= 0), through the ghost-cell map: a mirrored
 * coordinate negates the velocity component along that direction. */
static void vel_at(const setup_t *s, const double *q, const int co[3], int a, int oa, int b, int ob, double u[3])
{
    const orc_problem *pb = s->pb;
    int cc[3] = {co[0], co[1], co[2]};
    int fa = 0, fb = 0;
    cc[a] = map_index(pb, a, co[a] + oa, &fa);
    if (b >= 0) cc[b] = map_index(pb, b, co[b] + ob, &fb);
    int64_t c = lin(pb, cc[0], cc[1], cc[2]);
    for (int k = 0; k < 3; ++k) u[k] = k < s->nd ? q[(int64_t)(1 + k) * s->N + c] / q[c] : 0.0;
    if (fa) u[a] = -u[a];
    if (b >= 0 && fb) u[b] = -u[b];
}

/* Adds the viscous flux through face co of direction dir (between the cells co - e_dir and co). */
static void visc_flux(const setup_t *s, const double *q, int dir, const int co[3], double *F)
{
    const orc_problem *pb = s->pb;
    double uL[3], uR[3], g[3][3] = {{0.0}};   /* g[k][e] = d u_k / d x_e at the face */
    vel_at(s, q, co, dir, -1, -1, 0, uL);
    vel_at(s, q, co, dir, 0, -1, 0, uR);
    for (int k = 0; k < s->nd; ++k) g[k][dir] = (uR[k] - uL[k]) / pb->dx[dir];
    for (int e = 0; e < s->nd; ++e) {
        if (e == dir) continue;
        double lp[3], lm[3], rp[3], rm[3];
        vel_at(s, q, co, dir, -1, e, 1, lp);
        vel_at(s, q, co, dir, -1, e, -1, lm);
        vel_at(s, q, co, dir, 0, e, 1, rp);
        vel_at(s, q, co, dir, 0, e, -1, rm);
        /* central difference across e in each of the two cells, averaged */
        for (int k = 0; k < s->nd; ++k)
            g[k][e] = 0.5 * ((lp[k] - lm[k]) / (2.0 * pb->dx[e]) + (rp[k] - rm[k]) / (2.0 * pb->dx[e]));
    }
    double div = 0.0;
    for (int e = 0; e < s->nd; ++e) div += g[e][e];
    double work = 0.0;
    for (int k = 0; k < s->nd; ++k) {
        double T = pb->mu * (g[dir][k] + g[k][dir] - (k == dir ? 2.0 / 3.0 * div : 0.0));
        F[1 + k] -= T;
        work += T * 0.5 * (uL[k] + uR[k]);
    }
    F[s->iE] -= work;
}

static void cell_sources(const setup_t *s, const double *W, const aux_t *ax, double *L)
{
    const orc_problem *pb = s->pb;
    double a = W[s->wA];
    if (!(a > 0.0)) return;
    double n = W[s->wN];
    L[s->iA] += 3.0 * a * ax->M2d / ax->M3;
    for (int i = 0; i < s->nb; ++i) {
        double R = W[s->wR + i], V = W[s->wV + i];
        L[s->iNR + i] += n * V;
        if (s->nf == 4) {
            double pdot, mdot;
            orc_contents_rates(pb, R, V, W[s->wP + i], W[s->wM + i], s->mg[i], &pdot, &mdot);
            L[s->iNV + i] += n * orc_km_rddot_pb(pb, R, V, W[s->wP + i], pdot, W[s->wPL], ax->rhol, ax->c);
            L[s->iNP + i] += n * pdot;
            L[s->iNM + i] += n * mdot;
        } else {
            L[s->iNV + i] += n * orc_km_rddot(pb, R, V, s->r0[i], s->pg0[i], W[s->wPL], ax->rhol, ax->c);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Whole-grid right-hand side.                                              */
/* ------------------------------------------------------------------------ */
static int rhs_impl(const orc_problem *pb, const double *q, double *rhs, int with_sources, double t)
{
    setup_t s;
    if (setup(pb, &s) != 0) return -1;
    const int64_t N = s.N;
    const int nW = s.nW, nvar = s.nvar;
    double *W = (double *)malloc(sizeof(double) * nW * N);
    aux_t *AX = (aux_t *)malloc(sizeof(aux_t) * N);
    if (!W || !AX) { free(W); free(AX); return -2; }

#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        double qc[NVMAX], Wc[NWMAX];
        gather(&s, q, c, qc);
        primitives(&s, qc, Wc, &AX[c]);
        for (int k = 0; k < nW; ++k) W[(int64_t)k * N + c] = Wc[k];
    }
    memset(rhs, 0, sizeof(double) * nvar * N);

    for (int dir = 0; dir < s.nd; ++dir) {
        int fn[3] = {pb->n[0], pb->n[1], pb->n[2]};
        fn[dir] += 1;
        int64_t nf = (int64_t)fn[0] * fn[1] * fn[2];
        double *F = (double *)malloc(sizeof(double) * nvar * nf);
        if (!F) { free(W); free(AX); return -2; }
#pragma omp parallel for schedule(static)
        for (int64_t f = 0; f < nf; ++f) {
            int co[3];
            co[0] = (int)(f % fn[0]);
            co[1] = (int)((f / fn[0]) % fn[1]);
            co[2] = (int)(f / ((int64_t)fn[0] * fn[1]));
            double Wst[6][NWMAX];
            for (int o = 0; o < 6; ++o) {
                int flip = 0;
                int cc[3] = {co[0], co[1], co[2]};
                cc[dir] = map_index(pb, dir, co[dir] - 3 + o, &flip);
                int64_t c = lin(pb, cc[0], cc[1], cc[2]);
                for (int k = 0; k < nW; ++k) Wst[o][k] = W[(int64_t)k * N + c];
                if (flip) Wst[o][1 + dir] = -Wst[o][1 + dir];
            }
            double Ff[NVMAX];
            face_flux(&s, dir, Wst, Ff);
            if (pb->viscous) visc_flux(&s, q, dir, co, Ff);
            for (int v = 0; v < nvar; ++v) F[(int64_t)v * nf + f] = Ff[v];
        }
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
            int co[3];
            co[0] = (int)(c % pb->n[0]);
            co[1] = (int)((c / pb->n[0]) % pb->n[1]);
            co[2] = (int)(c / ((int64_t)pb->n[0] * pb->n[1]));
            int lo[3] = {co[0], co[1], co[2]}, hi[3] = {co[0], co[1], co[2]};
            hi[dir] += 1;
            int64_t fl = lo[0] + (int64_t)fn[0] * (lo[1] + (int64_t)fn[1] * lo[2]);
            int64_t fh = hi[0] + (int64_t)fn[0] * (hi[1] + (int64_t)fn[1] * hi[2]);
            for (int v = 0; v < nvar; ++v)
                rhs[(int64_t)v * N + c] += (F[(int64_t)v * nf + fl] - F[(int64_t)v * nf + fh]) / pb->dx[dir];
        }
        free(F);
    }

    if (with_sources || pb->src_on) {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
            double Wc[NWMAX], Lc[NVMAX];
            for (int k = 0; k < nW; ++k) Wc[k] = W[(int64_t)k * N + c];
            memset(Lc, 0, sizeof(Lc));
            if (with_sources) cell_sources(&s, Wc, &AX[c], Lc);
            if (pb->src_on) {
                int co[3] = {(int)(c % pb->n[0]), (int)((c / pb->n[0]) % pb->n[1]),
                             (int)(c / ((int64_t)pb->n[0] * pb->n[1]))};
                acoustic_source(&s, Wc, co, t, Lc);
            }
            for (int v = 0; v < nvar; ++v) rhs[(int64_t)v * N + c] += Lc[v];
        }
    }
    free(W);
    free(AX);
    return 0;
}

int orc_rhs(const orc_problem *pb, const double *q, double *rhs) { return rhs_impl(pb, q, rhs, 1, pb->t); }

int orc_rhs_flux_only(const orc_problem *pb, const double *q, double *rhs)
{
    return rhs_impl(pb, q, rhs, 0, pb->t);
}

/* The same right-hand side, one listed cell at a time (stencil primitives are
 * recomputed locally), for spot checks on grids too large for orc_rhs. */
int orc_rhs_cells(const orc_problem *pb, const double *q, const int64_t *cells, int64_t k, double *out)
{
    setup_t s;
    if (setup(pb, &s) != 0) return -1;
    const int nvar = s.nvar;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < k; ++t) {
        int64_t c = cells[t];
        if (c < 0 || c >= s.N) { bad = 1; continue; }
        int co[3];
        co[0] = (int)(c % pb->n[0]);
        co[1] = (int)((c / pb->n[0]) % pb->n[1]);
        co[2] = (int)(c / ((int64_t)pb->n[0] * pb->n[1]));
        double L[NVMAX];
        memset(L, 0, sizeof(L));
        for (int dir = 0; dir < s.nd; ++dir) {
            double Wst[7][NWMAX];
            for (int o = 0; o < 7; ++o) stencil_prim(&s, q, dir, co, o - 3, Wst[o]);
            double Fl[NVMAX], Fh[NVMAX];
            face_flux(&s, dir, &Wst[0], Fl);
            face_flux(&s, dir, &Wst[1], Fh);
            if (pb->viscous) {
                int hi[3] = {co[0], co[1], co[2]};
                hi[dir] += 1;
                visc_flux(&s, q, dir, co, Fl);
                visc_flux(&s, q, dir, hi, Fh);
            }
            for (int v = 0; v < nvar; ++v) L[v] += (Fl[v] - Fh[v]) / pb->dx[dir];
        }
        double qc[NVMAX], Wc[NWMAX];
        aux_t ax;
        gather(&s, q, c, qc);
        primitives(&s, qc, Wc, &ax);
        cell_sources(&s, Wc, &ax, L);
        if (pb->src_on) acoustic_source(&s, Wc, co, pb->t, L);
        for (int v = 0; v < nvar; ++v) out[t * nvar + v] = L[v];
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Initial state, diagnostics, time step.                                    */
/* ------------------------------------------------------------------------ */
int orc_init_state(const orc_problem *pb, const double *prim, double *q)
{
    setup_t s;
    if (setup(pb, &s) != 0) return -1;
    const int64_t N = s.N;
    double m3 = 0.0;
    for (int i = 0; i < s.nb; ++i) m3 += s.w[i] * pow(s.r0[i], 3.0);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        double rhol = prim[c];
        double ke2 = 0.0;
        double pl = prim[(int64_t)(s.nd + 1) * N + c];
        double a = prim[(int64_t)(s.nd + 2) * N + c];
        double rho = (1.0 - a) * rhol;
        q[c] = rho;
        for (int d = 0; d < s.nd; ++d) {
            double u = prim[(int64_t)(1 + d) * N + c];
            q[(int64_t)(1 + d) * N + c] = rho * u;
            ke2 += u * u;
        }
        q[(int64_t)s.iE * N + c] = (1.0 - a) * (pl + pb->gamma * pb->pi_inf) / (pb->gamma - 1.0) + 0.5 * rho * ke2;
        q[(int64_t)s.iA * N + c] = a;
        double n = a > 0.0 ? a / (4.0 * ORC_PI / 3.0 * m3) : 0.0;
        for (int i = 0; i < s.nb; ++i) {
            q[(int64_t)(s.iNR + i) * N + c] = n * s.r0[i];
            q[(int64_t)(s.iNV + i) * N + c] = 0.0;
            if (s.nf == 4) {
                q[(int64_t)(s.iNP + i) * N + c] = n * s.pb0[i];
                q[(int64_t)(s.iNM + i) * N + c] = n * s.mv0[i];
            }
        }
    }
    return 0;
}

int orc_moments(const orc_problem *pb, const double *q, double *out)
{
    setup_t s;
    if (setup(pb, &s) != 0) return -1;
    const int64_t N = s.N;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        double qc[NVMAX], W[NWMAX];
        aux_t ax;
        gather(&s, q, c, qc);
        primitives(&s, qc, W, &ax);
        out[0 * N + c] = W[s.wN];
        out[1 * N + c] = W[s.wA];
        out[2 * N + c] = ax.M3;
        out[3 * N + c] = ax.M2d;
        out[4 * N + c] = ax.Mp;
        out[5 * N + c] = ax.Mk;
        out[6 * N + c] = ax.pmix;
        out[7 * N + c] = W[s.wPL];
    }
    return 0;
}

double orc_cfl_dt(const orc_problem *pb, const double *q)
{
    setup_t s;
    if (setup(pb, &s) != 0) return -1.0;
    const int64_t N = s.N;
    double best = INFINITY;
#pragma omp parallel
    {
        double mine = INFINITY;
#pragma omp for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
            double qc[NVMAX], W[NWMAX];
            aux_t ax;
            gather(&s, q, c, qc);
            primitives(&s, qc, W, &ax);
            for (int d = 0; d < s.nd; ++d) {
                double t = pb->dx[d] / (fabs(W[1 + d]) + ax.c);
                if (t < mine) mine = t;
            }
        }
#pragma omp critical
        if (mine < best) best = mine;
    }
    return pb->cfl * best;
}

/* ------------------------------------------------------------------------ */
/* SSP-RK3 (Gottlieb & Shu 1998) and the Strang-split variant.              */
/* ------------------------------------------------------------------------ */
static int rk3_flux(const orc_problem *pb, double *q, double dt, int with_sources)
{
    setup_t s;
    if (setup(pb, &s) != 0) return -1;
    const int64_t M = (int64_t)s.nvar * s.N;
    double *u1 = (double *)malloc(sizeof(double) * M);
    double *u2 = (double *)malloc(sizeof(double) * M);
    double *L = (double *)malloc(sizeof(double) * M);
    if (!u1 || !u2 || !L) { free(u1); free(u2); free(L); return -2; }
    /* each stage's L at the time of the state it is evaluated on: u^n at t, u1 at t + dt, u2 at t + dt/2 */
    int rc = rhs_impl(pb, q, L, with_sources, pb->t);
    for (int64_t m = 0; m < M && rc == 0; ++m) u1[m] = q[m] + dt * L[m];
    if (rc == 0) rc = rhs_impl(pb, u1, L, with_sources, pb->t + dt);
    for (int64_t m = 0; m < M && rc == 0; ++m) u2[m] = 0.75 * q[m] + 0.25 * (u1[m] + dt * L[m]);
    if (rc == 0) rc = rhs_impl(pb, u2, L, with_sources, pb->t + 0.5 * dt);
    for (int64_t m = 0; m < M && rc == 0; ++m) q[m] = q[m] / 3.0 + 2.0 / 3.0 * (u2[m] + dt * L[m]);
    free(u1);
    free(u2);
    free(L);
    return rc;
}

/* Embedded SSP-RK3 / Heun-RK2 adaptive integration of one bin's (R, Rdot) over
 * tau with p_l, rho_l, c frozen (Sec. 3, Strang splitting).  Returns accepted
 * sub-steps, or -1 if the attempt budget is exhausted. */
static int bubble_ode(const orc_problem *pb, double R0, double pg0, double pl, double rhol, double c,
                      double tau, double *R, double *V)
{
    const double rtol = pb->sub_rtol;
    const double vfloor = 1e-3 * sqrt(pb->p0 / pb->rho0);
    double t = 0.0, h = tau, y0 = *R, y1 = *V;
    int accepted = 0, attempts = 0;
    while (t < tau) {
        if (attempts >= pb->max_substeps) return -1;
        ++attempts;
        if (h > tau - t) h = tau - t;
        double k1r = y1, k1v = orc_km_rddot(pb, y0, y1, R0, pg0, pl, rhol, c);
        double a0 = y0 + h * k1r, a1 = y1 + h * k1v;
        double k2r = a1, k2v = orc_km_rddot(pb, a0, a1, R0, pg0, pl, rhol, c);
        double b0 = 0.75 * y0 + 0.25 * (a0 + h * k2r), b1 = 0.75 * y1 + 0.25 * (a1 + h * k2v);
        double e0 = y0 + 0.5 * h * (k1r + k2r), e1 = y1 + 0.5 * h * (k1v + k2v);
        double k3r = b1, k3v = orc_km_rddot(pb, b0, b1, R0, pg0, pl, rhol, c);
        double n0 = y0 / 3.0 + 2.0 / 3.0 * (b0 + h * k3r), n1 = y1 / 3.0 + 2.0 / 3.0 * (b1 + h * k3v);
        double err = fmax(fabs(n0 - e0) / fabs(n0), fabs(n1 - e1) / fmax(fabs(n1), vfloor));
        if (!(err == err)) err = INFINITY;
        if (err <= rtol && n0 > 0.0) {
            t += h;
            y0 = n0;
            y1 = n1;
            ++accepted;
        }
        double fac = err > 0.0 ? 0.9 * pow(rtol / err, 1.0 / 3.0) : 4.0;
        if (!(n0 > 0.0)) fac = 0.25;
        if (fac > 4.0) fac = 4.0;
        if (fac < 0.25) fac = 0.25;
        h *= fac;
    }
    *R = y0;
    *V = y1;
    return accepted;
}

/* The same embedded pair and step control for the transfer contents' (R, Rdot, p_b, m_v); the error
 * norm adds |dp|/|p| and |dm|/(|m| + mg) (vapour mass against the bubble's whole contents). */
static void tr_rates(const orc_problem *pb, double mg, double pl, double rhol, double c, const double *y,
                     double *f)
{
    double pdot, mdot;
    orc_contents_rates(pb, y[0], y[1], y[2], y[3], mg, &pdot, &mdot);
    f[0] = y[1];
    f[1] = orc_km_rddot_pb(pb, y[0], y[1], y[2], pdot, pl, rhol, c);
    f[2] = pdot;
    f[3] = mdot;
}

static int bubble_ode_tr(const orc_problem *pb, double mg, double pl, double rhol, double c, double tau,
                         double *y)
{
    const double rtol = pb->sub_rtol;
    const double vfloor = 1e-3 * sqrt(pb->p0 / pb->rho0);
    double t = 0.0, h = tau;
    int accepted = 0, attempts = 0;
    while (t < tau) {
        if (attempts >= pb->max_substeps) return -1;
        ++attempts;
        if (h > tau - t) h = tau - t;
        double k1[4], k2[4], k3[4], a[4], b[4], e[4], nn[4];
        tr_rates(pb, mg, pl, rhol, c, y, k1);
        for (int j = 0; j < 4; ++j) a[j] = y[j] + h * k1[j];
        tr_rates(pb, mg, pl, rhol, c, a, k2);
        for (int j = 0; j < 4; ++j) {
            b[j] = 0.75 * y[j] + 0.25 * (a[j] + h * k2[j]);
            e[j] = y[j] + 0.5 * h * (k1[j] + k2[j]);
        }
        tr_rates(pb, mg, pl, rhol, c, b, k3);
        for (int j = 0; j < 4; ++j) nn[j] = y[j] / 3.0 + 2.0 / 3.0 * (b[j] + h * k3[j]);
        double err = fmax(fabs(nn[0] - e[0]) / fabs(nn[0]), fabs(nn[1] - e[1]) / fmax(fabs(nn[1]), vfloor));
        err = fmax(err, fabs(nn[2] - e[2]) / fabs(nn[2]));
        err = fmax(err, fabs(nn[3] - e[3]) / (fabs(nn[3]) + mg));
        if (!(err == err)) err = INFINITY;
        if (err <= rtol && nn[0] > 0.0 && nn[2] > 0.0) {
            t += h;
            for (int j = 0; j < 4; ++j) y[j] = nn[j];
            ++accepted;
        }
        double fac = err > 0.0 ? 0.9 * pow(rtol / err, 1.0 / 3.0) : 4.0;
        if (!(nn[0] > 0.0) || !(nn[2] > 0.0)) fac = 0.25;
        if (fac > 4.0) fac = 4.0;
        if (fac < 0.25) fac = 0.25;
        h *= fac;
    }
    return accepted;
}

int orc_bubble_advance(const orc_problem *pb, double *q, double dt, int32_t *nsub_out)
{
    setup_t s;
    if (setup(pb, &s) != 0) return -1;
    const int64_t N = s.N;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < N; ++c) {
        double qc[NVMAX], W[NWMAX];
        aux_t ax;
        gather(&s, q, c, qc);
        primitives(&s, qc, W, &ax);
        double a = W[s.wA];
        if (!(a > 0.0)) {
            if (nsub_out)
                for (int i = 0; i < s.nb; ++i) nsub_out[(int64_t)i * N + c] = 0;
            continue;
        }
        double n = W[s.wN];
        double m3new = 0.0;
        for (int i = 0; i < s.nb; ++i) {
            double R = W[s.wR + i], V = W[s.wV + i];
            int ns;
            if (s.nf == 4) {
                double y[4] = {R, V, W[s.wP + i], W[s.wM + i]};
                ns = bubble_ode_tr(pb, s.mg[i], W[s.wPL], ax.rhol, ax.c, dt, y);
                R = y[0];
                V = y[1];
                q[(int64_t)(s.iNP + i) * N + c] = n * y[2];
                q[(int64_t)(s.iNM + i) * N + c] = n * y[3];
            } else {
                ns = bubble_ode(pb, s.r0[i], s.pg0[i], W[s.wPL], ax.rhol, ax.c, dt, &R, &V);
            }
            if (ns < 0) fail = 1;
            if (nsub_out) nsub_out[(int64_t)i * N + c] = ns;
            q[(int64_t)(s.iNR + i) * N + c] = n * R;
            q[(int64_t)(s.iNV + i) * N + c] = n * V;
            m3new += s.w[i] * R * R * R;
        }
        q[(int64_t)s.iA * N + c] = a * m3new / ax.M3;
    }
    return fail ? -6 : 0;
}

int orc_rk3_step(const orc_problem *pb, double *q, double dt, double *dt_used)
{
    if (!(dt > 0.0)) dt = orc_cfl_dt(pb, q);
    if (!(dt > 0.0)) return -1;
    if (dt_used) *dt_used = dt;
    if (!pb->split) return rk3_flux(pb, q, dt, 1);
    int rc = orc_bubble_advance(pb, q, 0.5 * dt, NULL);
    if (rc == 0) rc = rk3_flux(pb, q, dt, 0);
    if (rc == 0) rc = orc_bubble_advance(pb, q, 0.5 * dt, NULL);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Single-bubble adaptive Dormand--Prince 5(4) (published tableau, 1980).   */
/* ------------------------------------------------------------------------ */
static void km_f(const orc_problem *pb, double R0, double pg0, double pinf, double rho, double c,
                 const double *y, double *f)
{
    f[0] = y[1];
    f[1] = orc_km_rddot(pb, y[0], y[1], R0, pg0, pinf, rho, c);
}

void orc_km_dp54_step(const orc_problem *pb, double R0, double pg0, double pinf, double rho, double c,
                      const double *y, double h, double *y5, double *y4)
{
    static const double a21 = 1.0 / 5.0;
    static const double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
    static const double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
    static const double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                        a54 = -212.0 / 729.0;
    static const double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                        a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
    static const double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                        b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
    static const double e1 = 5179.0 / 57600.0, e3 = 7571.0 / 16695.0, e4 = 393.0 / 640.0,
                        e5 = -92097.0 / 339200.0, e6 = 187.0 / 2100.0, e7 = 1.0 / 40.0;
    double k1[2], k2[2], k3[2], k4[2], k5[2], k6[2], k7[2], t[2];
    km_f(pb, R0, pg0, pinf, rho, c, y, k1);
    for (int m = 0; m < 2; ++m) t[m] = y[m] + h * a21 * k1[m];
    km_f(pb, R0, pg0, pinf, rho, c, t, k2);
    for (int m = 0; m < 2; ++m) t[m] = y[m] + h * (a31 * k1[m] + a32 * k2[m]);
    km_f(pb, R0, pg0, pinf, rho, c, t, k3);
    for (int m = 0; m < 2; ++m) t[m] = y[m] + h * (a41 * k1[m] + a42 * k2[m] + a43 * k3[m]);
    km_f(pb, R0, pg0, pinf, rho, c, t, k4);
    for (int m = 0; m < 2; ++m) t[m] = y[m] + h * (a51 * k1[m] + a52 * k2[m] + a53 * k3[m] + a54 * k4[m]);
    km_f(pb, R0, pg0, pinf, rho, c, t, k5);
    for (int m = 0; m < 2; ++m)
        t[m] = y[m] + h * (a61 * k1[m] + a62 * k2[m] + a63 * k3[m] + a64 * k4[m] + a65 * k5[m]);
    km_f(pb, R0, pg0, pinf, rho, c, t, k6);
    for (int m = 0; m < 2; ++m)
        y5[m] = y[m] + h * (b1 * k1[m] + b3 * k3[m] + b4 * k4[m] + b5 * k5[m] + b6 * k6[m]);
    km_f(pb, R0, pg0, pinf, rho, c, y5, k7);
    for (int m = 0; m < 2; ++m)
        y4[m] = y[m] + h * (e1 * k1[m] + e3 * k3[m] + e4 * k4[m] + e5 * k5[m] + e6 * k6[m] + e7 * k7[m]);
}

int64_t orc_km_integrate(const orc_problem *pb, double R0, double pg0, double pinf, double rho, double c,
                         double R_init, double V_init, double rtol, double atol_r, double atol_v, int nt,
                         const double *t_out, double *R_out, double *V_out, double r_stop, double *t_stop)
{
    double y[2] = {R_init, V_init};
    double t = 0.0;
    double t_end = nt > 0 ? t_out[nt - 1] : 0.0;
    double h = 1e-3 * (t_end > 0 ? t_end : 1e-6);
    int next = 0;
    int64_t steps = 0;
    if (t_stop) *t_stop = -1.0;
    while (next < nt && t_out[next] <= 0.0) {
        R_out[next] = y[0];
        V_out[next] = y[1];
        ++next;
    }
    while (next < nt || (r_stop > 0.0 && t_stop && *t_stop < 0.0)) {
        if (steps > 100000000LL) return -1;
        double target = next < nt ? t_out[next] : INFINITY;
        double hh = h;
        int hit = 0;
        if (t + hh >= target) { hh = target - t; hit = 1; }
        double y5[2], y4[2];
        orc_km_dp54_step(pb, R0, pg0, pinf, rho, c, y, hh, y5, y4);
        double sc0 = atol_r + rtol * fmax(fabs(y[0]), fabs(y5[0]));
        double sc1 = atol_v + rtol * fmax(fabs(y[1]), fabs(y5[1]));
        double err = fmax(fabs(y5[0] - y4[0]) / sc0, fabs(y5[1] - y4[1]) / sc1);
        if (!(err == err) || !(y5[0] > 0.0)) err = INFINITY;
        if (err <= 1.0) {
            if (r_stop > 0.0 && t_stop && *t_stop < 0.0 && y5[0] <= r_stop) {
                /* Locate the crossing by bisection on the step length from (t, y). */
                double lo = 0.0, hi = hh;
                for (int it = 0; it < 200; ++it) {
                    double mid = 0.5 * (lo + hi);
                    double z5[2], z4[2];
                    orc_km_dp54_step(pb, R0, pg0, pinf, rho, c, y, mid, z5, z4);
                    if (z5[0] > r_stop) lo = mid; else hi = mid;
                    if (hi - lo <= 1e-15 * (t + hi)) break;
                }
                *t_stop = t + 0.5 * (lo + hi);
                return steps;
            }
            t += hh;
            y[0] = y5[0];
            y[1] = y5[1];
            ++steps;
            if (hit) {
                t = target;
                R_out[next] = y[0];
                V_out[next] = y[1];
                ++next;
            }
        }
        double fac = err > 0.0 ? 0.9 * pow(1.0 / err, 0.2) : 5.0;
        if (fac > 5.0) fac = 5.0;
        if (fac < 0.2) fac = 0.2;
        if (!hit || err > 1.0) h = hh * fac;
    }
    return steps;
}

/* Number of OpenMP threads the oracle's parallel loops use (for reporting). */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the oracle's later parallel loops (for timing it on one core and on all). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
