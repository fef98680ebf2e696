/*
 * Plain FP64 CPU oracle, volume-averaged (Euler--Lagrange) variant, Sec. 2.1.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  Three-dimensional grids with a
 * uniform spacing.  Sequential over bubbles in the smear, so the sums are
 * deterministic; OpenMP only over independent cells, faces or bubbles.
 *
 *   kernel          eq. kernel3D, truncated at d/h = 3, width h = max(dx, R)
 *                   (eq. model_inequality and the rule that follows it).
 *   smear           alpha = sum_n V_n delta_n and its rate sum_n 4 pi R^2 Rdot delta_n
 *                   (the void-fraction definition and its time derivative; with
 *                   fixed bubbles the -u.grad(delta) part cancels against u.grad(alpha)
 *                   in the source bracket).
 *   gather          kernel-weighted liquid pressure, normalised by the kernel sum.
 *   liquid RHS      the liquid equations of Sec. 2.1 (inviscid): stiffened-gas
 *                   Euler fluxes by WENO5 + HLLC, sources
 *                   rho_l D/(1-alpha), rho_l u D/(1-alpha) - alpha grad p/(1-alpha),
 *                   E_l D/(1-alpha) - alpha div(p u)/(1-alpha), the gradients taken
 *                   from face averages of the reconstructed pressure.
 *   bubbles         Keller--Miksis per bubble, adaptive Dormand--Prince 5(4).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

double orc_el_kernel(double d, double h)
{
    if (d >= 3.0 * h) return 0.0;
    return exp(-d * d / (2.0 * h * h)) / (h * h * h * pow(2.0 * ORC_PI, 1.5));
}

static int el_check(const orc_problem *pb)
{
    if (pb->ndim != 3) return -7;
    if (pb->contents != 0) return -1;   /* the Lagrangian bubbles carry polytropic contents only */
    for (int d = 0; d < 3; ++d) {
        if (pb->n[d] < 3 || !(pb->dx[d] > 0.0)) return -1;
        if (pb->dx[d] != pb->dx[0]) return -1;
        for (int e = 0; e < 2; ++e)
            if (pb->bc[d][e] != 0 && pb->bc[d][e] != 1) return -1;
    }
    return 0;
}

static int64_t el_lin(const orc_problem *pb, const int c[3])
{
    return (int64_t)c[0] + (int64_t)pb->n[0] * ((int64_t)c[1] + (int64_t)pb->n[1] * c[2]);
}

/* Map one coordinate of a kernel-stencil cell: periodic wrap, or -1 when the
 * cell lies outside a reflective wall (such cells are skipped). */
static int el_wrap(const orc_problem *pb, int d, int i)
{
    int n = pb->n[d];
    if (i < 0) return pb->bc[d][0] == 0 ? ((i % n) + n) % n : -1;
    if (i >= n) return pb->bc[d][1] == 0 ? i % n : -1;
    return i;
}

typedef struct {
    double rho, u[3], p, E, c;
} liq_t;

static void liq_prim(const orc_problem *pb, const double *ql, int64_t N, int64_t c, liq_t *s)
{
    s->rho = ql[c];
    double ke = 0.0;
    for (int d = 0; d < 3; ++d) {
        s->u[d] = ql[(1 + d) * N + c] / s->rho;
        ke += 0.5 * s->rho * s->u[d] * s->u[d];
    }
    s->E = ql[4 * N + c];
    s->p = (pb->gamma - 1.0) * (s->E - ke) - pb->gamma * pb->pi_inf;
    s->c = sqrt(pb->gamma * (s->p + pb->pi_inf) / s->rho);
}

int orc_el_smear(const orc_problem *pb, const double *bub, int64_t nbub, double *alpha, double *dalpha)
{
    int rc = el_check(pb);
    if (rc) return rc;
    const int64_t N = (int64_t)pb->n[0] * pb->n[1] * pb->n[2];
    const double dx = pb->dx[0];
    memset(alpha, 0, sizeof(double) * N);
    memset(dalpha, 0, sizeof(double) * N);
    for (int64_t b = 0; b < nbub; ++b) {
        double xb[3] = {bub[0 * nbub + b], bub[1 * nbub + b], bub[2 * nbub + b]};
        double R = bub[4 * nbub + b], V = bub[5 * nbub + b];
        double h = R > dx ? R : dx;
        int m = (int)ceil(3.0 * h / dx);
        int host[3];
        for (int d = 0; d < 3; ++d) host[d] = (int)floor(xb[d] / dx);
        double vol = 4.0 / 3.0 * ORC_PI * R * R * R;
        double rate = 4.0 * ORC_PI * R * R * V;
        for (int k = -m; k <= m; ++k)
            for (int j = -m; j <= m; ++j)
                for (int i = -m; i <= m; ++i) {
                    int off[3] = {i, j, k}, cc[3], out = 0;
                    double d2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        double xc = (host[d] + off[d] + 0.5) * dx;
                        d2 += (xc - xb[d]) * (xc - xb[d]);
                        cc[d] = el_wrap(pb, d, host[d] + off[d]);
                        if (cc[d] < 0) out = 1;
                    }
                    if (out) continue;
                    double w = orc_el_kernel(sqrt(d2), h);
                    if (w == 0.0) continue;
                    int64_t c = el_lin(pb, cc);
                    alpha[c] += vol * w;
                    dalpha[c] += rate * w;
                }
    }
    return 0;
}

int orc_el_gather(const orc_problem *pb, const double *ql, const double *bub, int64_t nbub, double *p_inf,
                  double *rho_l, double *c_l)
{
    int rc = el_check(pb);
    if (rc) return rc;
    const int64_t N = (int64_t)pb->n[0] * pb->n[1] * pb->n[2];
    const double dx = pb->dx[0];
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nbub; ++b) {
        double xb[3] = {bub[0 * nbub + b], bub[1 * nbub + b], bub[2 * nbub + b]};
        double R = bub[4 * nbub + b];
        double h = R > dx ? R : dx;
        int m = (int)ceil(3.0 * h / dx);
        int host[3];
        for (int d = 0; d < 3; ++d) host[d] = (int)floor(xb[d] / dx);
        double sw = 0.0, swp = 0.0;
        for (int k = -m; k <= m; ++k)
            for (int j = -m; j <= m; ++j)
                for (int i = -m; i <= m; ++i) {
                    int off[3] = {i, j, k}, cc[3], out = 0;
                    double d2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        double xc = (host[d] + off[d] + 0.5) * dx;
                        d2 += (xc - xb[d]) * (xc - xb[d]);
                        cc[d] = el_wrap(pb, d, host[d] + off[d]);
                        if (cc[d] < 0) out = 1;
                    }
                    if (out) continue;
                    double w = orc_el_kernel(sqrt(d2), h);
                    if (w == 0.0) continue;
                    liq_t s;
                    liq_prim(pb, ql, N, el_lin(pb, cc), &s);
                    sw += w;
                    swp += w * s.p;
                }
        int hc[3];
        for (int d = 0; d < 3; ++d) {
            hc[d] = el_wrap(pb, d, host[d]);
            if (hc[d] < 0) hc[d] = host[d] < 0 ? 0 : pb->n[d] - 1;
        }
        liq_t s;
        liq_prim(pb, ql, N, el_lin(pb, hc), &s);
        p_inf[b] = swp / sw;
        rho_l[b] = s.rho;
        c_l[b] = s.c;
    }
    return 0;
}

/* Liquid primitive [rho, u, v, w, p] of the (possibly ghost) cell at offset off
 * along dir from coord; reflective ghosts mirror with the normal velocity negated. */
static void liq_stencil(const orc_problem *pb, const double *ql, int64_t N, int dir, const int co[3],
                        int off, double *W)
{
    int cc[3] = {co[0], co[1], co[2]};
    int i = co[dir] + off, n = pb->n[dir], flip = 0;
    if (i < 0) {
        if (pb->bc[dir][0] == 0) i = ((i % n) + n) % n;
        else { i = -1 - i; flip = 1; }
    } else if (i >= n) {
        if (pb->bc[dir][1] == 0) i = i % n;
        else { i = 2 * n - 1 - i; flip = 1; }
    }
    cc[dir] = i;
    liq_t s;
    liq_prim(pb, ql, N, el_lin(pb, cc), &s);
    W[0] = s.rho;
    W[1] = s.u[0];
    W[2] = s.u[1];
    W[3] = s.u[2];
    W[4] = s.p;
    if (flip) W[1 + dir] = -W[1 + dir];
}

/* Face between cells co-e_dir and co: HLLC flux (5 values) and the face states'
 * pressures and normal velocities for the gradient terms. */
static void liq_face(const orc_problem *pb, const double *ql, int64_t N, int dir, const int co[3],
                     double *F, double *pL, double *pR, double *uL, double *uR)
{
    double st[6][5], WL[5], WR[5], v[5];
    for (int o = 0; o < 6; ++o) liq_stencil(pb, ql, N, dir, co, o - 3, st[o]);
    for (int k = 0; k < 5; ++k) {
        for (int o = 0; o < 5; ++o) v[o] = st[o][k];
        WL[k] = orc_weno5(v);
        for (int o = 0; o < 5; ++o) v[o] = st[5 - o][k];
        WR[k] = orc_weno5(v);
    }
    if (!(WL[0] > 0.0 && WR[0] > 0.0 && WL[4] + pb->pi_inf > 0.0 && WR[4] + pb->pi_inf > 0.0)) {
        memcpy(WL, st[2], sizeof(WL));
        memcpy(WR, st[3], sizeof(WR));
    }
    /* Pure liquid through the mixture HLLC: alpha = 0, no bubbles (one empty bin). */
    orc_problem q = *pb;
    q.nb = 1;
    q.r0_median = 1.0;
    q.sigma_ln = 0.0;
    double EL_[10] = {WL[0], WL[1], WL[2], WL[3], WL[4], 0.0, 0.0, 0.0, 1.0, 0.0};
    double ER_[10] = {WR[0], WR[1], WR[2], WR[3], WR[4], 0.0, 0.0, 0.0, 1.0, 0.0};
    double Ff[8];
    orc_hllc(&q, dir, EL_, ER_, Ff);
    for (int k = 0; k < 5; ++k) F[k] = Ff[k];
    *pL = WL[4];
    *pR = WR[4];
    *uL = WL[1 + dir];
    *uR = WR[1 + dir];
}

int orc_el_rhs(const orc_problem *pb, const double *ql, const double *alpha, const double *dalpha, double *rhs)
{
    int rc = el_check(pb);
    if (rc) return rc;
    const int64_t N = (int64_t)pb->n[0] * pb->n[1] * pb->n[2];
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int co[3];
        co[0] = (int)(c % pb->n[0]);
        co[1] = (int)((c / pb->n[0]) % pb->n[1]);
        co[2] = (int)(c / ((int64_t)pb->n[0] * pb->n[1]));
        double L[5] = {0, 0, 0, 0, 0}, gradp[3], divpu = 0.0;
        for (int dir = 0; dir < 3; ++dir) {
            int hi[3] = {co[0], co[1], co[2]};
            hi[dir] += 1;
            double Fl[5], Fh[5], pl0, pr0, ul0, ur0, pl1, pr1, ul1, ur1;
            liq_face(pb, ql, N, dir, co, Fl, &pl0, &pr0, &ul0, &ur0);
            liq_face(pb, ql, N, dir, hi, Fh, &pl1, &pr1, &ul1, &ur1);
            for (int k = 0; k < 5; ++k) L[k] += (Fl[k] - Fh[k]) / pb->dx[dir];
            gradp[dir] = (0.5 * (pl1 + pr1) - 0.5 * (pl0 + pr0)) / pb->dx[dir];
            divpu += (0.5 * (pl1 * ul1 + pr1 * ur1) - 0.5 * (pl0 * ul0 + pr0 * ur0)) / pb->dx[dir];
        }
        liq_t s;
        liq_prim(pb, ql, N, c, &s);
        double a = alpha[c], D = dalpha[c];
        L[0] += s.rho * D / (1.0 - a);
        for (int d = 0; d < 3; ++d) L[1 + d] += s.rho * s.u[d] * D / (1.0 - a) - a * gradp[d] / (1.0 - a);
        L[4] += s.E * D / (1.0 - a) - a * divpu / (1.0 - a);
        for (int k = 0; k < 5; ++k) rhs[k * N + c] = L[k];
    }
    return 0;
}

static double el_cfl_dt(const orc_problem *pb, const double *ql)
{
    const int64_t N = (int64_t)pb->n[0] * pb->n[1] * pb->n[2];
    double best = INFINITY;
    for (int64_t c = 0; c < N; ++c) {
        liq_t s;
        liq_prim(pb, ql, N, c, &s);
        for (int d = 0; d < 3; ++d) {
            double t = pb->dx[d] / (fabs(s.u[d]) + s.c);
            if (t < best) best = t;
        }
    }
    return pb->cfl * best;
}

/* Adaptive DP5(4) over tau for every bubble, forcing frozen at its start. */
static int el_bubbles(const orc_problem *pb, const double *ql, double *bub, int64_t nbub, double tau,
                      int32_t *nsub)
{
    double *pinf = (double *)malloc(sizeof(double) * 3 * (nbub > 0 ? nbub : 1));
    if (!pinf) return -2;
    double *rl = pinf + nbub, *cl = pinf + 2 * nbub;
    int rc = orc_el_gather(pb, ql, bub, nbub, pinf, rl, cl);
    if (rc) { free(pinf); return rc; }
    const double rtol = pb->sub_rtol;
    const double vfloor = 1e-3 * sqrt(pb->p0 / pb->rho0);
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nbub; ++b) {
        double R0 = bub[3 * nbub + b], pg0 = bub[6 * nbub + b];
        double y[2] = {bub[4 * nbub + b], bub[5 * nbub + b]};
        double h = bub[7 * nbub + b];
        if (!(h > 0.0)) h = tau;
        double t = 0.0;
        int acc = 0, att = 0;
        while (t < tau) {
            if (att >= pb->max_substeps) { fail = 1; break; }
            ++att;
            double hs = h < tau - t ? h : tau - t;
            double y5[2], y4[2];
            orc_km_dp54_step(pb, R0, pg0, pinf[b], rl[b], cl[b], y, hs, y5, y4);
            double err = fmax(fabs(y5[0] - y4[0]) / fabs(y5[0]), fabs(y5[1] - y4[1]) / fmax(fabs(y5[1]), vfloor));
            if (!(err == err)) err = INFINITY;
            int ok = err <= rtol && y5[0] > 0.0;
            if (ok) {
                t += hs;
                y[0] = y5[0];
                y[1] = y5[1];
                ++acc;
            }
            double fac = err > 0.0 ? 0.9 * pow(rtol / err, 0.2) : 4.0;
            if (!(y5[0] > 0.0)) fac = 0.25;
            if (fac > 4.0) fac = 4.0;
            if (fac < 0.25) fac = 0.25;
            h = hs * fac;
        }
        bub[4 * nbub + b] = y[0];
        bub[5 * nbub + b] = y[1];
        bub[7 * nbub + b] = h;
        if (nsub) nsub[b] += acc;
    }
    free(pinf);
    return fail ? -6 : 0;
}

int orc_el_step(const orc_problem *pb, double *ql, double *bub, int64_t nbub, double dt, double *alpha,
                double *dalpha, int32_t *nsub_out, double *dt_used)
{
    int rc = el_check(pb);
    if (rc) return rc;
    const int64_t N = (int64_t)pb->n[0] * pb->n[1] * pb->n[2];
    if (!(dt > 0.0)) dt = el_cfl_dt(pb, ql);
    if (dt_used) *dt_used = dt;
    if (nsub_out) memset(nsub_out, 0, sizeof(int32_t) * nbub);
    rc = el_bubbles(pb, ql, bub, nbub, 0.5 * dt, nsub_out);
    if (rc) return rc;
    rc = orc_el_smear(pb, bub, nbub, alpha, dalpha);
    if (rc) return rc;
    const int64_t M = 5 * N;
    double *u1 = (double *)malloc(sizeof(double) * M);
    double *u2 = (double *)malloc(sizeof(double) * M);
    double *L = (double *)malloc(sizeof(double) * M);
    if (!u1 || !u2 || !L) { free(u1); free(u2); free(L); return -2; }
    rc = orc_el_rhs(pb, ql, alpha, dalpha, L);
    for (int64_t m = 0; m < M && !rc; ++m) u1[m] = ql[m] + dt * L[m];
    if (!rc) rc = orc_el_rhs(pb, u1, alpha, dalpha, L);
    for (int64_t m = 0; m < M && !rc; ++m) u2[m] = 0.75 * ql[m] + 0.25 * (u1[m] + dt * L[m]);
    if (!rc) rc = orc_el_rhs(pb, u2, alpha, dalpha, L);
    for (int64_t m = 0; m < M && !rc; ++m) ql[m] = ql[m] / 3.0 + 2.0 / 3.0 * (u2[m] + dt * L[m]);
    free(u1);
    free(u2);
    free(L);
    if (rc) return rc;
    rc = el_bubbles(pb, ql, bub, nbub, 0.5 * dt, nsub_out);
    if (rc) return rc;
    return orc_el_smear(pb, bub, nbub, alpha, dalpha);
}
