// Volume-averaged (Euler--Lagrange) variant, Sec. 2.1, for gfx950.
//
//  k_el_bubinit  bubble records (x, y, z, R0) -> state at rest at R0.
//  k_el_init     liquid primitives -> conserved liquid state.
//  k_el_prim     liquid primitives (rho, u, v, w, p) per cell, optional CFL max.
//  k_el_gather   one wavefront per bubble: kernel-weighted liquid pressure over
//                the truncated Gaussian support (normalised), host-cell rho, c.
//  k_el_ode      one thread per bubble: Keller--Miksis with adaptive
//                Dormand--Prince 5(4) sub-steps, forcing frozen.
//  k_el_scatter  one wavefront per bubble: volume and volume rate smeared with
//                the kernel (eq. kernel3D) by FP64 atomic adds.
//  k_el_stage    a workgroup per tile of cells: the tile's primitives and their
//                halos staged in LDS per direction, WENO5 + HLLC fluxes of the
//                liquid (stiffened gas), each face once; the bubble source
//                terms with alpha and its rate frozen; RK combine.
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace bub {

// bubble record slots
enum { BX_ = 0, BY_ = 1, BZ_ = 2, BR0 = 3, BRR = 4, BRD = 5, BPG = 6, BHS = 7, NBREC = 8 };

struct ElGrid {
    int n[3];
    int bc[3];
    double dx, inv_dx;
    long long N;
};

// stencil coordinate: periodic wrap, or -1 outside a reflective wall
__device__ inline int el_wrap(int i, int n, int bc)
{
    if ((unsigned)i < (unsigned)n) return i;
    if (bc != 0) return -1;
    int m = i % n;
    return m < 0 ? m + n : m;
}

__global__ void k_el_bubinit(const double *__restrict__ xyzr, double *__restrict__ b, long long nb, Phys ph,
                             double sigma2, double pv)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (long long)gridDim.x * blockDim.x) {
        double r0 = xyzr[3 * nb + i];
        b[BX_ * nb + i] = xyzr[i];
        b[BY_ * nb + i] = xyzr[nb + i];
        b[BZ_ * nb + i] = xyzr[2 * nb + i];
        b[BR0 * nb + i] = r0;
        b[BRR * nb + i] = r0;
        b[BRD * nb + i] = 0.0;
        b[BPG * nb + i] = ph.p0 + sigma2 / r0 - pv;
        b[BHS * nb + i] = 0.0;
    }
}

__global__ void k_el_init(const double *__restrict__ prim, double *__restrict__ ql, long long N, Phys ph)
{
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        double rho = prim[c], ke = 0.0;
        ql[c] = rho;
        for (int d = 0; d < 3; ++d) {
            double u = prim[(1 + d) * N + c];
            ql[(1 + d) * N + c] = rho * u;
            ke += u * u;
        }
        ql[4 * N + c] = (prim[4 * N + c] + ph.gpi) * ph.inv_gm1 + 0.5 * rho * ke;
    }
}

template <bool CFL>
__global__ void __launch_bounds__(256) k_el_prim(const double *__restrict__ ql, double *__restrict__ P, ElGrid g,
                                                 Phys ph, Scalars *sc)
{
    const long long N = g.N;
    double wmax = 0.0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        double rho = ql[c];
        double ir = frcp(rho);
        double u[3], ke = 0.0;
        for (int d = 0; d < 3; ++d) {
            u[d] = ql[(1 + d) * N + c] * ir;
            ke += u[d] * u[d];
        }
        double p = ph.gm1 * (ql[4 * N + c] - 0.5 * rho * ke) - ph.gpi;
        P[c] = rho;
        for (int d = 0; d < 3; ++d) P[(1 + d) * N + c] = u[d];
        P[4 * N + c] = p;
        if (!(rho > 0.0) || !(p + ph.pi_inf > 0.0)) raise_error(sc, E_NONFINITE, c, -1);
        if (CFL) {
            double cs = sqrt(ph.gamma * (p + ph.pi_inf) * ir);
            for (int d = 0; d < 3; ++d) wmax = dmax(wmax, (fabs(u[d]) + cs) * g.inv_dx);
        }
    }
    if (CFL) wmax_post(wmax, sc);
}

// Host cell of a bubble coordinate and the kernel support half-width in cells.
__device__ inline void el_support(const double *b, long long nb, long long i, const ElGrid &g, int host[3], double &h,
                                  int &m)
{
    double R = b[BRR * nb + i];
    h = dmax(g.dx, R);
    m = (int)ceil(3.0 * h * g.inv_dx);
    for (int d = 0; d < 3; ++d) host[d] = (int)floor(b[d * nb + i] * g.inv_dx);
}

// one wavefront (64 lanes) per bubble
// Visit the cells of a bubble's kernel support (eq. kernel3D: cut off at distance 3h).  The lanes of the
// bubble's wavefront take the (x, y) points of the (2m+1)^2 stencil plane (more passes when it exceeds 64)
// and each walks the 2m+1 z planes of its column, so no lane divides by the stencil width per cell.
// f(c, e) for every cell c inside the domain and the cut-off, e = exp(-d^2 / (2 h^2)) (the Gaussian
// without its normalisation).
template <typename F>
__device__ __forceinline__ void el_visit(const ElGrid &g, const int host[3], const double xb[3], double h, int m,
                                         int lane, F &&f)
{
    const int w = 2 * m + 1, w2 = w * w;
    const double cut = 9.0 * h * h, nh = -0.5 / (h * h);
    const long long nxy = (long long)g.n[0] * g.n[1];
    for (int p = lane; p < w2; p += 64) {
        const int ix = host[0] + p % w - m, iy = host[1] + p / w - m;
        const int cx = el_wrap(ix, g.n[0], g.bc[0]), cy = el_wrap(iy, g.n[1], g.bc[1]);
        if (cx < 0 || cy < 0) continue;
        const double ex = (ix + 0.5) * g.dx - xb[0], ey = (iy + 0.5) * g.dx - xb[1];
        const double dxy = ex * ex + ey * ey;
        if (!(dxy < cut)) continue;
        const long long cxy = cx + (long long)g.n[0] * cy;
        for (int iz = host[2] - m; iz <= host[2] + m; ++iz) {
            const int cz = el_wrap(iz, g.n[2], g.bc[2]);
            if (cz < 0) continue;
            const double ez = (iz + 0.5) * g.dx - xb[2];
            const double d2 = dxy + ez * ez;
            if (!(d2 < cut)) continue;
            f(cxy + nxy * cz, exp(d2 * nh));
        }
    }
}

__global__ void __launch_bounds__(256) k_el_gather(const double *__restrict__ P, const double *__restrict__ b,
                                                   long long nb, ElGrid g, Phys ph, double *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= nb) return;
    const long long N = g.N;
    int host[3], m;
    double h;
    el_support(b, nb, i, g, host, h, m);
    const double xb[3] = {b[BX_ * nb + i], b[BY_ * nb + i], b[BZ_ * nb + i]};
    // normalised weights: the Gaussian's constant factor cancels
    double sw = 0.0, swp = 0.0;
    el_visit(g, host, xb, h, m, lane, [&](long long c, double e) {
        sw += e;
        swp += e * P[4 * N + c];
    });
    for (int s = 32; s > 0; s >>= 1) {
        sw += __shfl_xor(sw, s, 64);
        swp += __shfl_xor(swp, s, 64);
    }
    if (lane == 0) {
        int hc[3];
        for (int d = 0; d < 3; ++d) {
            hc[d] = el_wrap(host[d], g.n[d], g.bc[d]);
            if (hc[d] < 0) hc[d] = host[d] < 0 ? 0 : g.n[d] - 1;
        }
        long long c = hc[0] + (long long)g.n[0] * (hc[1] + (long long)g.n[1] * hc[2]);
        double rho = P[c], p = P[4 * N + c];
        out[i] = swp / sw;
        out[nb + i] = rho;
        out[2 * nb + i] = sqrt(ph.gamma * (p + ph.pi_inf) / rho);
    }
}

// Dormand--Prince 5(4) step of (R, Rdot) (published tableau, 1980).
template <bool PW>
__device__ inline void dp54(const Phys &ph, double r0, double pg0, double pinf, double irho, double ic, double y0,
                            double y1, double h, double &r5, double &v5, double &r4, double &v4)
{
    const double a21 = 1.0 / 5.0;
    const double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
    const double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
    const double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0, a54 = -212.0 / 729.0;
    const double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0, a64 = 49.0 / 176.0,
                 a65 = -5103.0 / 18656.0;
    const double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0, b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
    const double e1 = 5179.0 / 57600.0, e3 = 7571.0 / 16695.0, e4 = 393.0 / 640.0, e5 = -92097.0 / 339200.0,
                 e6 = 187.0 / 2100.0, e7 = 1.0 / 40.0;
    auto f = [&](double R, double V) { return km_rddot<PW>(ph, R, V, r0, pg0, pinf, irho, ic); };
    double k1r = y1, k1v = f(y0, y1);
    double t0 = y0 + h * a21 * k1r, t1 = y1 + h * a21 * k1v;
    double k2r = t1, k2v = f(t0, t1);
    t0 = y0 + h * (a31 * k1r + a32 * k2r);
    t1 = y1 + h * (a31 * k1v + a32 * k2v);
    double k3r = t1, k3v = f(t0, t1);
    t0 = y0 + h * (a41 * k1r + a42 * k2r + a43 * k3r);
    t1 = y1 + h * (a41 * k1v + a42 * k2v + a43 * k3v);
    double k4r = t1, k4v = f(t0, t1);
    t0 = y0 + h * (a51 * k1r + a52 * k2r + a53 * k3r + a54 * k4r);
    t1 = y1 + h * (a51 * k1v + a52 * k2v + a53 * k3v + a54 * k4v);
    double k5r = t1, k5v = f(t0, t1);
    t0 = y0 + h * (a61 * k1r + a62 * k2r + a63 * k3r + a64 * k4r + a65 * k5r);
    t1 = y1 + h * (a61 * k1v + a62 * k2v + a63 * k3v + a64 * k4v + a65 * k5v);
    double k6r = t1, k6v = f(t0, t1);
    r5 = y0 + h * (b1 * k1r + b3 * k3r + b4 * k4r + b5 * k5r + b6 * k6r);
    v5 = y1 + h * (b1 * k1v + b3 * k3v + b4 * k4v + b5 * k5v + b6 * k6v);
    double k7r = v5, k7v = f(r5, v5);
    r4 = y0 + h * (e1 * k1r + e3 * k3r + e4 * k4r + e5 * k5r + e6 * k6r + e7 * k7r);
    v4 = y1 + h * (e1 * k1v + e3 * k3v + e4 * k4v + e5 * k5v + e6 * k6v + e7 * k7v);
}

struct ElOdeArgs {
    double *b;
    long long nb;
    const double *forcing;  // [3][nb]: p_inf, rho_l, c_l
    const double *taup;     // tau = *taup * tau_scale
    double tau_scale;
    double rtol;
    int max_substeps;
    int *nsub;              // accumulated accepted sub-steps per bubble, or null
};

template <bool PW>
__global__ void __launch_bounds__(256) k_el_ode(ElOdeArgs A, Phys ph, Scalars *sc)
{
    const long long nb = A.nb;
    const double tau = *A.taup * A.tau_scale;
    const double vfloor = 1e-3 * sqrt(ph.p0 / ph.rho0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (long long)gridDim.x * blockDim.x) {
        double *b = A.b;
        const double r0 = b[BR0 * nb + i], pg0 = b[BPG * nb + i];
        const double pinf = A.forcing[i], irho = frcp(A.forcing[nb + i]), ic = frcp(A.forcing[2 * nb + i]);
        double y0 = b[BRR * nb + i], y1 = b[BRD * nb + i];
        double h = b[BHS * nb + i];
        if (!(h > 0.0)) h = tau;
        double t = 0.0;
        int acc = 0, att = 0;
        while (t < tau) {
            if (att >= A.max_substeps) {
                raise_error(sc, E_SUBSTEP, i, -1);
                break;
            }
            ++att;
            double hs = h < tau - t ? h : tau - t;
            double r5, v5, r4, v4;
            dp54<PW>(ph, r0, pg0, pinf, irho, ic, y0, y1, hs, r5, v5, r4, v4);
            double err = dmax(fabs(r5 - r4) / fabs(r5), fabs(v5 - v4) / dmax(fabs(v5), vfloor));
            if (!(err == err)) err = INFINITY;
            if (err <= A.rtol && r5 > 0.0) {
                t += hs;
                y0 = r5;
                y1 = v5;
                ++acc;
            }
            double fac = err > 0.0 ? 0.9 * pow(A.rtol / err, 0.2) : 4.0;
            if (!(r5 > 0.0)) fac = 0.25;
            fac = dmin(4.0, dmax(0.25, fac));
            h = hs * fac;
        }
        b[BRR * nb + i] = y0;
        b[BRD * nb + i] = y1;
        b[BHS * nb + i] = h;
        if (A.nsub) A.nsub[i] += acc;
    }
}

// one wavefront per bubble: alpha += V delta, dalpha += 4 pi R^2 Rdot delta
__global__ void __launch_bounds__(256) k_el_scatter(const double *__restrict__ b, long long nb, ElGrid g,
                                                    double *__restrict__ aD)
{
    const int lane = threadIdx.x & 63;
    const long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= nb) return;
    const long long N = g.N;
    int host[3], m;
    double h;
    el_support(b, nb, i, g, host, h, m);
    const double xb[3] = {b[BX_ * nb + i], b[BY_ * nb + i], b[BZ_ * nb + i]};
    const double R = b[BRR * nb + i], V = b[BRD * nb + i];
    const double norm = 0.063493635934240969 / (h * h * h);   // (2 pi)^(-3/2) / h^3
    const double vol = FOUR_PI_3 * R * R * R * norm, rate = 3.0 * FOUR_PI_3 * R * R * V * norm;
    el_visit(g, host, xb, h, m, lane, [&](long long c, double e) {
        atomicAdd(&aD[c], vol * e);
        atomicAdd(&aD[N + c], rate * e);
    });
}

__global__ void k_fill(double *p, long long n, double v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

struct ElStageArgs {
    const double *qk, *qn;
    double *qo;
    const double *P;      // liquid primitives of qk
    const double *aD;     // frozen alpha, dalpha
    const double *dtp;
    double a, b;
    int rhs_mode;
    // RK mode: the epilogue also writes the primitives of the state it produces (the arithmetic of
    // k_el_prim) into Pout, which must not be P; null: the next stage needs a primitive pass.
    double *Pout;
    Scalars *sc;          // error word (with Pout)
    int cfl;              // with Pout: also post the wave-speed maxima of the written state (k_el_prim<true>)
};

// Liquid face between cell (c - e_d) and c from its six-cell stencil st[o][v] (cells c - 3 + o along d,
// primitives rho, u, v, w, p; mirrored ghosts already carry the negated normal velocity): HLLC flux and the
// face-state pressures and normal velocities.
template <int d>
__device__ inline void el_face_flux(const double (&st)[6][5], const Phys &ph, double F[5], double &pL, double &pR,
                                    double &uL, double &uR)
{
    double WL[5], WR[5];
    for (int v = 0; v < 5; ++v) {
        WL[v] = weno5(st[0][v], st[1][v], st[2][v], st[3][v], st[4][v]);
        WR[v] = weno5(st[5][v], st[4][v], st[3][v], st[2][v], st[1][v]);
    }
    if (!(WL[0] > 0.0 && WR[0] > 0.0 && WL[4] + ph.pi_inf > 0.0 && WR[4] + ph.pi_inf > 0.0)) {
        for (int v = 0; v < 5; ++v) {
            WL[v] = st[2][v];
            WR[v] = st[3][v];
        }
    }
    double EK[2], cK[2];
    const double *Ws[2] = {WL, WR};
    for (int s = 0; s < 2; ++s) {
        const double *W = Ws[s];
        EK[s] = (W[4] + ph.gpi) * ph.inv_gm1 + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
        cK[s] = sqrt(ph.gamma * (W[4] + ph.pi_inf) / W[0]);
    }
    double ul = WL[1 + d], ur = WR[1 + d];
    double SL = dmin(ul - cK[0], ur - cK[1]), SR = dmax(ul + cK[0], ur + cK[1]);
    double mL = WL[0] * (SL - ul), mR = WR[0] * (SR - ur);
    double Ss = (WR[4] - WL[4] + ul * mL - ur * mR) / (mL - mR);
    int side, star;
    if (SL >= 0.0) { side = 0; star = 0; }
    else if (Ss >= 0.0) { side = 0; star = 1; }
    else if (SR > 0.0) { side = 1; star = 1; }
    else { side = 1; star = 0; }
    const double *W = side ? WR : WL;
    double SK = side ? SR : SL, un = W[1 + d], ek = EK[side], pk = W[4], rk = W[0];
    double fac = star ? SK * (Ss - un) / (SK - Ss) : 0.0;
    F[0] = rk * un + fac * rk;
    for (int e = 0; e < 3; ++e) F[1 + e] = rk * un * W[1 + e] + (e == d ? pk : 0.0) + fac * rk * (e == d ? SK : W[1 + e]);
    F[4] = (ek + pk) * un + fac * (ek + pk + rk * Ss * (SK - un));
    pL = WL[4];
    pR = WR[4];
    uL = WL[1 + d];
    uR = WR[1 + d];
}

// Tile of the liquid stage: TX x TY x TZ cells, one thread per cell, every face of the tile computed
// once (the faces of direction d form the box T + e_d; at most one per thread in each direction).  For
// each direction the tile's cells and their 3-cell halos along it are first staged in LDS as a "line"
// array (extent T_d + 6 along d), so every face reads its six-cell stencil there at a constant stride;
// mirrored ghosts are stored with the normal velocity negated.
constexpr int ELT_X = 8, ELT_Y = 8, ELT_Z = 3, ELT_BLOCK = 256;

// Index in the line array of direction d of local cell (i, j, k), coordinate d in [-3, T_d + 3).
template <int d>
__device__ __forceinline__ int el_lidx(int i, int j, int k)
{
    if (d == 0) return (k * ELT_Y + j) * (ELT_X + 6) + (i + 3);
    if (d == 1) return (k * (ELT_Y + 6) + (j + 3)) * ELT_X + i;
    return ((k + 3) * ELT_Y + j) * ELT_X + i;
}

__global__ void __launch_bounds__(ELT_BLOCK) k_el_stage(ElStageArgs A, ElGrid g, Phys ph, int ntx, int nty, int ntiles,
                                                        int per_xcd)
{
    constexpr int TX = ELT_X, TY = ELT_Y, TZ = ELT_Z, T = TX * TY * TZ;
    constexpr int FMAX = TX * TY * (TZ + 1) > (TX + 1) * TY * TZ ? TX * TY * (TZ + 1) : (TX + 1) * TY * TZ;
    constexpr int LMAX = TX * TY * (TZ + 6) > (TX + 6) * TY * TZ ? TX * TY * (TZ + 6) : (TX + 6) * TY * TZ;
    // per face: flux[5], the face pressure (p_L + p_R)/2 and (p_L u_L + p_R u_R)/2; with the line
    // array 37 KB, so four workgroups (16 waves) fit a CU's LDS
    __shared__ double s_f[7][FMAX];
    __shared__ double s_l[5][LMAX];    // line array of the current direction: rho, u, v, w, p
    const long long N = g.N;
    const int tid = threadIdx.x;
    // XCD-aware order: blocks are dealt round-robin over the 8 XCDs, so block b takes tile
    // (b mod 8) per_xcd + b / 8 and neighbouring tiles (which share halos) share an XCD's L2
    const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= ntiles) return;
    const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
    const int li = tid % TX, lj = (tid / TX) % TY, lk = tid / (TX * TY);
    const int co[3] = {x0 + li, y0 + lj, z0 + lk};
    const bool active = tid < T && co[0] < g.n[0] && co[1] < g.n[1] && co[2] < g.n[2];
    const long long c = (long long)co[0] + (long long)g.n[0] * ((long long)co[1] + (long long)g.n[1] * co[2]);
    const double dt = A.rhs_mode ? 0.0 : *A.dtp;
    double L[5] = {0, 0, 0, 0, 0}, gradp[3] = {0, 0, 0}, divpu = 0.0;
    auto dir = [&](auto dtag) {
        constexpr int d = decltype(dtag)::value;
        constexpr int EX = TX + 6 * (d == 0), EY = TY + 6 * (d == 1), EZ = TZ + 6 * (d == 2), LD = EX * EY * EZ;
        constexpr int STRIDE = d == 0 ? 1 : (d == 1 ? TX : TX * TY);
        // stage the tile and its halos along d (every coordinate through the ghost map; only the
        // mirror along d flips a velocity, the only one the faces of d read across a wall)
        for (int e = tid; e < LD; e += ELT_BLOCK) {
            const int i = e % EX - 3 * (d == 0), j = (e / EX) % EY - 3 * (d == 1), k = e / (EX * EY) - 3 * (d == 2);
            bool fl[3] = {false, false, false};
            const int gx = map_coord(x0 + i, g.n[0], g.bc[0], fl[0]);
            const int gy = map_coord(y0 + j, g.n[1], g.bc[1], fl[1]);
            const int gz = map_coord(z0 + k, g.n[2], g.bc[2], fl[2]);
            const long long gc = (long long)gx + (long long)g.n[0] * ((long long)gy + (long long)g.n[1] * gz);
            const int li_ = el_lidx<d>(i, j, k);
#pragma unroll
            for (int v = 0; v < 5; ++v) s_l[v][li_] = A.P[v * N + gc];
            if (fl[d]) s_l[1 + d][li_] = -s_l[1 + d][li_];
        }
        __syncthreads();
        constexpr int BX = TX + (d == 0), BY = TY + (d == 1), BZ = TZ + (d == 2), FD = BX * BY * BZ;
        for (int t = tid; t < FD; t += ELT_BLOCK) {
            const int fi = t % BX, fj = (t / BX) % BY, fk = t / (BX * BY);
            const int f[3] = {x0 + fi, y0 + fj, z0 + fk};
            // faces of cells outside the grid are not needed (the face at n[d] closes the last cell)
            bool need = true;
            for (int e = 0; e < 3; ++e) need = need && (e == d ? f[e] <= g.n[e] : f[e] < g.n[e]);
            if (!need) continue;
            const int b0 = el_lidx<d>(fi - 3 * (d == 0), fj - 3 * (d == 1), fk - 3 * (d == 2));
            double st[6][5];
#pragma unroll
            for (int o = 0; o < 6; ++o)
#pragma unroll
                for (int v = 0; v < 5; ++v) st[o][v] = s_l[v][b0 + o * STRIDE];
            double F[5], pl, pr, ul, ur;
            el_face_flux<d>(st, ph, F, pl, pr, ul, ur);
            for (int k = 0; k < 5; ++k) s_f[k][t] = F[k];
            s_f[5][t] = 0.5 * (pl + pr);
            s_f[6][t] = 0.5 * (pl * ul + pr * ur);
        }
        __syncthreads();
        if (active) {
            const int lo = li + BX * (lj + BY * lk);
            const int hi = lo + (d == 0 ? 1 : (d == 1 ? BX : BX * BY));
#pragma unroll
            for (int k = 0; k < 5; ++k) L[k] += (s_f[k][lo] - s_f[k][hi]) * g.inv_dx;
            gradp[d] = (s_f[5][hi] - s_f[5][lo]) * g.inv_dx;
            divpu += (s_f[6][hi] - s_f[6][lo]) * g.inv_dx;
        }
        __syncthreads();   // s_l and s_f are rewritten by the next direction
    };
    dir(std::integral_constant<int, 0>{});
    dir(std::integral_constant<int, 1>{});
    dir(std::integral_constant<int, 2>{});
    double wcfl = 0.0;   // inactive lanes stay in the wave for the maxima's reduction
    if (active) {
        double rho = A.P[c], E = A.qk[4 * N + c];
        double a = A.aD[c], D = A.aD[N + c];
        double ioma = 1.0 / (1.0 - a);
        L[0] += rho * D * ioma;
        for (int d = 0; d < 3; ++d) L[1 + d] += rho * A.P[(1 + d) * N + c] * D * ioma - a * gradp[d] * ioma;
        L[4] += E * D * ioma - a * divpu * ioma;
        double out[5];
        for (int k = 0; k < 5; ++k) {
            long long o = (long long)k * N + c;
            if (A.rhs_mode) out[k] = L[k];
            else {
                out[k] = A.b * (A.qk[o] + dt * L[k]);
                if (A.a != 0.0) out[k] += A.a * A.qn[o];
            }
            A.qo[o] = out[k];
        }
        if (A.Pout) {
            const double rn = out[0], irn = frcp(rn);
            double un[3], ke = 0.0;
            for (int d = 0; d < 3; ++d) {
                un[d] = out[1 + d] * irn;
                ke += un[d] * un[d];
            }
            const double pn = ph.gm1 * (out[4] - 0.5 * rn * ke) - ph.gpi;
            A.Pout[c] = rn;
            for (int d = 0; d < 3; ++d) A.Pout[(1 + d) * N + c] = un[d];
            A.Pout[4 * N + c] = pn;
            if (!(rn > 0.0) || !(pn + ph.pi_inf > 0.0)) raise_error(A.sc, E_NONFINITE, c, -1);
            if (A.cfl) {
                const double cs = sqrt(ph.gamma * (pn + ph.pi_inf) * irn);
                for (int d = 0; d < 3; ++d) wcfl = dmax(wcfl, (fabs(un[d]) + cs) * g.inv_dx);
            }
        }
    }
    if (A.cfl) wmax_post(wcfl, A.sc);
}

}  // namespace bub
