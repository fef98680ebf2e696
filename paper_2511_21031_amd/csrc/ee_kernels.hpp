// Ensemble-averaged (Euler--Euler) kernels for gfx950.
//
//  k_init     primitives -> conserved state, bubbles at equilibrium.
//  k_prim     per cell: conserved -> primitive scratch P (rho, u, p_l, alpha,
//             n, B, alpha source), bin moments, optional CFL wave-speed max,
//             or the 8 diagnostic moments.  One thread per cell, coalesced
//             structure-of-arrays loads, each bin read once.
//  k_stage    the fused RK stage on a tile of cells: WENO5 + HLLC of the mixture
//             on every face, then the bins streamed one at a time through LDS
//             (upwind-side WENO5 of R and Rdot, passive HLLC flux,
//             Keller--Miksis source, RK combine, store), with the next bin's
//             global loads in flight while the current bin is reconstructed.
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace bub {

// ---------------------------------------------------------------------------
// Primitive scratch layout P[f][N]
//   0 rho | 1..D u | D+1 p_l | D+2 alpha | D+3 n | D+4 B | D+5 S_alpha
// ---------------------------------------------------------------------------
template <int D>
struct PL {
    static constexpr int RHO = 0, U = 1, PLQ = D + 1, A = D + 2, N = D + 3, B = D + 4, SA = D + 5;
    static constexpr int COUNT = D + 6;
};

enum PrimMode { PRIM_ONLY = 0, PRIM_CFL = 1, PRIM_MOMENTS = 2 };

template <int D, int MODE>
__global__ void __launch_bounds__(256) k_prim(const double *__restrict__ q, double *__restrict__ out,
                                              Grid g, Phys ph, Bins bins, Scalars *sc)
{
    const long long N = g.N;
    const int nb = bins.nb;
    const int iE = D + 1, iA = D + 2, iNR = D + 3, iNV = D + 3 + nb;
    double wmax = 0.0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        double rho = q[c];
        double u[3] = {0.0, 0.0, 0.0};
        double ke = 0.0;
        double irho = frcp(rho);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            u[d] = q[(1 + d) * N + c] * irho;
            ke += u[d] * u[d];
        }
        ke *= 0.5 * rho;
        double E = q[iE * N + c];
        double a = q[iA * N + c];
        double oma = 1.0 - a;
        double pl = ph.gm1 * (E - ke) / oma - ph.gpi;
        double rhol = rho / oma;
        double cs = sqrt(ph.gamma * (pl + ph.pi_inf) / rhol);
        double n = 0.0, B = 0.0, Sa = 0.0;
        double M3 = 0.0, M2d = 0.0, Mp = 0.0, Mk = 0.0;
        bool bad = !(rho > 0.0) || !(a >= 0.0 && a < 1.0) || !(pl + ph.pi_inf > 0.0) || !(cs < 1e300);
        bool negr = false;
        int badbin = -1;
        if (a > 0.0) {
            // One pass over the bins in the conserved variables x = nR, y = nRdot.  With
            // R = x/n and Rdot = y/n every moment is a power of n times a sum that does
            // not involve n, including the contents term:
            //   R^3 p_b(R) = p_g0 R^3 (R0/R)^(3 kappa) = n^(3 kappa - 3) p_g0 x^3 (R0/x)^(3 kappa).
            double s3 = 0.0, s2 = 0.0, s21 = 0.0, s32 = 0.0, sp = 0.0;
#pragma unroll 4
            for (int i = 0; i < nb; ++i) {
                double x = q[(iNR + i) * N + c];
                double y = q[(iNV + i) * N + c];
                if (!(x > 0.0) && !negr) {   // n > 0, so R_i has the sign of (nR)_i
                    negr = true;
                    badbin = i;
                }
                double wi = bins.w[i];
                double x2 = x * x, x3 = x2 * x;
                s3 += wi * x3;
                s2 += wi * x2;
                s21 += wi * x2 * y;
                s32 += wi * x3 * y * y;
                sp += wi * bins.pg0[i] * x3 * exp2(ph.kappa3 * log2(bins.r0[i] * frcp(x)));
            }
            n = sqrt(FOUR_PI_3 * s3 / a);
            double in = frcp(n);
            double in2 = in * in, in3 = in2 * in;
            M3 = s3 * in3;
            M2d = s21 * in3;
            Mk = s32 * in3 * in2;
            Mp = exp2((ph.kappa3 - 3.0) * log2(n)) * sp - ph.mu4 * M2d - ph.sigma2 * s2 * in2;
            double iM3 = frcp(M3);
            B = (Mp - rho * Mk) * iM3;
            Sa = 3.0 * a * M2d * iM3;
        } else {
            for (int i = 0; i < nb; ++i) {
                double r = bins.r0[i];
                M3 += bins.w[i] * r * r * r;
            }
        }
        if (!(B == B) || !(n == n)) bad = true;
        if (negr) raise_error(sc, E_NEGR, c, badbin);   // a negative radius also makes B non-finite
        else if (bad) raise_error(sc, E_NONFINITE, c, -1);
        if (MODE == PRIM_MOMENTS) {
            out[0 * N + c] = n;
            out[1 * N + c] = a;
            out[2 * N + c] = M3;
            out[3 * N + c] = M2d;
            out[4 * N + c] = Mp;
            out[5 * N + c] = Mk;
            out[6 * N + c] = oma * pl + a * B;
            out[7 * N + c] = pl;
        } else {
            out[PL<D>::RHO * N + c] = rho;
#pragma unroll
            for (int d = 0; d < D; ++d) out[(PL<D>::U + d) * N + c] = u[d];
            out[PL<D>::PLQ * N + c] = pl;
            out[PL<D>::A * N + c] = a;
            out[PL<D>::N * N + c] = n;
            out[PL<D>::B * N + c] = B;
            out[PL<D>::SA * N + c] = Sa;
            if (MODE == PRIM_CFL) {
#pragma unroll
                for (int d = 0; d < D; ++d) wmax = dmax(wmax, (fabs(u[d]) + cs) * g.inv_dx[d]);
            }
        }
    }
    if (MODE == PRIM_CFL) {
        // wavefront max, then one atomic per wave on the bit pattern (positive doubles order as integers)
        for (int off = 32; off > 0; off >>= 1) wmax = dmax(wmax, __shfl_xor(wmax, off, 64));
        if ((threadIdx.x & 63) == 0 && wmax > 0.0)
            atomicMax(&sc->wmax, (unsigned long long)__double_as_longlong(wmax));
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_init(const double *__restrict__ prim, double *__restrict__ q,
                                              Grid g, Phys ph, Bins bins)
{
    const long long N = g.N;
    const int nb = bins.nb;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        double rhol = prim[c];
        double pl = prim[(D + 1) * N + c];
        double a = prim[(D + 2) * N + c];
        double rho = (1.0 - a) * rhol;
        double ke = 0.0;
        q[c] = rho;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double u = prim[(1 + d) * N + c];
            q[(1 + d) * N + c] = rho * u;
            ke += u * u;
        }
        q[(D + 1) * N + c] = (1.0 - a) * (pl + ph.gpi) * ph.inv_gm1 + 0.5 * rho * ke;
        q[(D + 2) * N + c] = a;
        double n = a > 0.0 ? a / (FOUR_PI_3 * bins.m3_eq) : 0.0;
        for (int i = 0; i < nb; ++i) {
            q[(D + 3 + i) * N + c] = n * bins.r0[i];
            q[(D + 3 + nb + i) * N + c] = 0.0;
        }
    }
}

// Time step from the wave-speed max (or a fixed value); clears the max for the next step.
__global__ void k_dt(Scalars *sc, double fixed_dt, double cfl, double *user_dt)
{
    double dt = fixed_dt;
    if (!(dt > 0.0)) dt = cfl / __longlong_as_double((long long)sc->wmax);
    sc->dt = dt;
    sc->wmax = 0ull;
    if (user_dt) *user_dt = dt;
}

// ---------------------------------------------------------------------------
// Fused RK stage
// ---------------------------------------------------------------------------

// Tile geometry.  Faces of direction d form the box (T + e_d).  The "cross"
// region holds the tile plus 3-cell halos along each active direction; bins
// are staged into one "line" array per direction d, of extent T_d + 6 along d
// and T_e across, so every face stencil is affine (constant stride).
template <int D, int TX_, int TY_, int TZ_>
struct Geo {
    static constexpr int TX = TX_, TY = (D > 1 ? TY_ : 1), TZ = (D > 2 ? TZ_ : 1);
    static constexpr int T = TX * TY * TZ;
    static constexpr int FX = (TX + 1) * TY * TZ;
    static constexpr int FY = D > 1 ? TX * (TY + 1) * TZ : 0;
    static constexpr int FZ = D > 2 ? TX * TY * (TZ + 1) : 0;
    static constexpr int F = FX + FY + FZ;
    static constexpr int OFF[3] = {0, FX, FX + FY};
    static constexpr int HX = 3 * TY * TZ, HY = D > 1 ? 3 * TX * TZ : 0, HZ = D > 2 ? 3 * TX * TY : 0;
    static constexpr int C = T + 2 * (HX + HY + HZ);
    static constexpr int NC = D + 5;   // reconstructed core primitives
    static constexpr int NCF = D + 3;  // core fluxes: mass, momentum, energy, alpha
    // line arrays
    static constexpr int LX = (TX + 6) * TY * TZ;
    static constexpr int LY = D > 1 ? TX * (TY + 6) * TZ : 0;
    static constexpr int LZ = D > 2 ? TX * TY * (TZ + 6) : 0;
    static constexpr int LOFF[3] = {0, LX, LX + LY};
    static constexpr int L = LX + LY + LZ;
    static constexpr int LSTRIDE[3] = {1, TX, TX * TY};

    template <int d>
    static constexpr int BX() { return TX + (d == 0); }
    template <int d>
    static constexpr int BY() { return TY + (d == 1); }

    // line-array index of local cell (i,j,k) in the array of direction d
    // (coordinate d may lie in [-3, T_d + 3))
    template <int d>
    __host__ __device__ static inline int lidx(int i, int j, int k)
    {
        if (d == 0) return LOFF[0] + (k * TY + j) * (TX + 6) + (i + 3);
        if (d == 1) return LOFF[1] + (k * (TY + 6) + (j + 3)) * TX + i;
        return LOFF[2] + ((k + 3) * TY + j) * TX + i;
    }

    // local coordinates of cross-region index ci; returns the halo direction
    // (0,1,2) or -1 for a core cell
    __host__ __device__ static inline int cdecode(int ci, int &i, int &j, int &k)
    {
        if (ci < T) {
            i = ci % TX;
            j = (ci / TX) % TY;
            k = ci / (TX * TY);
            return -1;
        }
        ci -= T;
        if (ci < 2 * HX) {
            int hi = ci >= HX;
            if (hi) ci -= HX;
            int r = ci / 3;
            i = (ci % 3) + (hi ? TX : -3);
            j = r % TY;
            k = r / TY;
            return 0;
        }
        ci -= 2 * HX;
        if (ci < 2 * HY) {
            int hi = ci >= HY;
            if (hi) ci -= HY;
            i = ci % TX;
            int r = ci / TX;
            j = (r % 3) + (hi ? TY : -3);
            k = r / 3;
            return 1;
        }
        ci -= 2 * HY;
        int hi = ci >= HZ;
        if (hi) ci -= HZ;
        i = ci % TX;
        j = (ci / TX) % TY;
        k = (ci / (TX * TY)) + (hi ? TZ : -3);
        return 2;
    }
};

// RK combine: out = a * un + b * (uk + dt * L); a == 0 skips un.  RHS mode writes L.
struct StageArgs {
    const double *qk;   // u^(k): stencil source
    const double *qn;   // u^n (own cell only), may equal qk or be null when a == 0
    double *qo;         // output
    const double *P;    // primitive scratch of qk
    const double *dtp;  // device step (RK mode)
    double a, b;
    int rhs_mode;       // 1: write L instead of the combine
    int sources;        // 0: leave bubble source terms out (split mode flux part)
    int ntile[3];
    int nblk_per_xcd;
    int ntiles;
};

template <int D, int TX_, int TY_, int TZ_, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_stage(StageArgs A, Grid g, Phys ph, Bins bins)
{
    using G = Geo<D, TX_, TY_, TZ_>;
    constexpr int T = G::T, F = G::F, C = G::C, NC = G::NC, NCF = G::NCF, L = G::L;
    constexpr int CPT = (C + BLOCK - 1) / BLOCK;  // cross cells staged per thread
    constexpr int SCR = (NCF * F > 2 * L + 2 * F) ? NCF * F : 2 * L + 2 * F;
    __shared__ double s_coef[F];
    __shared__ double s_scr[SCR];
    __shared__ unsigned char s_flag[F];

    // XCD-aware tile order: consecutive tiles land on the same XCD (blocks are dealt round-robin).
    const int b = blockIdx.x;
    const int tile = (b & 7) * A.nblk_per_xcd + (b >> 3);
    if (tile >= A.ntiles) return;
    const int tx = tile % A.ntile[0];
    const int ty = (tile / A.ntile[0]) % A.ntile[1];
    const int tz = tile / (A.ntile[0] * A.ntile[1]);
    const int x0 = tx * G::TX, y0 = ty * G::TY, z0 = tz * G::TZ;
    const long long N = g.N;
    const int nb = bins.nb;
    const int tid = threadIdx.x;

    // ---- per-thread staging plan: global index, 1/n and line-array slots of its cross cells ----
    unsigned st_g[CPT];
    double st_in[CPT];
    int st_l[CPT][D];
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        int ci = tid + r * BLOCK;
        st_g[r] = 0;
        st_in[r] = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) st_l[r][d] = -1;
        if (ci < C) {
            int i, j, k;
            int h = G::cdecode(ci, i, j, k);
            bool f = false;
            int gx = map_coord(x0 + i, g.n[0], g.bc[0], f);
            int gy = D > 1 ? map_coord(y0 + j, g.n[1], g.bc[1], f) : 0;
            int gz = D > 2 ? map_coord(z0 + k, g.n[2], g.bc[2], f) : 0;
            unsigned gi = (unsigned)gx + (unsigned)g.n[0] * ((unsigned)gy + (unsigned)g.n[1] * (unsigned)gz);
            st_g[r] = gi;
            double n = A.P[PL<D>::N * N + gi];
            st_in[r] = n > 0.0 ? frcp(n) : 0.0;
            if (h == 0 || h < 0) st_l[r][0] = G::template lidx<0>(i, j, k);
            if (D > 1 && (h == 1 || h < 0)) st_l[r][D > 1 ? 1 : 0] = G::template lidx<(D > 1 ? 1 : 0)>(i, j, k);
            if (D > 2 && (h == 2 || h < 0)) st_l[r][D > 2 ? 2 : 0] = G::template lidx<(D > 2 ? 2 : 0)>(i, j, k);
        }
    }

    // ---- core faces: WENO5 of the mixture primitives, HLLC ----
    double *s_cf = s_scr;  // [NCF][F]
    auto core_faces = [&](auto dtag) {
        constexpr int d = decltype(dtag)::value;
        constexpr int BX = G::template BX<d>(), BY = G::template BY<d>();
        constexpr int FD = (d == 0) ? G::FX : (d == 1 ? G::FY : G::FZ);
        for (int t = tid; t < FD; t += BLOCK) {
            int fi = t % BX, fj = (t / BX) % BY, fk = t / (BX * BY);
            int lc[3] = {fi, fj, fk};
            int org[3] = {x0, y0, z0};
            // global index of the 6 cells along d (positions f-3 .. f+2)
            unsigned gi6[6];
            bool fl6[6];
            {
                bool fo = false;
                int gt[3];
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    gt[e] = (e < D && e != d) ? map_coord(org[e] + lc[e], g.n[e], g.bc[e], fo) : 0;
#pragma unroll
                for (int o = 0; o < 6; ++o) {
                    bool f = false;
                    int gd = map_coord(org[d] + lc[d] - 3 + o, g.n[d], g.bc[d], f);
                    int cc[3] = {gt[0], gt[1], gt[2]};
                    cc[d] = gd;
                    gi6[o] = (unsigned)cc[0] + (unsigned)g.n[0] * ((unsigned)cc[1] + (unsigned)g.n[1] * (unsigned)cc[2]);
                    fl6[o] = f;
                }
            }
            double WL[NC], WR[NC], WcL[NC], WcR[NC];
#pragma unroll
            for (int v = 0; v < NC; ++v) {
                double s[6];
#pragma unroll
                for (int o = 0; o < 6; ++o) s[o] = A.P[(long long)v * N + gi6[o]];
                if (v == 1 + d) {
#pragma unroll
                    for (int o = 0; o < 6; ++o) s[o] = fl6[o] ? -s[o] : s[o];
                }
                WL[v] = weno5(s[0], s[1], s[2], s[3], s[4]);
                WR[v] = weno5(s[5], s[4], s[3], s[2], s[1]);
                WcL[v] = s[2];
                WcR[v] = s[3];
            }
            constexpr int iPL = D + 1, iA = D + 2, iN = D + 3, iB = D + 4;
            bool ok = WL[0] > 0.0 && WR[0] > 0.0 && WL[iA] >= 0.0 && WL[iA] < 1.0 && WR[iA] >= 0.0 &&
                      WR[iA] < 1.0 && WL[iN] >= 0.0 && WR[iN] >= 0.0 && WL[iPL] + ph.pi_inf > 0.0 &&
                      WR[iPL] + ph.pi_inf > 0.0;
            if (!ok) {
#pragma unroll
                for (int v = 0; v < NC; ++v) {
                    WL[v] = WcL[v];
                    WR[v] = WcR[v];
                }
            }
            // HLLC (Davis speeds, Toro contact speed, difference-form star flux)
            double pK[2], EK[2], cK[2];
            const double *Ws[2] = {WL, WR};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const double *Wk = Ws[s];
                double a = Wk[iA], oma = 1.0 - a;
                double u2 = 0.0;
#pragma unroll
                for (int e = 0; e < D; ++e) u2 += Wk[1 + e] * Wk[1 + e];
                pK[s] = oma * Wk[iPL] + a * Wk[iB];
                EK[s] = oma * (Wk[iPL] + ph.gpi) * ph.inv_gm1 + 0.5 * Wk[0] * u2;
                cK[s] = sqrt(ph.gamma * (Wk[iPL] + ph.pi_inf) * oma / Wk[0]);
            }
            double uL = WL[1 + d], uR = WR[1 + d];
            double SL = dmin(uL - cK[0], uR - cK[1]);
            double SR = dmax(uL + cK[0], uR + cK[1]);
            double mL = WL[0] * (SL - uL), mR = WR[0] * (SR - uR);
            double Ss = (pK[1] - pK[0] + uL * mL - uR * mR) / (mL - mR);
            int side, star;
            if (SL >= 0.0) { side = 0; star = 0; }
            else if (Ss >= 0.0) { side = 0; star = 1; }
            else if (SR > 0.0) { side = 1; star = 1; }
            else { side = 1; star = 0; }
            const double *WK = side ? WR : WL;
            double SK = side ? SR : SL;
            double un = WK[1 + d], rk = WK[0], pk = side ? pK[1] : pK[0], ek = side ? EK[1] : EK[0];
            double fac = star ? SK * (Ss - un) / (SK - Ss) : 0.0;
            double F_[NCF];
            F_[0] = rk * un + fac * rk;
#pragma unroll
            for (int e = 0; e < D; ++e)
                F_[1 + e] = rk * un * WK[1 + e] + (e == d ? pk : 0.0) + fac * rk * (e == d ? SK : WK[1 + e]);
            F_[D + 1] = (ek + pk) * un + fac * (ek + pk + rk * Ss * (SK - un));
            F_[D + 2] = WK[iA] * un + fac * WK[iA];
            const int slot = G::OFF[d] + t;
#pragma unroll
            for (int v = 0; v < NCF; ++v) s_cf[v * F + slot] = F_[v];
            // passive bin flux = coef * phi_K with coef = n_K (u_K + fac)
            s_coef[slot] = WK[iN] * (un + fac);
            s_flag[slot] = (unsigned char)(side | (ok ? 0 : 2));
        }
    };
    core_faces(std::integral_constant<int, 0>{});
    if (D > 1) core_faces(std::integral_constant<int, (D > 1 ? 1 : 0)>{});
    if (D > 2) core_faces(std::integral_constant<int, (D > 2 ? 2 : 0)>{});

    // first bin's global loads go out while the core faces finish
    const int iNR = D + 3, iNV = D + 3 + nb;
    double pre_r[CPT], pre_v[CPT];
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        bool ok = tid + r * BLOCK < C;
        pre_r[r] = ok ? A.qk[(long long)iNR * N + st_g[r]] : 0.0;
        pre_v[r] = ok ? A.qk[(long long)iNV * N + st_g[r]] : 0.0;
    }
    __syncthreads();

    // ---- own cell: core divergence, sources, RK combine ----
    const bool own = tid < T;
    int ci_ = own ? tid : 0;
    int li = ci_ % G::TX, lj = (ci_ / G::TX) % G::TY, lk = ci_ / (G::TX * G::TY);
    const bool active = own && (x0 + li < g.n[0]) && (D < 2 || y0 + lj < g.n[1]) && (D < 3 || z0 + lk < g.n[2]);
    const long long gc = (long long)(x0 + li) + (long long)g.n[0] * ((long long)(y0 + lj) + (long long)g.n[1] * (z0 + lk));
    int flo[3], fhi[3];
    {
        // face slots of the own cell: lo face has the cell's coordinate, hi face +1 along d
        flo[0] = G::OFF[0] + li + (G::TX + 1) * (lj + G::TY * lk);
        fhi[0] = flo[0] + 1;
        flo[1] = D > 1 ? G::OFF[1] + li + G::TX * (lj + (G::TY + 1) * lk) : 0;
        fhi[1] = flo[1] + G::TX;
        flo[2] = D > 2 ? G::OFF[2] + li + G::TX * (lj + G::TY * lk) : 0;
        fhi[2] = flo[2] + G::TX * G::TY;
    }
    const int own_l = G::template lidx<0>(li, lj, lk);
    const double dt = A.rhs_mode ? 0.0 : *A.dtp;
    double own_n = 0.0, own_pl = 0.0, own_irhol = 1.0, own_ic = 1.0;
    if (active) {
        double Lc[NCF];
#pragma unroll
        for (int v = 0; v < NCF; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) acc += (s_cf[v * F + flo[d]] - s_cf[v * F + fhi[d]]) * g.inv_dx[d];
            Lc[v] = acc;
        }
        if (A.sources) Lc[D + 2] += A.P[PL<D>::SA * N + gc];
#pragma unroll
        for (int v = 0; v < NCF; ++v) {
            long long o = (long long)v * N + gc;
            if (A.rhs_mode) A.qo[o] = Lc[v];
            else {
                double r = A.b * (A.qk[o] + dt * Lc[v]);
                if (A.a != 0.0) r += A.a * A.qn[o];
                A.qo[o] = r;
            }
        }
        own_n = A.P[PL<D>::N * N + gc];
        own_pl = A.P[PL<D>::PLQ * N + gc];
        double a = A.P[PL<D>::A * N + gc];
        double rhol = A.P[PL<D>::RHO * N + gc] / (1.0 - a);
        own_irhol = frcp(rhol);
        own_ic = frcp(sqrt(ph.gamma * (own_pl + ph.pi_inf) * own_irhol));
    }
    __syncthreads();  // s_cf is reused below

    // ---- bins, one at a time: stage -> faces -> cells; next bin's loads overlap the faces ----
    double *s_R = s_scr, *s_V = s_scr + L, *s_fR = s_scr + 2 * L, *s_fV = s_scr + 2 * L + F;
    for (int ib = 0; ib < nb; ++ib) {
        const double r0 = bins.r0[ib];
#pragma unroll
        for (int r = 0; r < CPT; ++r) {
            if (tid + r * BLOCK < C) {
                double in = st_in[r];
                double Rv = in > 0.0 ? pre_r[r] * in : r0;
                double Vv = in > 0.0 ? pre_v[r] * in : 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    int l = st_l[r][d];
                    if (l >= 0) {
                        s_R[l] = Rv;
                        s_V[l] = Vv;
                    }
                }
            }
        }
        __syncthreads();
        double own_R = s_R[own_l], own_V = s_V[own_l];
        if (ib + 1 < nb) {
#pragma unroll
            for (int r = 0; r < CPT; ++r) {
                bool ok = tid + r * BLOCK < C;
                pre_r[r] = ok ? A.qk[(long long)(iNR + ib + 1) * N + st_g[r]] : 0.0;
                pre_v[r] = ok ? A.qk[(long long)(iNV + ib + 1) * N + st_g[r]] : 0.0;
            }
        }
        auto bin_faces = [&](auto dtag) {
            constexpr int d = decltype(dtag)::value;
            constexpr int BX = G::template BX<d>(), BY = G::template BY<d>();
            constexpr int FD = (d == 0) ? G::FX : (d == 1 ? G::FY : G::FZ);
            constexpr int S = G::LSTRIDE[d];
            for (int t = tid; t < FD; t += BLOCK) {
                int fi = t % BX, fj = (t / BX) % BY, fk = t / (BX * BY);
                const int slot = G::OFF[d] + t;
                unsigned fl = s_flag[slot];
                bool right = fl & 1;
                // cells f-3 .. f+2 along d start at the face's own coordinates in the line array
                int p[3] = {fi, fj, fk};
                p[d] -= 3;
                const int base = G::template lidx<d>(p[0], p[1], p[2]);
                double r6[6], v6[6];
#pragma unroll
                for (int o = 0; o < 6; ++o) {
                    r6[o] = s_R[base + o * S];
                    v6[o] = s_V[base + o * S];
                }
                // upwind side: L uses cells f-3..f+1, R the mirrored f+2..f-2
                double rr[5], vv[5];
#pragma unroll
                for (int o = 0; o < 5; ++o) {
                    rr[o] = right ? r6[5 - o] : r6[o];
                    vv[o] = right ? v6[5 - o] : v6[o];
                }
                double RK, VK;
                if (fl & 2) {
                    RK = rr[2];
                    VK = vv[2];
                } else {
                    RK = weno5(rr[0], rr[1], rr[2], rr[3], rr[4]);
                    VK = weno5(vv[0], vv[1], vv[2], vv[3], vv[4]);
                    if (!(RK > 0.0)) {
                        RK = rr[2];
                        VK = vv[2];
                    }
                }
                double cf = s_coef[slot];
                s_fR[slot] = cf * RK;
                s_fV[slot] = cf * VK;
            }
        };
        bin_faces(std::integral_constant<int, 0>{});
        if (D > 1) bin_faces(std::integral_constant<int, (D > 1 ? 1 : 0)>{});
        if (D > 2) bin_faces(std::integral_constant<int, (D > 2 ? 2 : 0)>{});
        __syncthreads();
        if (active) {
            double LR = 0.0, LV = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                LR += (s_fR[flo[d]] - s_fR[fhi[d]]) * g.inv_dx[d];
                LV += (s_fV[flo[d]] - s_fV[fhi[d]]) * g.inv_dx[d];
            }
            if (A.sources && own_n > 0.0) {
                LR += own_n * own_V;
                LV += own_n * km_rddot(ph, own_R, own_V, r0, bins.pg0[ib], own_pl, own_irhol, own_ic);
            }
            long long oR = (long long)(iNR + ib) * N + gc, oV = (long long)(iNV + ib) * N + gc;
            if (A.rhs_mode) {
                A.qo[oR] = LR;
                A.qo[oV] = LV;
            } else {
                double xr = A.b * (A.qk[oR] + dt * LR);
                double xv = A.b * (A.qk[oV] + dt * LV);
                if (A.a != 0.0) {
                    xr += A.a * A.qn[oR];
                    xv += A.a * A.qn[oV];
                }
                A.qo[oR] = xr;
                A.qo[oV] = xv;
            }
        }
        // the next bin's staging writes s_R/s_V only after every thread passed the barrier above,
        // and s_fR/s_fV are rewritten only after the next staging barrier.
    }
}

}  // namespace bub
