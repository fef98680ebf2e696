// The fused RK-stage kernel of the ensemble-averaged model (gfx950).
//
// One workgroup owns a tile of cells.  It computes the WENO5 + HLLC flux of the
// mixture on every face of the tile (all directions), then streams the bins
// one at a time through LDS: stage R = nR/n and Rdot = nRdot/n of the tile and
// its 3-cell halos, reconstruct the upwind side of every face (the passive
// HLLC flux of a bin variable needs only that side), difference the fluxes,
// add the Keller--Miksis source of the owned cell and write the RK combine.
// The next bin's global loads are in flight while the current bin is
// reconstructed.
//
// TF is the reconstruction precision: double (plain FP64) or float (the mixed
// form: reconstruction, Riemann solver and flux differences in FP32; the
// primitive pass, moments, Keller--Miksis and the RK combine stay FP64).
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "ee_kernels.hpp"

namespace bub {

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
    int ngroups;        // workgroups per tile, each taking a contiguous range of bpg bins
    int bpg;            // bins per group (ngroups * bpg >= nb)
    int nitems;         // ntiles * ngroups
    // Fused primitive pass (RK mode, one workgroup per tile): the epilogue writes the primitives of
    // the state it produces into Pout (the layout of P; must not be P) and, with cfl set, posts that
    // state's wave-speed maximum.  Null Pout: the next stage needs a primitive pass of its own.
    double *Pout;
    int cfl;
    Scalars *sc;        // error word and wave-speed maxima of the context
};

// LDS needs of one tile: coef[F] and scr[SCR] of TF, flag[F] bytes.  NF: state fields per bin (2, or 4
// for transfer contents), each with a line array and a face array.
template <int D, int TX_, int TY_, int TZ_, typename TF, int NF = 2>
struct StageLds {
    using G = Geo<D, TX_, TY_, TZ_>;
    // line arrays of R and Rdot are LP apart, a multiple of 64 elements, so one paired LDS
    // access (64-element stride form) serves both
    static constexpr int LP = (G::L + 63) / 64 * 64;
    static constexpr int SCR = (G::NCF * G::F > NF * LP + NF * G::F) ? G::NCF * G::F : NF * LP + NF * G::F;
    static constexpr int BYTES = (G::F + SCR) * (int)sizeof(TF) + G::F;
};

// The work of one tile (every thread of the workgroup calls it).  FUSE: the epilogue carries the
// primitive pass of the state it writes (A.Pout, A.cfl).
template <int D, int TX_, int TY_, int TZ_, int BLOCK, typename TF, bool FUSE, int CT>
// Bins b0 <= ib < b1 are this workgroup's; core_out: it also writes the mixture variables
// (exactly one workgroup per tile does).
__device__ __forceinline__ void stage_tile(const StageArgs &A, const Grid &g, const Phys &ph, const Bins &bins,
                                           int tile, int b0, int b1, bool core_out, TF *__restrict__ s_coef,
                                           TF *__restrict__ s_scr, unsigned char *__restrict__ s_flag,
                                           double *__restrict__ s_out, const double *__restrict__ s_pp)
{
    using G = Geo<D, TX_, TY_, TZ_>;
    constexpr int T = G::T, F = G::F, C = G::C, NC = G::NC, NCF = G::NCF, L = G::L;
    constexpr bool TR = CT == CT_TRANSFER;   // transfer contents: n p_b and n m_v per bin as well
    constexpr bool PW = CT == CT_FIFTHS;
    constexpr int CPT = (C + BLOCK - 1) / BLOCK;  // cross cells staged per thread
    const int tx = tile % A.ntile[0];
    const int ty = (tile / A.ntile[0]) % A.ntile[1];
    const int tz = tile / (A.ntile[0] * A.ntile[1]);
    const int x0 = tx * G::TX, y0 = ty * G::TY, z0 = tz * G::TZ;
    const long long N = g.N;
    const int nb = bins.nb;
    const int tid = threadIdx.x;
    const TF pinf = (TF)ph.pi_inf, gpi = (TF)ph.gpi, igm1 = (TF)ph.inv_gm1, gam = (TF)ph.gamma;

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
    TF *s_cf = s_scr;  // [NCF][F]
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
            TF WL[NC], WR[NC], WcL[NC], WcR[NC];
#pragma unroll
            for (int v = 0; v < NC; ++v) {
                TF s[6];
#pragma unroll
                for (int o = 0; o < 6; ++o) s[o] = (TF)A.P[(long long)v * N + gi6[o]];
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
            bool ok = WL[0] > TF(0) && WR[0] > TF(0) && WL[iA] >= TF(0) && WL[iA] < TF(1) && WR[iA] >= TF(0) &&
                      WR[iA] < TF(1) && WL[iN] >= TF(0) && WR[iN] >= TF(0) && WL[iPL] + pinf > TF(0) &&
                      WR[iPL] + pinf > TF(0);
            if (!ok) {
#pragma unroll
                for (int v = 0; v < NC; ++v) {
                    WL[v] = WcL[v];
                    WR[v] = WcR[v];
                }
            }
            // HLLC (Davis speeds, Toro contact speed, difference-form star flux)
            TF pK[2], EK[2], cK[2];
            const TF *Ws[2] = {WL, WR};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const TF *Wk = Ws[s];
                TF a = Wk[iA], oma = TF(1) - a;
                TF u2 = TF(0);
#pragma unroll
                for (int e = 0; e < D; ++e) u2 += Wk[1 + e] * Wk[1 + e];
                pK[s] = oma * Wk[iPL] + a * Wk[iB];
                EK[s] = oma * (Wk[iPL] + gpi) * igm1 + TF(0.5) * Wk[0] * u2;
                cK[s] = tsqrt(gam * (Wk[iPL] + pinf) * oma * trcp(Wk[0]));
            }
            TF uL = WL[1 + d], uR = WR[1 + d];
            TF SL = dmin(uL - cK[0], uR - cK[1]);
            TF SR = dmax(uL + cK[0], uR + cK[1]);
            TF mL = WL[0] * (SL - uL), mR = WR[0] * (SR - uR);
            TF Ss = tdiv(pK[1] - pK[0] + uL * mL - uR * mR, mL - mR);
            int side, star;
            if (SL >= TF(0)) { side = 0; star = 0; }
            else if (Ss >= TF(0)) { side = 0; star = 1; }
            else if (SR > TF(0)) { side = 1; star = 1; }
            else { side = 1; star = 0; }
            const TF *WK = side ? WR : WL;
            TF SK = side ? SR : SL;
            TF un = WK[1 + d], rk = WK[0], pk = side ? pK[1] : pK[0], ek = side ? EK[1] : EK[0];
            TF fac = star ? tdiv(SK * (Ss - un), SK - Ss) : TF(0);
            TF F_[NCF];
            F_[0] = rk * un + fac * rk;
#pragma unroll
            for (int e = 0; e < D; ++e)
                F_[1 + e] = rk * un * WK[1 + e] + (e == d ? pk : TF(0)) + fac * rk * (e == d ? SK : WK[1 + e]);
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
    const int iNR = D + 3, iNV = D + 3 + nb, iNP = D + 3 + 2 * nb, iNM = D + 3 + 3 * nb;
    double pre_r[CPT], pre_v[CPT];
    [[maybe_unused]] double pre_p[TR ? CPT : 1], pre_m[TR ? CPT : 1];
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        bool ok = tid + r * BLOCK < C;
        pre_r[r] = ok ? A.qk[(long long)(iNR + b0) * N + st_g[r]] : 0.0;
        pre_v[r] = ok ? A.qk[(long long)(iNV + b0) * N + st_g[r]] : 0.0;
        if constexpr (TR) {
            pre_p[r] = ok ? A.qk[(long long)(iNP + b0) * N + st_g[r]] : 0.0;
            pre_m[r] = ok ? A.qk[(long long)(iNM + b0) * N + st_g[r]] : 0.0;
        }
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
    const double dt = A.rhs_mode ? 0.0 : *A.dtp;
    double own_n = 0.0, own_in = 0.0, own_pl = 0.0, own_irhol = 1.0, own_ic = 1.0;
    // fused primitive pass: the owned cell's new rho and alpha, admissibility, wave speed, bin sums
    constexpr bool fuse = FUSE;
    double new_rho = 0.0, new_a = 0.0, wcfl = 0.0;
    bool new_bad = false;
    BinSums acc;
    acc.bad = nb;
    if (active && core_out) {
        TF Lc[NCF];
#pragma unroll
        for (int v = 0; v < NCF; ++v) {
            TF acc = TF(0);
#pragma unroll
            for (int d = 0; d < D; ++d) acc += (s_cf[v * F + flo[d]] - s_cf[v * F + fhi[d]]) * (TF)g.inv_dx[d];
            Lc[v] = acc;
        }
        double nq[NCF];
#pragma unroll
        for (int v = 0; v < NCF; ++v) {
            long long o = (long long)v * N + gc;
            double Lv = (double)Lc[v];
            if (v == D + 2 && A.sources) Lv += A.P[PL<D>::SA * N + gc];
            if (A.rhs_mode) A.qo[o] = Lv;
            else {
                double r = A.b * (A.qk[o] + dt * Lv);
                if (A.a != 0.0) r += A.a * A.qn[o];
                A.qo[o] = r;
                nq[v] = r;
            }
        }
        if constexpr (fuse) {
            const CellCore<D> k = cell_core<D>(nq[0], &nq[1], nq[D + 1], nq[D + 2], ph);
            A.Pout[PL<D>::RHO * N + gc] = nq[0];
#pragma unroll
            for (int d = 0; d < D; ++d) A.Pout[(PL<D>::U + d) * N + gc] = k.u[d];
            A.Pout[PL<D>::PLQ * N + gc] = k.pl;
            A.Pout[PL<D>::A * N + gc] = nq[D + 2];
            new_rho = nq[0];
            new_a = nq[D + 2];
            new_bad = k.bad;
            if (A.cfl) {
#pragma unroll
                for (int d = 0; d < D; ++d) wcfl = dmax(wcfl, (fabs(k.u[d]) + k.cs) * g.inv_dx[d]);
            }
        }
    }
    if (active) {
        own_n = A.P[PL<D>::N * N + gc];
        own_in = own_n > 0.0 ? frcp(own_n) : 0.0;
        own_pl = A.P[PL<D>::PLQ * N + gc];
        double a = A.P[PL<D>::A * N + gc];
        double rhol = A.P[PL<D>::RHO * N + gc] / (1.0 - a);
        own_irhol = frcp(rhol);
        own_ic = frcp(sqrt(ph.gamma * (own_pl + ph.pi_inf) * own_irhol));
    }
    __syncthreads();  // s_cf is reused below

    // ---- bins, one at a time: stage -> faces -> cells; next bin's loads overlap the faces ----
    // The owned cell is slot 0 of this thread's staging plan (cross index tid < T), so its own
    // bin values of u^(k) arrive with the staging loads; its u^n values are fetched one bin ahead too.
    const bool own_un = active && !A.rhs_mode && A.a != 0.0;
    double pre_nr = own_un ? A.qn[(long long)(iNR + b0) * N + gc] : 0.0;
    double pre_nv = own_un ? A.qn[(long long)(iNV + b0) * N + gc] : 0.0;
    [[maybe_unused]] double pre_np = 0.0, pre_nm = 0.0;
    if constexpr (TR) {
        pre_np = own_un ? A.qn[(long long)(iNP + b0) * N + gc] : 0.0;
        pre_nm = own_un ? A.qn[(long long)(iNM + b0) * N + gc] : 0.0;
    }
    constexpr int NF = TR ? 4 : 2;
    constexpr int LP = StageLds<D, TX_, TY_, TZ_, TF, NF>::LP;
    TF *s_R = s_scr, *s_V = s_scr + LP, *s_fR = s_scr + NF * LP, *s_fV = s_scr + NF * LP + F;
    [[maybe_unused]] TF *s_P = s_scr + 2 * LP, *s_M = s_scr + 3 * LP;
    [[maybe_unused]] TF *s_fP = s_scr + NF * LP + 2 * F, *s_fM = s_scr + NF * LP + 3 * F;
    // In 3D the owned cell's two results of a bin wait in this thread's own s_out slots and go
    // to HBM one bin late, ahead of the next bin's loads, so that the wait for those loads at
    // the next staging does not also wait for stores issued just before it (measured: 1-3 %
    // faster in 3D; in 2D the extra registers cost a wave per SIMD, so it stores at once).
    constexpr bool DEFER = D == 3 && !TR;
    for (int ib = b0; ib < b1; ++ib) {
        const double r0 = bins.r0[ib], pg0 = bins.pg0[ib];
        const double own_r = pre_r[0], own_v = pre_v[0], own_nr = pre_nr, own_nv = pre_nv;
        [[maybe_unused]] const double own_p = TR ? pre_p[0] : 0.0, own_m = TR ? pre_m[0] : 0.0;
        [[maybe_unused]] const double own_np = pre_np, own_nm = pre_nm;
#pragma unroll
        for (int r = 0; r < CPT; ++r) {
            if (tid + r * BLOCK < C) {
                double in = st_in[r];
                TF Rv = (TF)(in > 0.0 ? pre_r[r] * in : r0);
                TF Vv = (TF)(in > 0.0 ? pre_v[r] * in : 0.0);
                [[maybe_unused]] TF Pv = TF(0), Mv = TF(0);
                if constexpr (TR) {
                    Pv = (TF)(in > 0.0 ? pre_p[r] * in : bins.pb0[ib]);
                    Mv = (TF)(in > 0.0 ? pre_m[r] * in : bins.mv0[ib]);
                }
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    int l = st_l[r][d];
                    if (l >= 0) {
                        s_R[l] = Rv;
                        s_V[l] = Vv;
                        if constexpr (TR) {
                            s_P[l] = Pv;
                            s_M[l] = Mv;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (DEFER && active && ib > b0) {
            A.qo[(long long)(iNR + ib - 1) * N + gc] = s_out[tid];
            A.qo[(long long)(iNV + ib - 1) * N + gc] = s_out[BLOCK + tid];
        }
        if (ib + 1 < b1) {
            if (own_un) {
                pre_nr = A.qn[(long long)(iNR + ib + 1) * N + gc];
                pre_nv = A.qn[(long long)(iNV + ib + 1) * N + gc];
                if constexpr (TR) {
                    pre_np = A.qn[(long long)(iNP + ib + 1) * N + gc];
                    pre_nm = A.qn[(long long)(iNM + ib + 1) * N + gc];
                }
            }
#pragma unroll
            for (int r = 0; r < CPT; ++r) {
                bool ok = tid + r * BLOCK < C;
                pre_r[r] = ok ? A.qk[(long long)(iNR + ib + 1) * N + st_g[r]] : 0.0;
                pre_v[r] = ok ? A.qk[(long long)(iNV + ib + 1) * N + st_g[r]] : 0.0;
                if constexpr (TR) {
                    pre_p[r] = ok ? A.qk[(long long)(iNP + ib + 1) * N + st_g[r]] : 0.0;
                    pre_m[r] = ok ? A.qk[(long long)(iNM + ib + 1) * N + st_g[r]] : 0.0;
                }
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
                // upwind side only: L reads cells f-3..f+1, R the mirrored f+2..f-2 (a signed stride)
                const int st = right ? base + 5 * S : base;
                const int sd = right ? -S : S;
                TF rr[5], vv[5];
#pragma unroll
                for (int o = 0; o < 5; ++o) {
                    rr[o] = s_R[st + o * sd];
                    vv[o] = s_V[st + o * sd];
                }
                TF RK, VK;
                [[maybe_unused]] TF PK = TF(0), MK = TF(0);
                [[maybe_unused]] TF pp[5], mm[5];
                if constexpr (TR) {
#pragma unroll
                    for (int o = 0; o < 5; ++o) {
                        pp[o] = s_P[st + o * sd];
                        mm[o] = s_M[st + o * sd];
                    }
                }
                if (fl & 2) {
                    RK = rr[2];
                    VK = vv[2];
                    if constexpr (TR) {
                        PK = pp[2];
                        MK = mm[2];
                    }
                } else {
                    RK = weno5(rr[0], rr[1], rr[2], rr[3], rr[4]);
                    VK = weno5(vv[0], vv[1], vv[2], vv[3], vv[4]);
                    if constexpr (TR) {
                        PK = weno5(pp[0], pp[1], pp[2], pp[3], pp[4]);
                        MK = weno5(mm[0], mm[1], mm[2], mm[3], mm[4]);
                    }
                    if (!(RK > TF(0))) {
                        RK = rr[2];
                        VK = vv[2];
                        if constexpr (TR) {
                            PK = pp[2];
                            MK = mm[2];
                        }
                    }
                }
                TF cf = s_coef[slot];
                s_fR[slot] = cf * RK;
                s_fV[slot] = cf * VK;
                if constexpr (TR) {
                    s_fP[slot] = cf * PK;
                    s_fM[slot] = cf * MK;
                }
            }
        };
        bin_faces(std::integral_constant<int, 0>{});
        if (D > 1) bin_faces(std::integral_constant<int, (D > 1 ? 1 : 0)>{});
        if (D > 2) bin_faces(std::integral_constant<int, (D > 2 ? 2 : 0)>{});
        __syncthreads();
        if (active) {
            TF LRf = TF(0), LVf = TF(0);
            [[maybe_unused]] TF LPf = TF(0), LMf = TF(0);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                LRf += (s_fR[flo[d]] - s_fR[fhi[d]]) * (TF)g.inv_dx[d];
                LVf += (s_fV[flo[d]] - s_fV[fhi[d]]) * (TF)g.inv_dx[d];
                if constexpr (TR) {
                    LPf += (s_fP[flo[d]] - s_fP[fhi[d]]) * (TF)g.inv_dx[d];
                    LMf += (s_fM[flo[d]] - s_fM[fhi[d]]) * (TF)g.inv_dx[d];
                }
            }
            double LR = (double)LRf, LV = (double)LVf;
            [[maybe_unused]] double LP_ = (double)LPf, LM_ = (double)LMf;
            const double xr0 = own_r, xv0 = own_v;   // u^(k) of bin ib at the owned cell
            if (A.sources && own_n > 0.0) {
                // Keller--Miksis in FP64 from the FP64 state of the owned cell
                double own_R = xr0 * own_in, own_V = xv0 * own_in;
                LR += own_n * own_V;
                if constexpr (TR) {
                    const double own_P = own_p * own_in, own_M = own_m * own_in;
                    double pdot, mdot;
                    contents_rates(ph, own_R, own_V, own_P, own_M, bins.mg[ib], pdot, mdot);
                    LV += own_n * km_rddot_pb(ph, own_R, own_V, own_P, pdot, own_pl, own_irhol, own_ic);
                    LP_ += own_n * pdot;
                    LM_ += own_n * mdot;
                } else {
                    LV += own_n * km_rddot_t<PW>(ph, own_R, own_V, r0, pg0, own_pl, own_irhol, own_ic, s_pp);
                }
            }
            double xr = LR, xv = LV;
            [[maybe_unused]] double xp = LP_, xm = LM_;
            if (!A.rhs_mode) {
                xr = A.b * (xr0 + dt * LR);
                xv = A.b * (xv0 + dt * LV);
                if constexpr (TR) {
                    xp = A.b * (own_p + dt * LP_);
                    xm = A.b * (own_m + dt * LM_);
                }
                if (A.a != 0.0) {
                    xr += A.a * own_nr;   // u^n of bin ib at the owned cell
                    xv += A.a * own_nv;
                    if constexpr (TR) {
                        xp += A.a * own_np;
                        xm += A.a * own_nm;
                    }
                }
            }
            if constexpr (TR) {
                A.qo[(long long)(iNP + ib) * N + gc] = xp;
                A.qo[(long long)(iNM + ib) * N + gc] = xm;
            }
            if constexpr (fuse) {
                if constexpr (TR) bin_add_tr(acc, ib, xr, xv, xp, bins.w[ib], nb);
                else bin_add<PW>(acc, ib, xr, xv, bins.w[ib], pg0, r0, nb, ph, s_pp);
            }
            if constexpr (DEFER) {
                s_out[tid] = xr;
                s_out[BLOCK + tid] = xv;
            } else {
                A.qo[(long long)(iNR + ib) * N + gc] = xr;
                A.qo[(long long)(iNV + ib) * N + gc] = xv;
            }
        }
        // the next bin's staging writes s_R/s_V only after every thread passed the barrier above,
        // and s_fR/s_fV are rewritten only after the next staging barrier.
    }
    if (DEFER && active && b1 > b0) {
        A.qo[(long long)(iNR + b1 - 1) * N + gc] = s_out[tid];
        A.qo[(long long)(iNV + b1 - 1) * N + gc] = s_out[BLOCK + tid];
    }
    if constexpr (fuse) {
        // the primitive pass of the new state for the owned cell (same arithmetic as k_prim)
        if (active) {
            const CellBins m = cell_bins<CT>(new_rho, new_a, acc, ph, bins);
            A.Pout[PL<D>::N * N + gc] = m.n;
            A.Pout[PL<D>::B * N + gc] = m.B;
            A.Pout[PL<D>::SA * N + gc] = m.Sa;
            const bool bad = new_bad || !(m.B == m.B) || !(m.n == m.n);
            if (new_a > 0.0 && acc.bad < nb) raise_error(A.sc, E_NEGR, gc, acc.bad);
            else if (bad) raise_error(A.sc, E_NONFINITE, gc, -1);
        }
        if (A.cfl) wmax_post(wcfl, A.sc);
    }
    __syncthreads();  // a following tile on this workgroup may reuse the LDS at once
}

// The unfused 1D and 2D kernels of the mixed form with the fifth-root power fit 96 VGPRs without
// spilling and run five waves per SIMD (2D: 4 % faster stage than at four); the FP64 ones, the fused
// ones and those of the other contents would spill.
// The LDS arrays of one stage workgroup, declared in the kernel that uses them.
#define BUB_STAGE_SHARED(D, TX_, TY_, TZ_, BLOCK, TF, NF)                               \
    __shared__ TF s_coef[Geo<D, TX_, TY_, TZ_>::F];                                       \
    __shared__ TF s_scr[StageLds<D, TX_, TY_, TZ_, TF, NF>::SCR];                         \
    __shared__ unsigned char s_flag[Geo<D, TX_, TY_, TZ_>::F];                            \
    __shared__ double s_out[D == 3 ? 2 * BLOCK : 1]; /* 3D: results stored one bin late */ \
    __shared__ double s_pp[PPOW_N];                  /* constants of the polytropic power */ \
    if (threadIdx.x < PPOW_N) s_pp[threadIdx.x] = PPOW_TABLE[threadIdx.x]; /* read after the tile's barriers */

// Work item `item` (a tile, or one bin group of a tile) of a stage.
template <int D, int TX_, int TY_, int TZ_, int BLOCK, typename TF, bool FUSE, int CT>
__device__ __forceinline__ void stage_item(const StageArgs &A, const Grid &g, const Phys &ph, const Bins &bins,
                                           int item, TF *__restrict__ s_coef, TF *__restrict__ s_scr,
                                           unsigned char *__restrict__ s_flag, double *__restrict__ s_out,
                                           const double *__restrict__ s_pp)
{
    const int tile = item / A.ngroups, grp = item - tile * A.ngroups;
    const int b0 = grp * A.bpg, b1 = b0 + A.bpg < bins.nb ? b0 + A.bpg : bins.nb;
    stage_tile<D, TX_, TY_, TZ_, BLOCK, TF, FUSE, CT>(A, g, ph, bins, tile, b0, b1, grp == 0, s_coef, s_scr, s_flag,
                                                      s_out, s_pp);
}

template <int D, int TX_, int TY_, int TZ_, int BLOCK, typename TF, bool FUSE, int CT>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu((D <= 2 && sizeof(TF) == 4 && !FUSE && CT == CT_FIFTHS) ? 5 : 1))) k_stage(StageArgs A, Grid g, Phys ph, Bins bins)
{
    BUB_STAGE_SHARED(D, TX_, TY_, TZ_, BLOCK, TF, (CT == CT_TRANSFER ? 4 : 2))
    // XCD-aware order: consecutive items land on the same XCD (blocks are dealt round-robin), and
    // the bin groups of a tile are consecutive items, so they share that XCD's L2.
    const int b = blockIdx.x;
    const int item = (b & 7) * A.nblk_per_xcd + (b >> 3);
    if (item >= A.nitems) return;
    stage_item<D, TX_, TY_, TZ_, BLOCK, TF, FUSE, CT>(A, g, ph, bins, item, s_coef, s_scr, s_flag, s_out, s_pp);
}

}  // namespace bub
