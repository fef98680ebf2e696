// Ensemble-averaged (Euler--Euler) kernels for gfx950.
//
//  k_init     primitives -> conserved state, bubbles at equilibrium.
//  k_prim     per cell: conserved -> primitive scratch P (rho, u, p_l, alpha,
//             n, B, alpha source), bin moments, optional CFL wave-speed max,
//             or the 8 diagnostic moments.  On small grids PRIM_SLOTS threads
//             per cell share its bins (one wave finishes the cells from the
//             slot sums); large grids take one thread per cell.  Coalesced
//             structure-of-arrays loads, each bin read once.
//  k_dt       the step of an rk3_step from the wave-speed max.
// The fused stage kernel is in stage_kernel.hpp.
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

constexpr int PRIM_SLOTS = 8;   // threads per cell in the primitive pass

// Bin sums of the primitive pass in the conserved variables x = nR, y = nRdot.  With R = x/n and
// Rdot = y/n every moment is a power of n times a sum that does not involve n, including the
// contents term
//   R^3 p_b(R) = p_g0 R^3 (R0/R)^(3 kappa) = n^(3 kappa - 3) p_g0 x^3 (R0/x)^(3 kappa),
// or, for transfer contents with z = n p_b in the state, R^3 p_b = n^-4 x^3 z.
// bad = the first bin with x <= 0 (n > 0, so R_i has the sign of x) or z <= 0, or nb.
struct BinSums {
    double s3 = 0.0, s2 = 0.0, s21 = 0.0, s32 = 0.0, sp = 0.0;
    int bad;
};

// One bin's terms added to the sums.  Shared by the primitive pass and the epilogue of the fused
// stage kernel, with its operation order fixed (explicit fused multiply-adds, no contraction), so both
// give bitwise the same primitives.  C: the power's constant table (PPOW_TABLE, in LDS).
template <bool PW>
__device__ __forceinline__ void bin_add(BinSums &r, int i, double x, double y, double w, double pg0, double r0,
                                        int nb, const Phys &ph, const double *__restrict__ C)
{
#pragma clang fp contract(off)
    if (!(x > 0.0) && r.bad == nb) r.bad = i;
    const double x2 = x * x, x3 = x2 * x;
    const double wx2 = w * x2, wx3 = w * x3;
    r.s3 = fma(w, x3, r.s3);
    r.s2 = fma(w, x2, r.s2);
    r.s21 = fma(wx2, y, r.s21);
    r.s32 = fma(wx3 * y, y, r.s32);
    r.sp = fma(wx3 * pg0, kpow<PW>(r0 * frcp(x), ph, C), r.sp);
}

// One bin's terms of transfer contents (z = n p_b).
__device__ __forceinline__ void bin_add_tr(BinSums &r, int i, double x, double y, double z, double w, int nb)
{
#pragma clang fp contract(off)
    if (!(x > 0.0 && z > 0.0) && r.bad == nb) r.bad = i;
    const double x2 = x * x, x3 = x2 * x;
    const double wx2 = w * x2, wx3 = w * x3;
    r.s3 = fma(w, x3, r.s3);
    r.s2 = fma(w, x2, r.s2);
    r.s21 = fma(wx2, y, r.s21);
    r.s32 = fma(wx3 * y, y, r.s32);
    r.sp = fma(wx3, z, r.sp);
}

template <int D, int CT>
__device__ __forceinline__ BinSums bin_sums(const double *__restrict__ q, const Phys &ph, const Bins &bins,
                                            long long N, long long c, int first, int stride,
                                            const double *__restrict__ C)
{
    const int nb = bins.nb, iNR = D + 3, iNV = D + 3 + nb;
    BinSums r;
    r.bad = nb;
    if constexpr (CT == CT_TRANSFER) {
        const int iNP = D + 3 + 2 * nb;
        for (int i = first; i < nb; i += stride)
            bin_add_tr(r, i, q[(iNR + i) * N + c], q[(iNV + i) * N + c], q[(iNP + i) * N + c], bins.w[i], nb);
        return r;
    }
    constexpr bool PW = CT == CT_FIFTHS;
    // The pass is bound by the latency of the bin loads: four bins' values are loaded together,
    // then summed one bin at a time in bin order (scheduling barriers keep the loads grouped and
    // the four sums apart, so registers stay few).
    int i = first;
    for (; i + 3 * stride < nb; i += 4 * stride) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = q[(iNR + i + u * stride) * N + c];
            y[u] = q[(iNV + i + u * stride) * N + c];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            __builtin_amdgcn_sched_barrier(0);
            const int k = i + u * stride;
            bin_add<PW>(r, k, x[u], y[u], bins.w[k], bins.pg0[k], bins.r0[k], nb, ph, C);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    for (; i < nb; i += stride)
        bin_add<PW>(r, i, q[(iNR + i) * N + c], q[(iNV + i) * N + c], bins.w[i], bins.pg0[i], bins.r0[i], nb, ph, C);
    return r;
}

// Mixture primitives of one cell from its conserved mixture variables (rho, rho u, E, alpha):
// u, p_l (eq. eos_liquid through the mixture energy), the liquid sound speed, and whether the
// state is admissible.  Shared by the primitive pass and the fused stage epilogue.
template <int D>
struct CellCore {
    double u[3], pl, cs;
    bool bad;
};

template <int D>
__device__ __forceinline__ CellCore<D> cell_core(double rho, const double *mom, double E, double a, const Phys &ph)
{
#pragma clang fp contract(off)
    CellCore<D> o;
    double ke = 0.0;
    const double irho = frcp(rho);
    o.u[0] = o.u[1] = o.u[2] = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        o.u[d] = mom[d] * irho;
        ke = fma(o.u[d], o.u[d], ke);
    }
    ke *= 0.5 * rho;
    const double oma = 1.0 - a;
    o.pl = ph.gm1 * (E - ke) / oma - ph.gpi;
    const double rhol = rho / oma;
    o.cs = sqrt(ph.gamma * (o.pl + ph.pi_inf) / rhol);
    o.bad = !(rho > 0.0) || !(a >= 0.0 && a < 1.0) || !(o.pl + ph.pi_inf > 0.0) || !(o.cs < 1e300);
    return o;
}

// Bin moments, n, B = (Mp - rho Mk)/M3 (eq. e:pressure) and the alpha source 3 alpha M2d/M3
// (eq. e:alpha) of one cell from its bin sums (eq. e:ndf gives n).
struct CellBins {
    double n, B, Sa, M3, M2d, Mp, Mk;
};

template <int CT>
__device__ __forceinline__ CellBins cell_bins(double rho, double a, const BinSums &t, const Phys &ph, const Bins &bins)
{
#pragma clang fp contract(off)
    CellBins o{};
    if (a > 0.0) {
        o.n = sqrt(FOUR_PI_3 * t.s3 / a);
        const double in = frcp(o.n);
        const double in2 = in * in, in3 = in2 * in;
        o.M3 = t.s3 * in3;
        o.M2d = t.s21 * in3;
        o.Mk = t.s32 * in3 * in2;
        if constexpr (CT == CT_TRANSFER) o.Mp = t.sp * (in3 * in) - ph.mu4 * o.M2d - ph.sigma2 * t.s2 * in2;
        else o.Mp = exp2((ph.kappa3 - 3.0) * log2(o.n)) * t.sp - ph.mu4 * o.M2d - ph.sigma2 * t.s2 * in2;
        const double iM3 = frcp(o.M3);
        o.B = (o.Mp - rho * o.Mk) * iM3;
        o.Sa = 3.0 * a * o.M2d * iM3;
    } else {
        for (int i = 0; i < bins.nb; ++i) {
            const double r = bins.r0[i];
            o.M3 += bins.w[i] * r * r * r;
        }
    }
    return o;
}

// The rest of one cell of the primitive pass, given its bin sums: primitives, moments,
// B, the alpha source, error checks; returns max_d (|u_d| + c)/dx_d in CFL mode (0 otherwise).
template <int D, int MODE, int CT>
__device__ __forceinline__ double prim_finish(const double *__restrict__ q, double *__restrict__ out, const Grid &g,
                                              const Phys &ph, const Bins &bins, Scalars *sc, long long c,
                                              const BinSums &t)
{
    const long long N = g.N;
    const int nb = bins.nb;
    const double rho = q[c];
    double mom[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < D; ++d) mom[d] = q[(1 + d) * N + c];
    const double E = q[(D + 1) * N + c];
    const double a = q[(D + 2) * N + c];
    const CellCore<D> k = cell_core<D>(rho, mom, E, a, ph);
    const CellBins m = cell_bins<CT>(rho, a, t, ph, bins);
    bool bad = k.bad || !(m.B == m.B) || !(m.n == m.n);
    const bool negr = a > 0.0 && t.bad < nb;
    if (negr) raise_error(sc, E_NEGR, c, t.bad);   // a negative radius also makes B non-finite
    else if (bad) raise_error(sc, E_NONFINITE, c, -1);
    double wmax = 0.0;
    if (MODE == PRIM_MOMENTS) {
        out[0 * N + c] = m.n;
        out[1 * N + c] = a;
        out[2 * N + c] = m.M3;
        out[3 * N + c] = m.M2d;
        out[4 * N + c] = m.Mp;
        out[5 * N + c] = m.Mk;
        out[6 * N + c] = (1.0 - a) * k.pl + a * m.B;
        out[7 * N + c] = k.pl;
    } else {
        out[PL<D>::RHO * N + c] = rho;
#pragma unroll
        for (int d = 0; d < D; ++d) out[(PL<D>::U + d) * N + c] = k.u[d];
        out[PL<D>::PLQ * N + c] = k.pl;
        out[PL<D>::A * N + c] = a;
        out[PL<D>::N * N + c] = m.n;
        out[PL<D>::B * N + c] = m.B;
        out[PL<D>::SA * N + c] = m.Sa;
        if (MODE == PRIM_CFL) {
#pragma unroll
            for (int d = 0; d < D; ++d) wmax = dmax(wmax, (fabs(k.u[d]) + k.cs) * g.inv_dx[d]);
        }
    }
    return wmax;
}

// Wavefront max of the CFL wave speed, posted to the workgroup's partial-max slot.
__device__ inline void cfl_reduce(double wmax, Scalars *sc) { wmax_post(wmax, sc); }

// Primitive pass; grid = ceil(N / CELLS) workgroups of CELLS * S threads.  A workgroup owns CELLS
// consecutive cells; thread (cell, slot) sums the bins slot, slot + S, ... (each wave reads
// consecutive cells of one bin).  With S > 1 the slots post their sums to LDS and bump the cell's
// counter; the slot that arrives last finishes the cell from the sums taken in slot order, so
// waves that are done leave without waiting for the others.  S = 1 is one thread per cell (large
// grids, which fill the chip on cells alone).
// Block `blk` of the pass (cells blk*CELLS ..); every thread of the workgroup calls it.  s_pp: the
// power's constant table in LDS, filled by the caller before a barrier.
template <int D, int MODE, int S, int CELLS, int CT>
__device__ __forceinline__ void prim_block(const double *__restrict__ q, double *__restrict__ out, const Grid &g,
                                           const Phys &ph, const Bins &bins, Scalars *sc, long long blk,
                                           const double *__restrict__ s_pp)
{
    const int cl = S == 1 ? (int)threadIdx.x : (int)threadIdx.x % CELLS;
    const int slot = S == 1 ? 0 : (int)threadIdx.x / CELLS;
    const long long N = g.N;
    const long long c = blk * CELLS + cl;
    const bool live = c < N;
    double wmax = 0.0;
    if constexpr (S == 1) {
        BinSums p;
        p.bad = bins.nb;
        if (live && q[(D + 2) * N + c] > 0.0) p = bin_sums<D, CT>(q, ph, bins, N, c, 0, 1, s_pp);
        if (live) wmax = prim_finish<D, MODE, CT>(q, out, g, ph, bins, sc, c, p);
    } else {
        __shared__ double s_sum[5][S][CELLS];
        __shared__ int s_bad[S][CELLS];
        __shared__ unsigned s_cnt[CELLS];
        if (slot == 0) s_cnt[cl] = 0u;
        __syncthreads();
        BinSums p;
        p.bad = bins.nb;
        if (live && q[(D + 2) * N + c] > 0.0) p = bin_sums<D, CT>(q, ph, bins, N, c, slot, S, s_pp);
        s_sum[0][slot][cl] = p.s3;
        s_sum[1][slot][cl] = p.s2;
        s_sum[2][slot][cl] = p.s21;
        s_sum[3][slot][cl] = p.s32;
        s_sum[4][slot][cl] = p.sp;
        s_bad[slot][cl] = p.bad;
        __threadfence_block();
        const unsigned arrived = atomicAdd(&s_cnt[cl], 1u);
        if (arrived == S - 1 && live) {
            __threadfence_block();
            BinSums t;
            t.bad = bins.nb;
#pragma unroll
            for (int k = 0; k < S; ++k) {
                t.s3 += s_sum[0][k][cl];
                t.s2 += s_sum[1][k][cl];
                t.s21 += s_sum[2][k][cl];
                t.s32 += s_sum[3][k][cl];
                t.sp += s_sum[4][k][cl];
                t.bad = s_bad[k][cl] < t.bad ? s_bad[k][cl] : t.bad;
            }
            wmax = prim_finish<D, MODE, CT>(q, out, g, ph, bins, sc, c, t);
        }
    }
    if (MODE == PRIM_CFL) cfl_reduce(wmax, sc);
}

template <int D, int MODE, int S, int CELLS, int CT>
__global__ void __launch_bounds__(S * CELLS) k_prim(const double *__restrict__ q, double *__restrict__ out,
                                                    Grid g, Phys ph, Bins bins, Scalars *sc)
{
    __shared__ double s_pp[PPOW_N];   // constants of the polytropic power
    if (threadIdx.x < PPOW_N) s_pp[threadIdx.x] = PPOW_TABLE[threadIdx.x];
    __syncthreads();
    prim_block<D, MODE, S, CELLS, CT>(q, out, g, ph, bins, sc, blockIdx.x, s_pp);
}

// Threads per cell for a grid of N cells: enough to give about 2^19 threads, at most PRIM_SLOTS.
__host__ __device__ inline int slots_for(long long N)
{
    int s = 1;
    while (s < PRIM_SLOTS && N * s < (1LL << 19)) s *= 2;
    return s;
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
            if (bins.nf == 4) {
                q[(D + 3 + 2 * nb + i) * N + c] = n * bins.pb0[i];
                q[(D + 3 + 3 * nb + i) * N + c] = n * bins.mv0[i];
            }
        }
    }
}

// Time step from the wave-speed max (or a fixed value); clears the partial maxima for the next
// step and advances the clock (t: this step's start, t_next: its end).  One wave of WMAX_SLOTS threads.
__device__ __forceinline__ void dt_block(Scalars *sc, double fixed_dt, double cfl, double *user_dt)
{
    const int i = threadIdx.x;
    unsigned long long m = sc->wmax[i * WMAX_STRIDE];
    sc->wmax[i * WMAX_STRIDE] = 0ull;
    for (int off = WMAX_SLOTS / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if (i == 0) {
        double dt = fixed_dt;
        if (!(dt > 0.0)) dt = cfl / __longlong_as_double((long long)m);
        sc->dt = dt;
        sc->t = sc->t_next;        // the step starts where the last one ended
        sc->t_next = sc->t + dt;
        if (user_dt) *user_dt = dt;
    }
}

__global__ void __launch_bounds__(WMAX_SLOTS) k_dt(Scalars *sc, double fixed_dt, double cfl, double *user_dt)
{
    dt_block(sc, fixed_dt, cfl, user_dt);
}


}  // namespace bub
