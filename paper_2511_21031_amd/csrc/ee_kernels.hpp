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

// Bin sums of the primitive pass over bins i = first, first + stride, ... in the
// conserved variables x = nR, y = nRdot.  With R = x/n and Rdot = y/n every moment
// is a power of n times a sum that does not involve n, including the contents term
//   R^3 p_b(R) = p_g0 R^3 (R0/R)^(3 kappa) = n^(3 kappa - 3) p_g0 x^3 (R0/x)^(3 kappa).
// bad = the first bin of the subset with x <= 0 (n > 0, so R_i has the sign of x), or nb.
struct BinSums {
    double s3 = 0.0, s2 = 0.0, s21 = 0.0, s32 = 0.0, sp = 0.0;
    int bad;
};

template <int D>
__device__ __forceinline__ BinSums bin_sums(const double *__restrict__ q, const Phys &ph, const Bins &bins,
                                            long long N, long long c, int first, int stride)
{
    const int nb = bins.nb, iNR = D + 3, iNV = D + 3 + nb;
    BinSums r;
    r.bad = nb;
    auto add = [&](int i, double x, double y) {
        if (!(x > 0.0) && r.bad == nb) r.bad = i;
        double wi = bins.w[i];
        double x2 = x * x, x3 = x2 * x;
        r.s3 += wi * x3;
        r.s2 += wi * x2;
        r.s21 += wi * x2 * y;
        r.s32 += wi * x3 * y * y;
        r.sp += wi * bins.pg0[i] * x3 * exp2(ph.kappa3 * log2(bins.r0[i] * frcp(x)));
    };
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
            add(i + u * stride, x[u], y[u]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    for (; i < nb; i += stride) add(i, q[(iNR + i) * N + c], q[(iNV + i) * N + c]);
    return r;
}

// The rest of one cell of the primitive pass, given its bin sums: primitives, moments,
// B, the alpha source, error checks; returns max_d (|u_d| + c)/dx_d in CFL mode (0 otherwise).
template <int D, int MODE>
__device__ __forceinline__ double prim_finish(const double *__restrict__ q, double *__restrict__ out, const Grid &g,
                                              const Phys &ph, const Bins &bins, Scalars *sc, long long c,
                                              const BinSums &t)
{
    const long long N = g.N;
    const int nb = bins.nb;
    const int iE = D + 1, iA = D + 2;
    double wmax = 0.0;
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
    const bool negr = a > 0.0 && t.bad < nb;
    if (a > 0.0) {
        n = sqrt(FOUR_PI_3 * t.s3 / a);
        double in = frcp(n);
        double in2 = in * in, in3 = in2 * in;
        M3 = t.s3 * in3;
        M2d = t.s21 * in3;
        Mk = t.s32 * in3 * in2;
        Mp = exp2((ph.kappa3 - 3.0) * log2(n)) * t.sp - ph.mu4 * M2d - ph.sigma2 * t.s2 * in2;
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
    if (negr) raise_error(sc, E_NEGR, c, t.bad);   // a negative radius also makes B non-finite
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
template <int D, int MODE, int S, int CELLS>
__global__ void __launch_bounds__(S * CELLS) k_prim(const double *__restrict__ q, double *__restrict__ out,
                                                    Grid g, Phys ph, Bins bins, Scalars *sc)
{
    const int cl = S == 1 ? (int)threadIdx.x : (int)threadIdx.x % CELLS;
    const int slot = S == 1 ? 0 : (int)threadIdx.x / CELLS;
    const long long N = g.N;
    const long long c = (long long)blockIdx.x * CELLS + cl;
    const bool live = c < N;
    double wmax = 0.0;
    if constexpr (S == 1) {
        BinSums p;
        p.bad = bins.nb;
        if (live && q[(D + 2) * N + c] > 0.0) p = bin_sums<D>(q, ph, bins, N, c, 0, 1);
        if (live) wmax = prim_finish<D, MODE>(q, out, g, ph, bins, sc, c, p);
    } else {
        __shared__ double s_sum[5][S][CELLS];
        __shared__ int s_bad[S][CELLS];
        __shared__ unsigned s_cnt[CELLS];
        if (slot == 0) s_cnt[cl] = 0u;
        __syncthreads();
        BinSums p;
        p.bad = bins.nb;
        if (live && q[(D + 2) * N + c] > 0.0) p = bin_sums<D>(q, ph, bins, N, c, slot, S);
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
            wmax = prim_finish<D, MODE>(q, out, g, ph, bins, sc, c, t);
        }
    }
    if (MODE == PRIM_CFL) cfl_reduce(wmax, sc);
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
        }
    }
}

// Time step from the wave-speed max (or a fixed value); clears the partial maxima for the next
// step.  One wave of WMAX_SLOTS threads.
__global__ void __launch_bounds__(WMAX_SLOTS) k_dt(Scalars *sc, double fixed_dt, double cfl, double *user_dt)
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
        if (user_dt) *user_dt = dt;
    }
}


}  // namespace bub
