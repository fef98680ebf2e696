// Ensemble-averaged (Euler--Euler) kernels for gfx950.
//
//  k_init     primitives -> conserved state, bubbles at equilibrium.
//  k_prim     per cell: conserved -> primitive scratch P (rho, u, p_l, alpha,
//             n, B, alpha source), bin moments, optional CFL wave-speed max,
//             or the 8 diagnostic moments.  One thread per cell, coalesced
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

// One cell of the primitive pass; returns max_d (|u_d| + c)/dx_d in CFL mode (0 otherwise).
template <int D, int MODE>
__device__ __forceinline__ double prim_cell(const double *__restrict__ q, double *__restrict__ out, const Grid &g,
                                            const Phys &ph, const Bins &bins, Scalars *sc, long long c)
{
    const long long N = g.N;
    const int nb = bins.nb;
    const int iE = D + 1, iA = D + 2, iNR = D + 3, iNV = D + 3 + nb;
    double wmax = 0.0;
    {
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
    return wmax;
}

// Wavefront max of the CFL wave speed, then one atomic per wave on the bit
// pattern (positive doubles order as unsigned integers).
__device__ inline void cfl_reduce(double wmax, Scalars *sc)
{
    for (int off = 32; off > 0; off >>= 1) wmax = dmax(wmax, __shfl_xor(wmax, off, 64));
    if ((threadIdx.x & 63) == 0 && wmax > 0.0) atomicMax(&sc->wmax, (unsigned long long)__double_as_longlong(wmax));
}

template <int D, int MODE>
__global__ void __launch_bounds__(256) k_prim(const double *__restrict__ q, double *__restrict__ out,
                                              Grid g, Phys ph, Bins bins, Scalars *sc)
{
    double wmax = 0.0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x)
        wmax = dmax(wmax, prim_cell<D, MODE>(q, out, g, ph, bins, sc, c));
    if (MODE == PRIM_CFL) cfl_reduce(wmax, sc);
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


}  // namespace bub
