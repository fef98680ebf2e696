// Viscous stress of the liquid (eq. stressTensor) in the mixture fluxes (gfx950).
//
// T = mu (grad u + grad u^T - 2/3 div(u) I) enters the momentum flux as -T and the energy flux as -T.u
// (eq. euler_transport).  It is a separate pass that runs after a stage kernel when the problem is
// viscous, so the stage kernels carry no code for it: every owned cell forms the viscous fluxes through
// its 2 ndim faces from the velocities of the stage's input state (the primitive scratch P), by
// second-order central differences at the face -- normal derivatives from the two cells beside it,
// transverse derivatives as the mean of those two cells' central differences, face velocity the mean
// of the two cells' -- and adds scale * (F_lo - F_hi)/dx to the momentum and energy the stage wrote
// (scale = b dt of the RK combine, 1 for a right-hand side).  Mirrored ghost cells negate the velocity
// component along the mirrored direction.
#pragma once

#include "device_common.hpp"
#include "ee_kernels.hpp"

namespace bub {

// Velocity of the cell at co + oa e_a (+ ob e_b when b >= 0), through the ghost-cell map.
template <int D>
__device__ __forceinline__ void visc_vel(const double *__restrict__ P, const Grid &g, const int co[3], int a, int oa,
                                         int b, int ob, double u[3])
{
    int cc[3] = {co[0], co[1], co[2]};
    bool fa = false, fb = false;
    cc[a] = map_coord(co[a] + oa, g.n[a], g.bc[a], fa);
    if (b >= 0) cc[b] = map_coord(co[b] + ob, g.n[b], g.bc[b], fb);
    const long long gi = (long long)cc[0] + (long long)g.n[0] * ((long long)cc[1] + (long long)g.n[1] * cc[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = k < D ? P[(long long)(PL<D>::U + k) * g.N + gi] : 0.0;
    if (fa) u[a] = -u[a];
    if (b >= 0 && fb) u[b] = -u[b];
}

// Viscous flux through the face co of direction d (between the cells co - e_d and co):
// F[k] = -T_dk (momentum k), F[D] = -(T.u)_d (energy).
template <int D>
__device__ __forceinline__ void visc_face(const double *__restrict__ P, const Grid &g, double mu, int d,
                                          const int co[3], double F[D + 1])
{
    double uL[3], uR[3], gr[3][3];   // gr[k][e] = d u_k / d x_e at the face
    visc_vel<D>(P, g, co, d, -1, -1, 0, uL);
    visc_vel<D>(P, g, co, d, 0, -1, 0, uR);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int e = 0; e < 3; ++e) gr[k][e] = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) gr[k][d] = (uR[k] - uL[k]) * g.inv_dx[d];
#pragma unroll 1
    for (int e = 0; e < D; ++e) {
        if (e == d) continue;
        double lp[3], lm[3], rp[3], rm[3];
        visc_vel<D>(P, g, co, d, -1, e, 1, lp);
        visc_vel<D>(P, g, co, d, -1, e, -1, lm);
        visc_vel<D>(P, g, co, d, 0, e, 1, rp);
        visc_vel<D>(P, g, co, d, 0, e, -1, rm);
#pragma unroll
        for (int k = 0; k < D; ++k) gr[k][e] = ((lp[k] - lm[k]) + (rp[k] - rm[k])) * (0.25 * g.inv_dx[e]);
    }
    double div = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) div += gr[e][e];
    double work = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double T = mu * (gr[d][k] + gr[k][d] - (k == d ? (2.0 / 3.0) * div : 0.0));
        F[k] = -T;
        work += T * 0.5 * (uL[k] + uR[k]);
    }
    F[D] = -work;
}

// qo (momentum and energy) += scale * viscous rates of every cell; scale = b * (*dtp), or 1 when dtp is null.
template <int D>
__global__ void __launch_bounds__(256) k_viscous(const double *__restrict__ P, double *__restrict__ qo, Grid g,
                                                 double mu, const double *__restrict__ dtp, double b)
{
    const double scale = dtp ? b * *dtp : 1.0;
    const long long N = g.N;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        const int co[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
        double L[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) L[k] = 0.0;
#pragma unroll 1
        for (int d = 0; d < D; ++d) {
            double Flo[D + 1], Fhi[D + 1];
            int hi[3] = {co[0], co[1], co[2]};
            hi[d] += 1;
            visc_face<D>(P, g, mu, d, co, Flo);
            visc_face<D>(P, g, mu, d, hi, Fhi);
#pragma unroll
            for (int k = 0; k <= D; ++k) L[k] += (Flo[k] - Fhi[k]) * g.inv_dx[d];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) qo[(long long)(1 + k) * N + c] += scale * L[k];
        qo[(long long)(D + 1) * N + c] += scale * L[D];
    }
}

}  // namespace bub
