// One-way planar acoustic source (Sec. 2, source-term forcing of the mass, momentum and energy
// equations) for gfx950.
//
// About the reference liquid state (sound speed c0), forcing the pressure rate with S_p = c0 A(t) g(s),
// the momentum along the emission direction with S_p / c0 and the mass with S_p / c0^2 drives only the
// characteristic that runs along that direction: the plane emits p' = A(t - s/c0) (smoothed by g)
// downstream and nothing upstream.  s is the distance from the plane along its axis, g the normal pdf of
// standard deviation `width` cut at 6 widths, A a sine burst whose amplitude carries the factor
// exp((k width)^2 / 2), k = 2 pi f / c0, that the Gaussian's smoothing takes off a sinusoid.  The energy
// forcing is the change of E that S_p, S_m and S_rho make at fixed alpha:
//   S_E = (1 - alpha) S_p / (gamma - 1) + u.S_m - |u|^2 S_rho / 2.
// It is a pass after a stage kernel (like the viscous one) over the slab of cells that can lie within 6
// widths of the plane; each cell adds scale * S to the state the stage wrote.
#pragma once

#include "device_common.hpp"
#include "ee_kernels.hpp"

namespace bub {

struct Source {
    int dir, sign;          // axis of the plane's normal; +1 / -1: the wave runs toward +axis / -axis
    int lo, m[3];           // the launch covers cells lo .. lo + m[dir] - 1 along dir, all cells across
    double x, width, dx;    // plane position, Gaussian standard deviation, spacing along dir
    double norm;            // 1 / (sqrt(2 pi) width)
    double amp_eff;         // sine amplitude with the smoothing factor
    double omega, t0, dur;  // 2 pi f, start time, burst length (<= 0: continuous)
    double c0, inv_c0;      // reference sound speed and its inverse
    double inv_gm1;         // 1 / (gamma - 1)
};

// qo += scale * S(t).  RK stage (tc >= 0): t = sc->t + tc * sc->dt, scale = b * sc->dt (the stage
// evaluates its right-hand side at the time of its input state: tc = 0, 1, 1/2 for stages 1, 2, 3).
// Right-hand side (tc < 0): t = sc->t_next (the context's clock), scale = 1.
template <int D>
__global__ void __launch_bounds__(256) k_source(const double *__restrict__ P, double *__restrict__ qo, Grid g,
                                                Source S, const Scalars *__restrict__ sc, double tc, double b)
{
    const bool rk = tc >= 0.0;
    const double t = rk ? sc->t + tc * sc->dt : sc->t_next;
    const double scale = rk ? b * sc->dt : 1.0;
    const double tau = t - S.t0;
    if (!(tau >= 0.0) || (S.dur > 0.0 && tau > S.dur)) return;
    const double A = S.amp_eff * sin(S.omega * tau);
    const long long N = g.N;
    const long long total = (long long)S.m[0] * S.m[1] * S.m[2];
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (long long)gridDim.x * blockDim.x) {
        int co[3] = {(int)(k % S.m[0]), (int)((k / S.m[0]) % S.m[1]), (int)(k / ((long long)S.m[0] * S.m[1]))};
        co[S.dir] += S.lo;
        const double s = (co[S.dir] + 0.5) * S.dx - S.x;
        if (fabs(s) > 6.0 * S.width) continue;
        const double z = s / S.width;
        const double gs = exp(-0.5 * (z * z)) * S.norm;
        const long long c = (long long)co[0] + (long long)g.n[0] * ((long long)co[1] + (long long)g.n[1] * co[2]);
        double u2 = 0.0, ud = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double u = P[(long long)(PL<D>::U + d) * N + c];
            u2 += u * u;
            if (d == S.dir) ud = u;
        }
        const double alpha = P[(long long)PL<D>::A * N + c];
        const double Sp = S.c0 * A * gs;
        const double Srho = Sp * S.inv_c0 * S.inv_c0;
        const double Sm = S.sign * Sp * S.inv_c0;
        const double SE = (1.0 - alpha) * Sp * S.inv_gm1 + ud * Sm - 0.5 * u2 * Srho;
        qo[c] += scale * Srho;
        qo[(long long)(1 + S.dir) * N + c] += scale * Sm;
        qo[(long long)(D + 1) * N + c] += scale * SE;
    }
}

}  // namespace bub
