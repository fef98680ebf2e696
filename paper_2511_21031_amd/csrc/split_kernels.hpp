// Bubble half-step of the Strang splitting (Sec. 3) for gfx950.
//
// One thread per cell walks its bins in order (the paper's per-cell bin loop);
// each (R, Rdot) pair is advanced over tau by Keller--Miksis with the cell's
// liquid state frozen, using the embedded SSP-RK3 / Heun-RK2 pair that shares
// the first two stages.  Lanes of a wave hold neighbouring cells, whose bins
// take similar sub-step counts, so divergence stays low.  Every attempt counts
// toward max_substeps, so every lane leaves the loop.
#pragma once

#include "device_common.hpp"

namespace bub {

struct BubbleArgs {
    double *q;
    const double *taup;   // device step; tau = *taup * tau_scale when taup != null
    double tau_scale;
    double tau_fixed;     // used when taup == null
    double rtol;
    int max_substeps;
    int *nsub;            // [nb][N] accepted sub-steps, or null
};

template <int D>
__device__ __forceinline__ void bubble_cell(const BubbleArgs &A, const Grid &g, const Phys &ph, const Bins &bins,
                                            Scalars *sc, long long c)
{
    const long long N = g.N;
    const int nb = bins.nb;
    const int iE = D + 1, iA = D + 2, iNR = D + 3, iNV = D + 3 + nb;
    const double tau = A.taup ? *A.taup * A.tau_scale : A.tau_fixed;
    const double vfloor = 1e-3 * sqrt(ph.p0 / ph.rho0);
    const double rtol = A.rtol;
    double *q = A.q;
    {
        double rho = q[c];
        double a = q[iA * N + c];
        if (!(a > 0.0)) {
            if (A.nsub)
                for (int i = 0; i < nb; ++i) A.nsub[i * N + c] = 0;
            return;
        }
        double ke = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double m = q[(1 + d) * N + c];
            ke += m * m;
        }
        ke *= 0.5 / rho;
        double oma = 1.0 - a;
        double pl = ph.gm1 * (q[iE * N + c] - ke) / oma - ph.gpi;
        double rhol = rho / oma;
        double irhol = frcp(rhol);
        double ic = frcp(sqrt(ph.gamma * (pl + ph.pi_inf) * irhol));
        double s3 = 0.0;
        for (int i = 0; i < nb; ++i) {
            double x = q[(iNR + i) * N + c];
            s3 += bins.w[i] * (x * x * x);
        }
        double n = sqrt(FOUR_PI_3 * s3 / a);
        double in = frcp(n);
        double m3_old = 0.0, m3_new = 0.0;
        for (int i = 0; i < nb; ++i) {
            const double r0 = bins.r0[i], pg0 = bins.pg0[i];
            double y0 = q[(iNR + i) * N + c] * in;
            double y1 = q[(iNV + i) * N + c] * in;
            m3_old += bins.w[i] * y0 * y0 * y0;
            double t = 0.0, h = tau;
            int accepted = 0, attempts = 0;
            while (t < tau) {
                if (attempts >= A.max_substeps) {
                    raise_error(sc, E_SUBSTEP, c, i);
                    break;
                }
                ++attempts;
                if (h > tau - t) h = tau - t;
                double k1r = y1, k1v = km_rddot(ph, y0, y1, r0, pg0, pl, irhol, ic);
                double a0 = y0 + h * k1r, a1 = y1 + h * k1v;
                double k2r = a1, k2v = km_rddot(ph, a0, a1, r0, pg0, pl, irhol, ic);
                double b0 = 0.75 * y0 + 0.25 * (a0 + h * k2r), b1 = 0.75 * y1 + 0.25 * (a1 + h * k2v);
                double e0 = y0 + 0.5 * h * (k1r + k2r), e1 = y1 + 0.5 * h * (k1v + k2v);
                double k3r = b1, k3v = km_rddot(ph, b0, b1, r0, pg0, pl, irhol, ic);
                double n0 = y0 * (1.0 / 3.0) + (2.0 / 3.0) * (b0 + h * k3r);
                double n1 = y1 * (1.0 / 3.0) + (2.0 / 3.0) * (b1 + h * k3v);
                double err = dmax(fabs(n0 - e0) / fabs(n0), fabs(n1 - e1) / dmax(fabs(n1), vfloor));
                if (!(err == err)) err = INFINITY;
                if (err <= rtol && n0 > 0.0) {
                    t += h;
                    y0 = n0;
                    y1 = n1;
                    ++accepted;
                }
                double fac = err > 0.0 ? 0.9 * pow(rtol / err, 1.0 / 3.0) : 4.0;
                if (!(n0 > 0.0)) fac = 0.25;
                fac = dmin(4.0, dmax(0.25, fac));
                h *= fac;
            }
            q[(iNR + i) * N + c] = n * y0;
            q[(iNV + i) * N + c] = n * y1;
            m3_new += bins.w[i] * y0 * y0 * y0;
            if (A.nsub) A.nsub[i * N + c] = accepted;
        }
        q[iA * N + c] = a * m3_new / m3_old;
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_bubble(BubbleArgs A, Grid g, Phys ph, Bins bins, Scalars *sc)
{
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x)
        bubble_cell<D>(A, g, ph, bins, sc, c);
}

}  // namespace bub
