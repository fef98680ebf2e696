// Bubble half-step of the Strang splitting (Sec. 3) for gfx950.
//
// Every (R, Rdot) pair (with transfer contents: (R, Rdot, p_b, m_v)) is
// advanced over tau by Keller--Miksis with its cell's liquid state frozen, using the embedded SSP-RK3 / Heun-RK2 pair that shares
// the first two stages.  A workgroup owns consecutive cells and gives each cell
// S threads: the lanes of a wave hold neighbouring cells of the same bin subset
// (bins slot, slot + S, ...), whose sub-step counts are similar, so divergence
// stays low, and a small problem still spreads over S times more threads than
// cells.  Every attempt counts toward max_substeps, so every lane leaves its
// loop.
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


// Step-size factor 0.9 (rtol/err)^(1/3) of the embedded pair, without the FP64 library power (about a
// hundred instructions, a third of an attempt's work).  The ratio is first held in [0.01, 100], which
// changes no result: outside [0.0214, 87.8] the factor leaves [1/4, 4] and the caller's clamp takes the
// limit either way.  Then z = x^(-1/3) from the FP32 hardware log2 and exp2 and two Newton steps on
// x z^3 = 1, z <- z (4 - x z^3) / 3 (quadratic, no division), and x^(1/3) = x z^2, to a few ulp of the
// library power, so attempts are sized as the oracle sizes them.
__device__ __forceinline__ double step_factor3(double rtol, double err)
{
    const double x = dmin(100.0, dmax(0.01, rtol / err));
    double z = (double)__builtin_amdgcn_exp2f((-1.0f / 3.0f) * __builtin_amdgcn_logf((float)x));
#pragma unroll
    for (int k = 0; k < 2; ++k) z = (z * (1.0 / 3.0)) * fma(-x, z * z * z, 4.0);
    return 0.9 * (x * z * z);
}

// Adaptive integration of one bin over tau: (y0, y1) = (R, Rdot) in, advanced values out.
// Returns the accepted sub-steps; raises E_SUBSTEP when the attempt budget runs out.
template <bool PW>
__device__ inline int bubble_bin(const Phys &ph, double &y0, double &y1, double r0, double pg0, double pl,
                                 double irhol, double ic, double tau, double rtol, double vfloor, int max_substeps,
                                 Scalars *sc, long long c, int i)
{
    double t = 0.0, h = tau;
    int accepted = 0, attempts = 0;
    while (t < tau) {
        if (attempts >= max_substeps) {
            raise_error(sc, E_SUBSTEP, c, i);
            break;
        }
        ++attempts;
        if (h > tau - t) h = tau - t;
        double k1r = y1, k1v = km_rddot<PW>(ph, y0, y1, r0, pg0, pl, irhol, ic);
        double a0 = y0 + h * k1r, a1 = y1 + h * k1v;
        double k2r = a1, k2v = km_rddot<PW>(ph, a0, a1, r0, pg0, pl, irhol, ic);
        double b0 = 0.75 * y0 + 0.25 * (a0 + h * k2r), b1 = 0.75 * y1 + 0.25 * (a1 + h * k2v);
        double e0 = y0 + 0.5 * h * (k1r + k2r), e1 = y1 + 0.5 * h * (k1v + k2v);
        double k3r = b1, k3v = km_rddot<PW>(ph, b0, b1, r0, pg0, pl, irhol, ic);
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
        double fac = err > 0.0 ? step_factor3(rtol, err) : 4.0;
        if (!(n0 > 0.0)) fac = 0.25;
        fac = dmin(4.0, dmax(0.25, fac));
        h *= fac;
    }
    return accepted;
}

// The same pair for transfer contents, y = (R, Rdot, p_b, m_v) of one bubble of gas mass mg; the error
// norm adds |dp_b|/|p_b| and |dm_v|/(|m_v| + mg), and a sub-step needs R > 0 and p_b > 0.
__device__ inline void tr_rates(const Phys &ph, double mg, double pl, double irhol, double ic, const double *y,
                                double *f)
{
    double pdot, mdot;
    contents_rates(ph, y[0], y[1], y[2], y[3], mg, pdot, mdot);
    f[0] = y[1];
    f[1] = km_rddot_pb(ph, y[0], y[1], y[2], pdot, pl, irhol, ic);
    f[2] = pdot;
    f[3] = mdot;
}

__device__ inline int bubble_bin_tr(const Phys &ph, double *y, double mg, double pl, double irhol, double ic,
                                    double tau, double rtol, double vfloor, int max_substeps, Scalars *sc,
                                    long long c, int i)
{
    double t = 0.0, h = tau;
    int accepted = 0, attempts = 0;
    while (t < tau) {
        if (attempts >= max_substeps) {
            raise_error(sc, E_SUBSTEP, c, i);
            break;
        }
        ++attempts;
        if (h > tau - t) h = tau - t;
        double k1[4], k2[4], k3[4], a[4], b[4], e[4], nn[4];
        tr_rates(ph, mg, pl, irhol, ic, y, k1);
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = y[j] + h * k1[j];
        tr_rates(ph, mg, pl, irhol, ic, a, k2);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b[j] = 0.75 * y[j] + 0.25 * (a[j] + h * k2[j]);
            e[j] = y[j] + 0.5 * h * (k1[j] + k2[j]);
        }
        tr_rates(ph, mg, pl, irhol, ic, b, k3);
#pragma unroll
        for (int j = 0; j < 4; ++j) nn[j] = y[j] * (1.0 / 3.0) + (2.0 / 3.0) * (b[j] + h * k3[j]);
        double err = dmax(fabs(nn[0] - e[0]) / fabs(nn[0]), fabs(nn[1] - e[1]) / dmax(fabs(nn[1]), vfloor));
        err = dmax(err, fabs(nn[2] - e[2]) / fabs(nn[2]));
        err = dmax(err, fabs(nn[3] - e[3]) / (fabs(nn[3]) + mg));
        if (!(err == err)) err = INFINITY;
        const bool pos = nn[0] > 0.0 && nn[2] > 0.0;
        if (err <= rtol && pos) {
            t += h;
#pragma unroll
            for (int j = 0; j < 4; ++j) y[j] = nn[j];
            ++accepted;
        }
        double fac = err > 0.0 ? step_factor3(rtol, err) : 4.0;
        if (!pos) fac = 0.25;
        fac = dmin(4.0, dmax(0.25, fac));
        h *= fac;
    }
    return accepted;
}

// One bubble half-step over the whole grid; grid = ceil(N / CELLS) workgroups of CELLS * S
// threads (S threads per cell; S = 1 walks all bins of a cell in one thread).  With S > 1 the
// slots first pool sum w (nR)^3 for n (one barrier), then each advances its bins, posts its part
// of sum w R^3 before and after, and bumps the cell's LDS counter; the slot that arrives last
// updates alpha, so waves whose bins need fewer sub-steps leave without waiting.
// Block `blk` of the half-step (cells blk*CELLS ..); every thread of the workgroup calls it.
template <int D, int S, int CELLS, int CT>
__device__ __forceinline__ void bubble_block(const BubbleArgs &A, const Grid &g, const Phys &ph, const Bins &bins,
                                             Scalars *sc, long long blk)
{
    const int cl = S == 1 ? (int)threadIdx.x : (int)threadIdx.x % CELLS;
    const int slot = S == 1 ? 0 : (int)threadIdx.x / CELLS;
    const long long N = g.N;
    const long long c = blk * CELLS + cl;
    const bool live = c < N;
    const int nb = bins.nb;
    const int iE = D + 1, iA = D + 2, iNR = D + 3, iNV = D + 3 + nb;
    double *q = A.q;
    double a = 0.0, pl = 0.0, irhol = 0.0, ic = 0.0;
    if (live) {
        double rho = q[c];
        a = q[iA * N + c];
        double ke = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double m = q[(1 + d) * N + c];
            ke += m * m;
        }
        ke *= 0.5 / rho;
        double oma = 1.0 - a;
        pl = ph.gm1 * (q[iE * N + c] - ke) / oma - ph.gpi;
        irhol = frcp(rho / oma);
        ic = frcp(sqrt(ph.gamma * (pl + ph.pi_inf) * irhol));
    }
    const bool act = live && a > 0.0;
    // n from sum w (nR)^3
    double s3 = 0.0;
    if (act)
        for (int i = slot; i < nb; i += S) {
            double x = q[(iNR + i) * N + c];
            s3 += bins.w[i] * (x * x * x);
        }
    [[maybe_unused]] double *s_a = nullptr, *s_b = nullptr;
    [[maybe_unused]] unsigned *s_cnt = nullptr;
    if constexpr (S > 1) {
        __shared__ double s_pa[S][CELLS], s_pb[S][CELLS];
        __shared__ unsigned s_pc[CELLS];
        s_a = &s_pa[0][0];
        s_b = &s_pb[0][0];
        s_cnt = s_pc;
        s_a[slot * CELLS + cl] = s3;
        if (slot == 0) s_cnt[cl] = 0u;
        __syncthreads();
        s3 = 0.0;
#pragma unroll
        for (int k = 0; k < S; ++k) s3 += s_a[k * CELLS + cl];
        __syncthreads();   // s_a is reused for the alpha sums
    }
    const double tau = A.taup ? *A.taup * A.tau_scale : A.tau_fixed;
    const double vfloor = 1e-3 * sqrt(ph.p0 / ph.rho0);
    double m3_old = 0.0, m3_new = 0.0;
    if (act) {
        const double n = sqrt(FOUR_PI_3 * s3 / a);
        const double in = frcp(n);
        for (int i = slot; i < nb; i += S) {
            double y0 = q[(iNR + i) * N + c] * in;
            double y1 = q[(iNV + i) * N + c] * in;
            const double wi = bins.w[i];
            m3_old += wi * y0 * y0 * y0;
            int acc;
            if constexpr (CT == CT_TRANSFER) {
                const int iNP = D + 3 + 2 * nb, iNM = D + 3 + 3 * nb;
                double y[4] = {y0, y1, q[(iNP + i) * N + c] * in, q[(iNM + i) * N + c] * in};
                acc = bubble_bin_tr(ph, y, bins.mg[i], pl, irhol, ic, tau, A.rtol, vfloor, A.max_substeps, sc, c, i);
                y0 = y[0];
                y1 = y[1];
                q[(iNP + i) * N + c] = n * y[2];
                q[(iNM + i) * N + c] = n * y[3];
            } else {
                acc = bubble_bin<CT == CT_FIFTHS>(ph, y0, y1, bins.r0[i], bins.pg0[i], pl, irhol, ic, tau, A.rtol,
                                                  vfloor, A.max_substeps, sc, c, i);
            }
            q[(iNR + i) * N + c] = n * y0;
            q[(iNV + i) * N + c] = n * y1;
            m3_new += wi * y0 * y0 * y0;
            if (A.nsub) A.nsub[i * N + c] = acc;
        }
    } else if (live && A.nsub) {
        for (int i = slot; i < nb; i += S) A.nsub[i * N + c] = 0;
    }
    if constexpr (S == 1) {
        if (act) q[iA * N + c] = a * m3_new / m3_old;   // alpha = (4 pi/3) n mean(R^3) at fixed n
    } else {
        s_a[slot * CELLS + cl] = m3_old;
        s_b[slot * CELLS + cl] = m3_new;
        __threadfence_block();
        const unsigned arrived = atomicAdd(&s_cnt[cl], 1u);
        if (arrived == S - 1 && act) {
            __threadfence_block();
            double mo = 0.0, mn = 0.0;
#pragma unroll
            for (int k = 0; k < S; ++k) {
                mo += s_a[k * CELLS + cl];
                mn += s_b[k * CELLS + cl];
            }
            q[iA * N + c] = a * mn / mo;
        }
    }
}

template <int D, int S, int CELLS, int CT>
__global__ void __launch_bounds__(S * CELLS) k_bubble(BubbleArgs A, Grid g, Phys ph, Bins bins, Scalars *sc)
{
    bubble_block<D, S, CELLS, CT>(A, g, ph, bins, sc, blockIdx.x);
}

}  // namespace bub
