// Device building blocks of the ensemble-averaged RHS stage (gfx950).
//
// Every formula here follows the paper: stiffened-gas liquid (eq. eos_liquid),
// mixture pressure (eq. e:pressure), Keller--Miksis with polytropic or transfer
// contents (eq. keller_miksis, eq. massVaporRate and the contents-pressure
// equation), WENO5 reconstruction and HLLC fluxes (Sec. 3).  The
// arithmetic is arranged for the GPU (one reciprocal per WENO weight set,
// products instead of divisions where the value is unchanged), so results
// agree with a plain evaluation to rounding, not bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bub {

constexpr int NB_MAX = 63;
constexpr double FOUR_PI_3 = 4.18879020478639098461685784437;  // 4 pi / 3
constexpr double FOUR_PI = 12.5663706143591729538505735331;    // 4 pi

// Bubble contents of a context, compiled into the kernels that need them: polytropic gas with the
// general power, polytropic gas with the fifth-root power (3 kappa a whole number of fifths), or gas and
// vapour with heat and vapour transfer at the wall (four state fields per bin instead of two).
enum Contents : int { CT_POLY = 0, CT_FIFTHS = 1, CT_TRANSFER = 2 };

// Physical constants, passed by value (kernel argument segment -> SGPRs).
struct Phys {
    double gamma, pi_inf, gm1, inv_gm1, gpi;  // gpi = gamma * pi_inf
    double kappa3, sigma2, mu4;               // 3 kappa, 2 sigma, 4 mu
    double p0, rho0;
    int pw_c, pw_d;   // 3 kappa = (5 pw_c - pw_d) / 5 for the fifth-root power (pw_c = 0: the general one)
    // transfer contents (CT_TRANSFER): 3 gamma_b, gas constants, wall temperature and vapour pressure,
    // the heat coefficient (gamma_b - 1)/gamma_b k_b beta_T, D_v beta_c, and the products used below
    double g3, Rg, Rv, T0, pv, kh, betaT, dbc, pvRg, RvT0, inv_RgRv2T0;
};

// Grid: cells per direction, boundary kind per direction (0 periodic,
// 1 reflective, 2 non-reflective; both ends equal), inverse spacing.
struct Grid {
    int n[3];
    int bc[3];
    double inv_dx[3];
    long long N;
};

// Bin table in device memory: r0[nb], w[nb], pg0[nb]; with transfer contents also the equilibrium
// contents pressure pb0[nb], vapour mass mv0[nb] and the gas mass mg[nb] of one bubble of each bin.
struct Bins {
    const double *r0, *w, *pg0;
    const double *pb0, *mv0, *mg;
    int nb;
    int nf;        // state fields per bin: 2 (n R, n Rdot) or 4 (and n p_b, n m_v)
    double m3_eq;  // sum w r0^3
};

// The wave-speed max is gathered in WMAX_SLOTS partial maxima, one per 128-byte line, each
// workgroup posting to slot blockIdx % WMAX_SLOTS: with one counter, the one atomic per wave of
// a large grid (10^5 waves) queues at a single address.
constexpr int WMAX_SLOTS = 64, WMAX_STRIDE = 16;

// Device scalars of one context.
struct Scalars {
    double dt;                // step used by the last rk3_step
    int err_code;             // sticky first error (0 = none)
    int err_bin;
    long long err_cell;
    double t;                 // time at the start of the current step (the stages' clock)
    double t_next;            // time of the state after the last step (the context's clock)
    long long pad_[11];
    // bit patterns of partial maxima of (|u_d| + c)/dx_d (positive doubles order as integers)
    unsigned long long wmax[WMAX_SLOTS * WMAX_STRIDE];
};

// Wavefront max of the CFL wave speed, then one atomic per wave into this workgroup's slot.
__device__ inline void wmax_post(double w, Scalars *sc)
{
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(w, off, 64);
        w = o > w ? o : w;
    }
    if ((threadIdx.x & 63) == 0 && w > 0.0)
        atomicMax(&sc->wmax[(blockIdx.x % WMAX_SLOTS) * WMAX_STRIDE], (unsigned long long)__double_as_longlong(w));
}

enum { E_NONFINITE = -4, E_NEGR = -5, E_SUBSTEP = -6 };

__device__ inline void raise_error(Scalars *s, int code, long long cell, int bin)
{
    if (atomicCAS(&s->err_code, 0, code) == 0) {
        s->err_cell = cell;
        s->err_bin = bin;
    }
}

// Ghost-cell map of one coordinate.  Periodic: wrap.  Reflective: fold with
// period 2n (one mirror per wall crossing); `flip` toggles on every mirror so
// the normal velocity of the ghost is negated.  Non-reflective (Sec. 5.1, after
// Thompson): the boundary cell itself, so the Riemann problem at the boundary
// face has no jump and no wave enters from outside.
__host__ __device__ inline int map_coord(int i, int n, int bc, bool &flip)
{
    if ((unsigned)i < (unsigned)n) return i;
    if (bc == 0) {
        int m = i % n;
        return m < 0 ? m + n : m;
    }
    if (bc == 2) return i < 0 ? 0 : n - 1;   // non-reflective: the boundary cell's own state
    int p = 2 * n;
    int m = i % p;
    if (m < 0) m += p;
    if (m >= n) {
        m = p - 1 - m;
        flip = !flip;
    }
    return m;
}

// 1/x to full FP64 precision: hardware reciprocal estimate refined by two
// Newton steps (x finite and nonzero).  Cheaper than an IEEE division; agrees
// with 1/x to about one ulp.
__device__ inline double frcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

// The same with one Newton step: the estimate is good to about 2^-24, one step leaves at most
// 11 ulp (measured on 4M inputs over 2^+-60; two steps: exact).  For the WENO5 weight sum, whose
// reciprocal scales weights that sum to one.
__device__ inline double frcp1(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    return fma(fma(-x, r, 1.0), r, r);
}

// x^p in FP64 for the polytropic gas pressure (R0/R)^(3 kappa) of a bubble, about 65 vector
// instructions against about 110 for the library power (which carries its logarithm in
// double-double arithmetic).  Textbook reductions (e.g. J.-M. Muller, Elementary Functions,
// 3rd ed., 2016):
//   ln x: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m-1)/(m+1),
//         |s| < 0.172, by the odd series of atanh up to s^23 (the next term is below 1e-17
//         of the sum); e ln 2 with ln 2 split in a 32-bit head and a tail.  The leading
//         parts (2s and e ln 2) and the product p ln x keep their rounding errors as a
//         second word, so y = p ln x is known to about 2^-60 relative.
//   e^y:  y = k ln 2 + r, |r| <= ln2 / 2, reduced with the same split (Cody and Waite), e^r
//         by its Taylor series up to r^14 (next term below 5e-18), scaled by 2^k.
// Measured against an 80-bit reference: at most 1.2 ulp for x in [e^-160, e^160].
// The series coefficients and constants come from table C (PPOW_TABLE, copied to LDS by the
// caller): as literals the compiler keeps all of them in registers across the caller's loop.
// Zero, infinite, negative or NaN x take the special values of pow.
constexpr int PPOW_N = 28;
constexpr double PPOW_TABLE[PPOW_N] = {
    1.0 / 23.0, 1.0 / 21.0, 1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0, 1.0 / 9.0, 1.0 / 7.0,
    1.0 / 5.0, 1.0 / 3.0,                                                  // atanh series, 0..10
    1.0 / 87178291200.0, 1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0,
    1.0 / 362880.0, 1.0 / 40320.0, 1.0 / 5040.0, 1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0,
    0.5,                                                                   // 1/14! .. 1/2!, 11..23
    6.93147180369123816490e-01,   // LN2_HI = 0x3FE62E42FEE00000: k * LN2_HI is exact, 24
    1.90821492927058770002e-10,   // LN2_LO = ln 2 - LN2_HI, 25
    1.44269504088896338700e+00,   // log2(e), 26
    0.70710678118654752440};      // sqrt(1/2), 27

__device__ inline double ppow(double x, double p, const double *__restrict__ C)
{
    // (a class test: x - x == 0 would be contracted into fma(a, b, -x) when x = a * b)
    if (!(x > 0.0) || __builtin_isinf(x)) {
        if (x == 0.0) return p > 0.0 ? 0.0 : (p == 0.0 ? 1.0 : __builtin_huge_val());
        if (x > 0.0) return p > 0.0 ? x : (p == 0.0 ? 1.0 : 0.0);
        return __builtin_nan("");
    }
    int e;
    double m = frexp(x, &e);
    if (m < C[27]) {
        m += m;
        e -= 1;
    }
    // s = f / u with f = m - 1 (exact) and u = m + 1 as a rounded head plus its exact error
    const double f = m - 1.0, u = m + 1.0, ulo = m - (u - 1.0);
    const double iu = frcp(u);
    const double sh = f * iu;
    const double sl = (fma(-sh, u, f) - sh * ulo) * iu;
    const double s2 = sh * sh;
    double t = C[0];
#pragma unroll
    for (int j = 1; j <= 10; ++j) t = fma(t, s2, C[j]);
    // ln x = e LN2_HI + 2 sh + (e LN2_LO + 2 sl + 2 sh^3 t), the first sum kept exactly
    const double fe = (double)e;
    const double a0 = fe * C[24], b0 = 2.0 * sh;
    const double H = a0 + b0;
    const double bb = H - a0;
    const double L = ((a0 - (H - bb)) + (b0 - bb)) + fma(fe, C[25], 2.0 * sl + 2.0 * sh * s2 * t);
    const double lh = H + L, ll = L - (lh - H);
    // y = p ln x as yh + yl
    const double yh = p * lh;
    const double yl = fma(p, lh, -yh) + p * ll;
    const double k = rint(yh * C[26]);
    const double r = (fma(-k, C[24], yh) - k * C[25]) + yl;
    double q = C[11];
#pragma unroll
    for (int j = 12; j <= 23; ++j) q = fma(q, r, C[j]);
    q = fma(q * r, r, r);                     // e^r - 1
    const int ki = (int)fmax(fmin(k, 2100.0), -2100.0);
    return ldexp(1.0 + q, ki);
}

// x^p for p = (5c - d)/5, c >= 1 and 0 <= d <= 4 (the polytropic power 3 kappa of kappa = 1, 1.4, 5/3,
// ...), as x^c z^d with z = x^(-1/5): Newton's iteration on x z^5 = 1, z <- z (6 - x z^5) / 5, converges
// quadratically without a division; it starts from the FP32 hardware log2 / exp2 estimate (relative error
// below 2e-6 for x in [1e-30, 1e30]) and takes two steps (below 1e-20 before rounding).  Measured against
// an 80-bit reference: at most 14 ulp for p = 4.2 over x in [e^-8, e^8], the error of z^4 (the general
// power is within 1.2 ulp, at about three times the instructions).  x must lie in [1e-30, 1e30].
__device__ __forceinline__ double pow_fifths(double x, int c, int d)
{
    double z = (double)__builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf((float)x));
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double z2 = z * z, z4 = z2 * z2;
        z = (z * 0.2) * fma(-x, z4 * z, 6.0);
    }
    if (c == 5 && d == 4) {   // air, 3 kappa = 21/5: straight-line powers (the branch is uniform)
        const double x2 = x * x, z2 = z * z;
        return ((x2 * x2) * x) * (z2 * z2);
    }
    double xc = 1.0, b = x;
    for (int e = c; e; e >>= 1) {
        if (e & 1) xc *= b;
        b *= b;
    }
    double zd = 1.0;
    for (int k = 0; k < d; ++k) zd *= z;
    return xc * zd;
}

// The polytropic power x^(3 kappa) of a bubble's contents.  PW: the fifth-root form, for contexts whose
// 3 kappa is a whole number of fifths; it needs x in float's normal range and returns NaN for x <= 0 (a
// ratio no admissible state has).  Otherwise ppow (table C in LDS) or, with C null, the library's
// exp2(p log2 x).  The form is a template parameter of the kernels, not a branch: a branch kept both
// forms' registers live through the callers' bin loops (the 2D stage kernel went from 128 to 162 VGPRs
// and lost a wave per SIMD).
template <bool PW>
__device__ __forceinline__ double kpow(double x, const Phys &ph, const double *__restrict__ C)
{
    if constexpr (PW) return pow_fifths(x, ph.pw_c, ph.pw_d);
    else return C ? ppow(x, ph.kappa3, C) : exp2(ph.kappa3 * log2(x));
}

// WENO5-JS face value at the right face of v2 from v0..v4 (cells i-2..i+2).
// The nonlinear weights d_k/(eps+beta_k)^2 are normalised through products over
// the other two indicators, so one reciprocal serves all three (the FP64 range
// holds them); the linear weights (1/10, 6/10, 3/10) ride on the candidate
// values, whose 1/6 is folded into their coefficients, and eps into the
// indicator's last fused multiply-add.
__device__ inline double weno5(double v0, double v1, double v2, double v3, double v4)
{
    const double eps = 1e-16;
    const double c1312 = 13.0 / 12.0;
    // candidate values: q0 = (2 v0 - 7 v1 + 11 v2)/6, 6 q1 = -v1 + 5 v2 + 2 v3, 3 q2 = (2 v2 + 5 v3 - v4)/2
    double q0 = fma(1.0 / 3.0, v0, fma(-7.0 / 6.0, v1, (11.0 / 6.0) * v2));
    double q1x6 = fma(2.0, v3, fma(5.0, v2, -v1));
    double q2x3 = fma(-0.5, v4, fma(2.5, v3, v2));
    double d0 = fma(-2.0, v1, v0) + v2, e0 = fma(3.0, v2, fma(-4.0, v1, v0));
    double d1 = fma(-2.0, v2, v1) + v3, e1 = v1 - v3;
    double d2 = fma(-2.0, v3, v2) + v4, e2 = fma(-4.0, v3, fma(3.0, v2, v4));
    double s0 = fma(c1312 * d0, d0, fma(0.25 * e0, e0, eps));
    double s1 = fma(c1312 * d1, d1, fma(0.25 * e1, e1, eps));
    double s2 = fma(c1312 * d2, d2, fma(0.25 * e2, e2, eps));
    s0 *= s0;
    s1 *= s1;
    s2 *= s2;
    // a0 : a1 : a2 = 0.1 s1 s2 : 0.6 s0 s2 : 0.3 s0 s1 = p12 : 6 p02 : 3 p01
    double p12 = s1 * s2, p02 = s0 * s2, p01 = s0 * s1;
    double num = fma(p12, q0, fma(p02, q1x6, p01 * q2x3));
    double den = fma(3.0, p01, fma(6.0, p02, p12));
    return num * frcp1(den);
}

// FP32 WENO5-JS for the mixed form: the product form of the FP64 version on
// indicators rescaled into FP32's range (below).  FP32 reciprocals issue at a
// quarter of the rate of other vector instructions, so one reciprocal per
// reconstruction matters here (a ratio form with four took 69 instructions, this
// takes about 52).
__device__ inline float weno5(float v0, float v1, float v2, float v3, float v4)
{
    const float eps = 1e-16f;
    const float c1312 = 13.0f / 12.0f;
    // the FP64 form's candidates and indicators
    float q0 = fmaf(1.0f / 3.0f, v0, fmaf(-7.0f / 6.0f, v1, (11.0f / 6.0f) * v2));
    float q1x6 = fmaf(2.0f, v3, fmaf(5.0f, v2, -v1));
    float q2x3 = fmaf(-0.5f, v4, fmaf(2.5f, v3, v2));
    float d0 = fmaf(-2.0f, v1, v0) + v2, e0 = fmaf(3.0f, v2, fmaf(-4.0f, v1, v0));
    float d1 = fmaf(-2.0f, v2, v1) + v3, e1 = v1 - v3;
    float d2 = fmaf(-2.0f, v3, v2) + v4, e2 = fmaf(-4.0f, v3, fmaf(3.0f, v2, v4));
    float s0 = fmaf(c1312 * d0, d0, fmaf(0.25f * e0, e0, eps));
    float s1 = fmaf(c1312 * d1, d1, fmaf(0.25f * e1, e1, eps));
    float s2 = fmaf(c1312 * d2, d2, fmaf(0.25f * e2, e2, eps));
    // The products of squared indicators leave FP32's range, so each indicator is first divided by
    // the power of two of the smallest (exact: t_i = s_i 2^-e >= 1/2) and held at 2^16 at most: a
    // weight 2^-32 times another is below FP32 resolution, and with t <= 2^16 the products stay
    // below 2^64.  One reciprocal, against one per indicator and one more in a ratio form.
    const int ex = __builtin_amdgcn_frexp_expf(fminf(s0, fminf(s1, s2)));
    float t0 = fminf(__builtin_amdgcn_ldexpf(s0, -ex), 65536.0f);
    float t1 = fminf(__builtin_amdgcn_ldexpf(s1, -ex), 65536.0f);
    float t2 = fminf(__builtin_amdgcn_ldexpf(s2, -ex), 65536.0f);
    t0 *= t0;
    t1 *= t1;
    t2 *= t2;
    // a0 : a1 : a2 = 0.1 t1 t2 : 0.6 t0 t2 : 0.3 t0 t1 = p12 : 6 p02 : 3 p01
    float p12 = t1 * t2, p02 = t0 * t2, p01 = t0 * t1;
    float num = fmaf(p12, q0, fmaf(p02, q1x6, p01 * q2x3));
    float den = fmaf(3.0f, p01, fmaf(6.0f, p02, p12));
    return num * __builtin_amdgcn_rcpf(den);
}

// Reciprocal, square root and division in the reconstruction precision.
__device__ inline double trcp(double x) { return frcp(x); }
__device__ inline float trcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double tsqrt(double x) { return sqrt(x); }
__device__ inline float tsqrt(float x) { return __builtin_sqrtf(x); }
__device__ inline double tdiv(double a, double b) { return a / b; }
__device__ inline float tdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Keller--Miksis wall acceleration (eq. keller_miksis) with polytropic
// contents; the R-ddot part of d(p_bw)/dt that comes from the viscous term is
// moved to the left-hand side (exact rearrangement).
// irho = 1/rho and ic = 1/c of the driving liquid are passed in (shared by all bins of a cell).
template <bool PW>
__device__ inline double km_rddot(const Phys &ph, double R, double V, double r0, double pg0,
                                  double pinf, double irho, double ic)
{
    double iR = frcp(R);
    double pb = pg0 * kpow<PW>(r0 * iR, ph, nullptr);
    double pbw = pb - ph.mu4 * V * iR - ph.sigma2 * iR;
    double dpbw = (-ph.kappa3 * pb * V + ph.mu4 * V * V * iR + ph.sigma2 * V * iR) * iR;
    double irc = irho * ic;
    double num = (1.0 + V * ic) * (pbw - pinf) * irho + R * dpbw * irc - 1.5 * V * V * (1.0 - V * ic * (1.0 / 3.0));
    double den = R * (1.0 - V * ic) + ph.mu4 * irc;
    return num * frcp(den);
}

// The same with the general form of the power from ppow (table C in LDS).
template <bool PW>
__device__ inline double km_rddot_t(const Phys &ph, double R, double V, double r0, double pg0,
                                    double pinf, double irho, double ic, const double *__restrict__ C)
{
    double iR = frcp(R);
    double pb = pg0 * kpow<PW>(r0 * iR, ph, C);
    double pbw = pb - ph.mu4 * V * iR - ph.sigma2 * iR;
    double dpbw = (-ph.kappa3 * pb * V + ph.mu4 * V * V * iR + ph.sigma2 * V * iR) * iR;
    double irc = irho * ic;
    double num = (1.0 + V * ic) * (pbw - pinf) * irho + R * dpbw * irc - 1.5 * V * V * (1.0 - V * ic * (1.0 / 3.0));
    double den = R * (1.0 - V * ic) + ph.mu4 * irc;
    return num * frcp(den);
}

// Transfer contents of one bubble (Sec. 2, eq. massVaporRate and the contents-pressure equation): the
// rates of p_b and m_v for radius R, wall velocity V, pressure p and vapour mass m, gas mass mg.  The
// contents are an ideal-gas mixture at uniform p with mean temperature Tbar = p V_b/(mg Rg + m Rv); the
// wall keeps the liquid temperature T0 with its vapour saturated (partial pressure pv), so with
// S = pv Rg + (p - pv) Rv its vapour mass fraction is chi_w = pv Rg / S and the factor rho_w/(1 - chi_w)
// of the vapour flux is S^2 / (Rg Rv^2 T0 (p - pv)) (rho_w = S/(Rg Rv T0)).  Wall gradients: the transfer
// coefficients times (wall value - bubble mean)/R.
__device__ inline void contents_rates(const Phys &ph, double R, double V, double p, double m, double mg,
                                      double &pdot, double &mdot)
{
    const double iR = frcp(R);
    const double Tbar = p * (FOUR_PI_3 * R * R * R) / (mg * ph.Rg + m * ph.Rv);
    const double chibar = m / (m + mg);
    const double S = ph.pvRg + (p - ph.pv) * ph.Rv;
    const double iS = frcp(S);
    const double chiw = ph.pvRg * iS;
    const double flux = ph.dbc * (S * S * ph.inv_RgRv2T0) / (p - ph.pv) * (chiw - chibar) * iR;
    const double dTdr = ph.betaT * (ph.T0 - Tbar) * iR;
    pdot = ph.g3 * iR * (-V * p + ph.RvT0 * flux + ph.kh * dTdr);
    mdot = FOUR_PI * R * R * flux;
}

// Keller--Miksis wall acceleration for contents of pressure p changing at the rate pdot (transfer
// contents); the R-ddot part of d(p_bw)/dt is moved to the left as above.
__device__ inline double km_rddot_pb(const Phys &ph, double R, double V, double p, double pdot, double pinf,
                                     double irho, double ic)
{
    double iR = frcp(R);
    double pbw = p - ph.mu4 * V * iR - ph.sigma2 * iR;
    double dpbw = pdot + (ph.mu4 * V * V * iR + ph.sigma2 * V * iR) * iR;
    double irc = irho * ic;
    double num = (1.0 + V * ic) * (pbw - pinf) * irho + R * dpbw * irc - 1.5 * V * V * (1.0 - V * ic * (1.0 / 3.0));
    double den = R * (1.0 - V * ic) + ph.mu4 * irc;
    return num * frcp(den);
}

template <typename T>
__device__ inline T dmin(T a, T b) { return a < b ? a : b; }
template <typename T>
__device__ inline T dmax(T a, T b) { return a > b ? a : b; }

}  // namespace bub
