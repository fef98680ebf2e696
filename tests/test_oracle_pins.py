"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms
(Rayleigh collapse, the linearised Keller--Miksis oscillator, Simpson
exactness, polynomial exactness of WENO), an independent exact Riemann solver,
and invariants of the discrete scheme (free stream, conservation, symmetry,
contact at rest, 0D reduction and its order).  None of them needs a GPU.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import workloads as W
from tests import exact_riemann

ATM = W.ATM


def _pb(orc, **kw):
    base = dict(ndim=1, n=(8, 1, 1), dx=(1e-4, 1, 1), bc=((0, 0), (0, 0), (0, 0)), nb=1)
    base.update(kw)
    return orc.problem(**base)


# ---------------------------------------------------------------------------
# Bins (Sec. 2.2: log-normal PDF of R0, Simpson's rule)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nb,sig", [(3, 0.3), (11, 0.3), (21, 0.3), (31, 0.5)])
def test_bins_simpson_pattern(orc, nb, sig):
    r0, w = orc.bins(nb, 10e-6, sig)
    assert abs(w.sum() - 1.0) < 1e-15
    phi = np.log(r0 / 10e-6)
    h = 6 * sig / (nb - 1)
    assert np.allclose(phi, -3 * sig + h * np.arange(nb), rtol=0, atol=1e-14)
    # w_i / pdf(phi_i) must follow the composite Simpson pattern 1,4,2,...,2,4,1
    ratio = w / stats.norm.pdf(phi, scale=sig)
    pattern = np.array([1.0] + [4.0 if i % 2 else 2.0 for i in range(1, nb - 1)] + [1.0])
    assert np.allclose(ratio / ratio[0], pattern, rtol=1e-13)


def test_bins_simpson_exact_for_cubics(orc):
    # Unnormalised Simpson weights (h/3) s_i integrate any cubic exactly on [-3s, 3s].
    nb, sig = 11, 0.3
    r0, w = orc.bins(nb, 1.0, sig)
    phi = np.log(r0)
    f = stats.norm.pdf(phi, scale=sig)
    h = 6 * sig / (nb - 1)
    simpson = w / f * (h / 3) / (w[0] / f[0])     # recover (h/3) s_i
    rng = np.random.default_rng(1)
    c = rng.normal(size=4)
    g = lambda x: c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
    exact = integrate.quad(g, -3 * sig, 3 * sig, epsabs=1e-15)[0]
    assert abs((simpson * g(phi)).sum() - exact) < 1e-13


def test_bins_lognormal_moments_within_simpson_bound(orc):
    """Sum w R0^3 equals the truncated lognormal moment within Simpson's error bound
    (b-a) h^4 max|f4| / 180 (f4 the fourth derivative), applied to numerator and normaliser."""
    sig, rmed = 0.3, 10e-6
    x = np.linspace(-3 * sig, 3 * sig, 20001)
    dxg = x[1] - x[0]

    def d4max(f):
        y = f(x)
        for _ in range(4):
            y = np.gradient(y, dxg)
        return np.abs(y[50:-50]).max()

    fnum = lambda t: np.exp(3 * t) * stats.norm.pdf(t, scale=sig)
    fden = lambda t: stats.norm.pdf(t, scale=sig)
    num = integrate.quad(fnum, -3 * sig, 3 * sig, epsabs=0, epsrel=1e-13)[0]
    den = integrate.quad(fden, -3 * sig, 3 * sig, epsabs=0, epsrel=1e-13)[0]
    errs = []
    for nb in (11, 21, 41):
        r0, w = orc.bins(nb, rmed, sig)
        h = 6 * sig / (nb - 1)
        bound = 6 * sig * h ** 4 / 180 * (2 * d4max(fnum) / num + 2 * d4max(fden) / den)
        err = abs((w * (r0 / rmed) ** 3).sum() / (num / den) - 1.0)
        assert err <= bound, (nb, err, bound)
        errs.append(err)
    assert errs[2] < errs[0] / 100


def test_bins_monodisperse(orc):
    r0, w = orc.bins(1, 7e-6, 0.0)
    assert r0[0] == 7e-6 and w[0] == 1.0


# ---------------------------------------------------------------------------
# Keller--Miksis (eq. keller_miksis)
# ---------------------------------------------------------------------------

def test_km_equilibrium(orc):
    pb = _pb(orc)
    R0 = 10e-6
    pg0 = pb.p0 + 2 * pb.sigma / R0
    c = math.sqrt(pb.gamma * (pb.p0 + pb.pi_inf) / pb.rho0)
    a = orc.km_rddot(pb, R0, 0.0, R0, pg0, pb.p0, pb.rho0, c)
    assert abs(a) * R0 / (pb.p0 / pb.rho0) < 1e-12


def test_km_rayleigh_collapse_time(orc):
    """Empty cavity, incompressible, inviscid: Rayleigh's collapse time."""
    gas = dict(W.AIR, sigma=0.0, mu=0.0)
    pb = _pb(orc, gas=gas)
    R0, dp, rho = 10e-6, ATM, 1000.0
    # Closed form t_c = R0 sqrt(3 rho / 2 dp) B(5/6, 1/2) / 3 = 0.9146814 R0 sqrt(rho/dp)
    tc = R0 * math.sqrt(1.5 * rho / dp) * special.beta(5 / 6, 0.5) / 3.0
    assert abs(tc / (R0 * math.sqrt(rho / dp)) - 0.9146814) < 1e-7
    # Time to reach R = 0.01 R0 from the exact quadrature of the energy integral
    t1 = R0 * math.sqrt(1.5 * rho / dp) * integrate.quad(lambda x: x ** 1.5 / math.sqrt(1 - x ** 3), 0.01, 1,
                                                         epsabs=0, epsrel=1e-12, limit=200)[0]
    assert abs(t1 / tc - (1 - 5.36e-6)) < 2e-8
    _, _, tstop, steps = orc.km_integrate(pb, R0, 0.0, dp, rho, 1e30, R0, 0.0, [1e-5],
                                          rtol=1e-12, atol_r=1e-20, atol_v=1e-12, r_stop=0.01 * R0)
    assert tstop > 0
    assert abs(tstop / t1 - 1.0) < 1e-5


def test_km_linear_oscillator(orc):
    """Small oscillations follow the linearised KM equation (all of mu, sigma, kappa, c enter)."""
    pb = _pb(orc)
    R0 = 10e-6
    rho, p0 = pb.rho0, pb.p0
    c = math.sqrt(pb.gamma * (p0 + pb.pi_inf) / rho)
    pg0 = p0 + 2 * pb.sigma / R0
    K = 3 * pb.kappa * pg0 - 2 * pb.sigma / R0
    m = R0 ** 2 + 4 * pb.mu * R0 / (rho * c)
    b = 4 * pb.mu / rho + R0 * K / (rho * c)
    w0sq = K / rho / m
    beta = b / (2 * m)
    wd = math.sqrt(w0sq - beta ** 2)
    # published-form check of the numbers for this bubble
    assert abs(math.sqrt(w0sq) / 2.17262e6 - 1) < 1e-5
    assert abs(beta / 3.6004e4 - 1) < 1e-4
    assert abs(wd / (2 * math.pi) / 345.74e3 - 1) < 1e-4
    x0 = 1e-6 * R0
    t = np.linspace(0, 4 * 2 * math.pi / wd, 400)
    R, V, _, _ = orc.km_integrate(pb, R0, pg0, p0, rho, c, R0 + x0, 0.0, t, rtol=1e-11, atol_r=1e-22,
                                  atol_v=1e-14)
    lin = x0 * np.exp(-beta * t) * (np.cos(wd * t) + beta / wd * np.sin(wd * t))
    err = np.abs((R - R0) - lin).max() / x0
    assert err < 1e-4, err


# ---------------------------------------------------------------------------
# WENO5 (Sec. 3)
# ---------------------------------------------------------------------------

def _cell_avg(F, xl, h):
    return (F(xl + h) - F(xl)) / h


def test_weno_quadratic_exact(orc):
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b, c = rng.normal(size=3) * [1.0, 10.0, 100.0]
        P = lambda x: a + b * x + c * x * x
        Pint = lambda x: a * x + b * x * x / 2 + c * x ** 3 / 3
        h = 0.1
        xl = np.arange(-2, 3) * h - h / 2
        v = _cell_avg(Pint, xl, h)
        got = orc.weno5(v)
        assert abs(got - P(h / 2)) <= 1e-12 * max(1.0, abs(P(h / 2)))


def test_weno_fifth_order_smooth(orc):
    errs = []
    for h in (0.04, 0.02, 0.01):
        Fint = lambda x: -np.cos(x + 0.3)
        xl = np.arange(-2, 3) * h - h / 2 + 0.5
        v = _cell_avg(Fint, xl, h)
        errs.append(abs(orc.weno5(v) - math.sin(0.5 + h / 2 + 0.3)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 4.5, orders


def test_weno_mirror_and_bounded(orc):
    rng = np.random.default_rng(4)
    for _ in range(20):
        v = rng.normal(size=5)
        # mirrored data -> value at the mirrored face equals the reversed-stencil call
        assert orc.weno5(v[::-1].copy()) == orc.weno5(np.ascontiguousarray(v[::-1]))
    step = np.array([0.0, 0.0, 0.0, 1.0, 1.0])
    val = orc.weno5(step)
    assert -1e-6 <= val <= 1.0 + 1e-6
    step2 = np.array([0.0, 0.0, 1.0, 1.0, 1.0])
    assert abs(orc.weno5(step2) - 1.0) < 1e-6


# ---------------------------------------------------------------------------
# HLLC (Sec. 3)
# ---------------------------------------------------------------------------

def test_hllc_consistency(orc):
    """F(W, W) is the physical flux of the governing equations."""
    rng = np.random.default_rng(5)
    for ndim in (1, 2, 3):
        nb = 3
        pb = _pb(orc, ndim=ndim, n=(8, 8 if ndim > 1 else 1, 8 if ndim > 2 else 1), dx=(1e-4,) * 3, nb=nb)
        for _ in range(10):
            rho = 1000 * (1 + 0.01 * rng.normal())
            u = rng.normal(size=ndim) * 5
            pl = 1e5 * (1 + 0.5 * rng.uniform())
            a = 1e-4 * rng.uniform(0.5, 2)
            n = 1e10 * rng.uniform(0.5, 2)
            B = 1e5 * (1 + 0.1 * rng.normal())
            R = 1e-5 * rng.uniform(0.5, 2, size=nb)
            V = rng.normal(size=nb)
            Wv = np.concatenate([[rho], u, [pl, a, n, B], R, V])
            for d in range(ndim):
                F = orc.hllc(pb, d, Wv, Wv)
                p = (1 - a) * pl + a * B
                E = (1 - a) * (pl + pb.gamma * pb.pi_inf) / (pb.gamma - 1) + 0.5 * rho * (u ** 2).sum()
                exp = np.concatenate([[rho * u[d]], rho * u[d] * u + p * (np.arange(ndim) == d),
                                      [(E + p) * u[d], a * u[d]], n * R * u[d], n * V * u[d]])
                assert np.allclose(F, exp, rtol=1e-13, atol=1e-13 * np.abs(exp).max())


def _run_riemann(orc, N, left, right, gamma, pi_inf, t_end, length=1.0, cfl=0.3):
    liq = dict(gamma=gamma, pi_inf=pi_inf, rho0=1.0, p0=1.0)
    pb = orc.problem(1, (N, 1, 1), (length / N, 1, 1), ((1, 1), (0, 0), (0, 0)), 1, cfl=cfl, liquid=liq)
    x = (np.arange(N) + 0.5) * length / N
    prim = np.zeros((4, N))
    L = x < 0.5 * length
    prim[0] = np.where(L, left[0], right[0])
    prim[1] = np.where(L, left[1], right[1])
    prim[2] = np.where(L, left[2], right[2])
    prim[3] = 0.0
    q = orc.init_state(pb, prim)
    t = 0.0
    while t < t_end * (1 - 1e-14):
        dt = min(orc.cfl_dt(pb, q), t_end - t)
        orc.rk3_step(pb, q, dt)
        t += dt
    rho = q[0]
    u = q[1] / rho
    p = (gamma - 1) * (q[2] - 0.5 * rho * u * u) - gamma * pi_inf
    ex = exact_riemann.sample(left, right, gamma, (x - 0.5 * length) / t_end, pi_inf)
    return x, rho, u, p, ex


def test_exact_riemann_reference_values():
    ps, us = exact_riemann.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    assert abs(ps - 0.30313) < 1e-5 and abs(us - 0.92745) < 1e-5


def test_sod_exact(orc):
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ps, us = exact_riemann.star_state(left, right, 1.4)
    l1 = []
    for N in (100, 200, 400, 800):
        x, rho, u, p, ex = _run_riemann(orc, N, left, right, 1.4, 0.0, 0.2)
        l1.append(np.abs(rho - ex[0]).mean())
        if N == 800:
            plateau = (x > 0.5 + 0.2 * 0.2) & (x < 0.5 + 0.2 * 0.85)   # between the rarefaction tail and the contact
            assert abs(np.median(p[plateau]) / ps - 1) < 5e-3
            assert abs(np.median(u[plateau]) / us - 1) < 5e-3
    assert all(l1[i + 1] < l1[i] for i in range(3)), l1


def test_stiffened_water_shock_tube(orc):
    """Water shock tube through the pressure shift p + pi_inf."""
    g, pinf = 7.1, 3.06e8
    left, right = (1010.0, 0.0, 2e8), (1000.0, 0.0, 1e5)
    ps, us = exact_riemann.star_state(left, right, g, pinf)
    x, rho, u, p, ex = _run_riemann(orc, 800, left, right, g, pinf, 1e-4, length=0.5)
    c = math.sqrt(g * (left[2] + pinf) / left[0])
    xs = 0.25 + us * 1e-4
    plateau = (x > 0.25 - 0.5 * c * 1e-4) & (x < 0.25 + 0.5 * us * 1e-4 + 0.02)
    plateau &= np.abs(x - xs) > 0.02
    assert plateau.sum() > 20
    assert abs(np.median(p[plateau]) / ps - 1) < 5e-3
    assert abs(np.median(u[plateau]) / us - 1) < 5e-3
    assert np.abs(p - ex[2]).mean() < 0.02 * (left[2] - right[2])


# ---------------------------------------------------------------------------
# Primitives and moments (eqs. e:pressure, e:ndf)
# ---------------------------------------------------------------------------

def test_equilibrium_pressure_and_n(orc):
    case = W.random_smooth(2, (12, 10), 1e-4, 5, seed=7, amp_atm=0.0, umax=0.0)
    pb = orc.problem_from_case(case)
    q = orc.init_state(pb, case.prim)
    m = orc.moments(pb, q)
    r0, w = orc.bins(5, 10e-6, 0.3)
    n_exp = case.prim[-1] / (4 * math.pi / 3 * (w * r0 ** 3).sum())
    assert np.allclose(m[0], n_exp, rtol=1e-14)
    assert np.allclose(m[6], pb.p0, rtol=1e-14)    # p_mix = p0 at equilibrium for any alpha
    assert np.allclose(m[7], pb.p0, rtol=1e-12)


# ---------------------------------------------------------------------------
# Discrete invariants of the semi-discrete scheme (Sec. 3)
# ---------------------------------------------------------------------------

def test_free_stream_preservation(orc):
    case = W.uniform(2, (10, 8), 1e-4, 3, u=(3.0, -2.0, 0.0), alpha=2e-4)
    pb = orc.problem_from_case(case)
    q = orc.init_state(pb, case.prim)
    q0 = q.copy()
    for _ in range(5):
        orc.rk3_step(pb, q)
    rel = np.abs(q - q0).max(axis=1) / np.maximum(np.abs(q0).max(axis=1), 1e-300)
    assert rel.max() < 5e-13, rel


def test_contact_at_rest(orc):
    n = 40
    case = W.uniform(1, (n,), 1e-4, 3, alpha=1e-4)
    x = np.arange(n)
    case.prim[3] = np.where((x > 10) & (x < 25), 3e-3, 1e-4)
    pb = orc.problem_from_case(case)
    q = orc.init_state(pb, case.prim)
    for _ in range(100):
        orc.rk3_step(pb, q)
    u = q[1] / q[0]
    assert np.abs(u).max() < 1e-12


def test_periodic_conservation(orc):
    case = W.random_smooth(2, (16, 12), 1e-4, 3, seed=11)
    pb = orc.problem_from_case(case)
    q = orc.init_state(pb, case.prim)
    tot0 = q[:4].sum(axis=1)
    for _ in range(5):
        orc.rk3_step(pb, q)
    tot = q[:4].sum(axis=1)
    scale = np.abs(q[:4]).sum(axis=1)
    assert (np.abs(tot - tot0) / scale).max() < 5e-14 * 5


def test_mirror_symmetry_1d(orc):
    n = 64
    case = W.c1(n=n, length=n * 2.5e-4, nb=3, steps=1)
    case.prim[2] = W.WATER["p0"] + 0.5 * ATM * np.exp(-((np.arange(n) + 0.5 - n / 2) / 6.0) ** 2)
    case.bc = ((0, 0), (0, 0), (0, 0))
    pb = orc.problem_from_case(case)
    q = orc.init_state(pb, case.prim)
    for _ in range(20):
        orc.rk3_step(pb, q)
    m = q[:, ::-1].copy()
    m[1] = -m[1]
    for v in range(q.shape[0]):
        scale = np.abs(q[v]).max()
        if scale == 0:
            continue
        assert np.abs(q[v] - m[v]).max() <= 1e-12 * scale, v


def test_xy_permutation_2d(orc):
    n = 16
    case = W.c3(n=n, nb=3)  # placeholder for constants; build a 2D symmetric field below
    c2 = W.uniform(2, (n, n), 1e-4, 3)
    xs = (np.arange(n) + 0.5 - n / 2)
    r2 = xs[None, :] ** 2 + xs[:, None] ** 2
    c2.prim[3] = (W.WATER["p0"] + 2 * ATM * np.exp(-r2 / 8.0)).reshape(-1)
    c2.bc = ((1, 1), (1, 1), (0, 0))
    pb = orc.problem_from_case(c2)
    q = orc.init_state(pb, c2.prim)
    for _ in range(10):
        orc.rk3_step(pb, q)
    Q = q.reshape(q.shape[0], n, n)
    T = np.swapaxes(Q, 1, 2).copy()
    T[[1, 2]] = T[[2, 1]]
    for v in range(q.shape[0]):
        scale = np.abs(Q[v]).max()
        assert np.abs(Q[v] - T[v]).max() <= 1e-12 * scale, v
    del case


def test_2d_with_uniform_y_equals_1d(orc):
    n = 48
    c1 = W.c1(n=n, length=n * 2.5e-4, nb=3, steps=1)
    c1.bc = ((0, 0), (0, 0), (0, 0))
    pb1 = orc.problem_from_case(c1)
    q1 = orc.init_state(pb1, c1.prim)
    c2 = W.uniform(2, (n, 4), c1.dx[0], 3)
    c2.prim[0] = np.tile(c1.prim[0], 4)
    c2.prim[1] = np.tile(c1.prim[1], 4)
    c2.prim[2] = 0.0
    c2.prim[3] = np.tile(c1.prim[2], 4)
    c2.prim[4] = np.tile(c1.prim[3], 4)
    pb2 = orc.problem_from_case(c2)
    q2 = orc.init_state(pb2, c2.prim)
    for _ in range(10):
        dt = orc.cfl_dt(pb1, q1)
        orc.rk3_step(pb1, q1, dt)
        orc.rk3_step(pb2, q2, dt)
    Q2 = q2.reshape(q2.shape[0], 4, n)
    keep = [0, 1, 3, 4] + list(range(5, q2.shape[0]))
    for k, v in enumerate(keep):
        scale = np.abs(q1[k]).max()
        for j in range(4):
            assert np.abs(Q2[v, j] - q1[k]).max() <= 1e-13 * scale
    assert np.abs(Q2[2]).max() == 0.0


def test_rhs_cells_matches_full(orc):
    case = W.random_smooth(3, (8, 7, 6), 1e-4, 3, seed=13, bc=1)
    pb = orc.problem_from_case(case)
    q = orc.init_state(pb, case.prim)
    q[-3:] += 0.05 * q[4 + 3] * 0  # keep bins at rest
    L = orc.rhs(pb, q)
    rng = np.random.default_rng(0)
    cells = rng.choice(q.shape[1], 25, replace=False)
    Lc = orc.rhs_cells(pb, q, cells)
    assert np.array_equal(Lc, L[:, cells].T)


# ---------------------------------------------------------------------------
# 0D reduction: a uniform periodic state reduces the PDE to the bubble ODEs
# ---------------------------------------------------------------------------

def _uniform_out_of_eq(orc, nb=3, pratio=1.6, split=0):
    case = W.uniform(1, (4,), 1e-4, nb, p=pratio * W.WATER["p0"], alpha=5e-4)
    pb = orc.problem_from_case(case, split=split)
    return pb, orc.init_state(pb, case.prim)


def test_0d_reduction_rk3_order(orc):
    pb, q0 = _uniform_out_of_eq(orc)
    T = 4e-7

    def run(nsteps):
        q = q0.copy()
        for _ in range(nsteps):
            orc.rk3_step(pb, q, T / nsteps)
        return q

    ref = run(640)
    errs = []
    for ns in (20, 40, 80):
        q = run(ns)
        assert np.array_equal(q[:, 0:1].repeat(4, 1), q)     # stays uniform
        errs.append(np.abs(q[5:, 0] - ref[5:, 0]).max() / np.abs(ref[5:, 0]).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 2.8, orders
    # n is invariant of the ODE system: drift is a time-stepping error only
    m0, m1 = orc.moments(pb, q0), orc.moments(pb, run(80))
    assert abs(m1[0, 0] / m0[0, 0] - 1) < 1e-6


def test_0d_reduction_matches_ode_solution(orc):
    """Bins of a uniform state follow KM with p_inf = p_l(alpha): check against scipy."""
    from scipy.integrate import solve_ivp
    pb, q0 = _uniform_out_of_eq(orc, nb=3)
    r0, w = orc.bins(3, 10e-6, 0.3)
    pg0 = pb.p0 + 2 * pb.sigma / r0
    rho, E = q0[0, 0], q0[2, 0]
    n = orc.moments(pb, q0)[0, 0]

    def f(t, y):
        R, V, a = y[:3], y[3:6], y[6]
        pl = (pb.gamma - 1) * E / (1 - a) - pb.gamma * pb.pi_inf
        rhol = rho / (1 - a)
        c = math.sqrt(pb.gamma * (pl + pb.pi_inf) / rhol)
        acc = [orc.km_rddot(pb, R[i], V[i], r0[i], pg0[i], pl, rhol, c) for i in range(3)]
        da = 3 * a * (w * R * R * V).sum() / (w * R ** 3).sum()
        return np.concatenate([V, acc, [da]])

    T = 4e-7
    sol = solve_ivp(f, (0, T), np.concatenate([r0, np.zeros(3), [q0[3, 0]]]), method="DOP853",
                    rtol=1e-12, atol=1e-20)
    q = q0.copy()
    for _ in range(400):
        orc.rk3_step(pb, q, T / 400)
    R = q[4:7, 0] / n
    assert np.abs(R / sol.y[:3, -1] - 1).max() < 1e-7
    assert abs(q[3, 0] / sol.y[6, -1] - 1) < 1e-7


# ---------------------------------------------------------------------------
# Strang-split adaptive bubble sub-steps (Sec. 3)
# ---------------------------------------------------------------------------

def test_split_equilibrium_one_substep(orc):
    case = W.uniform(1, (6,), 1e-4, 5)
    pb = orc.problem_from_case(case, split=1)
    q = orc.init_state(pb, case.prim)
    q0 = q.copy()
    ns = orc.bubble_advance(pb, q, 1e-7)
    assert (ns == 1).all()
    assert np.abs(q - q0).max() <= 1e-12 * np.abs(q0).max()


def test_split_substeps_follow_km(orc):
    pb, q = _uniform_out_of_eq(orc, nb=3, pratio=3.0, split=1)
    r0, w = orc.bins(3, 10e-6, 0.3)
    pg0 = pb.p0 + 2 * pb.sigma / r0
    m = orc.moments(pb, q)
    pl, n = m[7, 0], m[0, 0]
    rhol = q[0, 0] / (1 - q[3, 0])
    c = math.sqrt(pb.gamma * (pl + pb.pi_inf) / rhol)
    tau = 3e-7
    ns = orc.bubble_advance(pb, q, tau)
    assert ns.min() > 1
    for i in range(3):
        R, V, _, _ = orc.km_integrate(pb, r0[i], pg0[i], pl, rhol, c, r0[i], 0.0, [tau], rtol=1e-12,
                                      atol_r=1e-22, atol_v=1e-14)
        assert abs(q[4 + i, 0] / n / R[0] - 1) < 2e-3
    # alpha follows M3 with n frozen
    Rn = q[4:7, 0] / n
    assert abs(q[3, 0] / (5e-4 * (w * Rn ** 3).sum() / (w * r0 ** 3).sum()) - 1) < 1e-13
