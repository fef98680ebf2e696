"""Pins of the oracle's transfer contents (Sec. 2: gas and vapour in the bubble, heat and vapour transfer
at the wall through constant coefficients, eq. massVaporRate and the contents-pressure equation).

The paper gives the model's equations but not its coefficients, so what is pinned is what the equations
fix whatever the coefficients are:

* equilibrium: a bubble at R0 at rest with its contents at the Laplace pressure and the vapour saturated
  has every rate zero, and the full right-hand side of a uniform bubbly liquid vanishes;
* no transfer (beta_T = 0, no vapour) reduces the contents to a polytropic gas with exponent gamma_b:
  the whole EE trajectory follows the polytropic model with kappa = gamma_b, converging at third order
  in the step (the two differ only in integrating p_b instead of evaluating it);
* strong heat transfer drives the contents to the wall temperature: p_b R^3 stays constant;
* the first law of the contents with vapour transfer and no heat transfer, d(p V)/(gamma_b - 1) =
  -p dV + c_p,v T0 dm_v, along a driven nonlinear oscillation;
* the linearised heat-transfer oscillator (derived by hand from the model: small x = R/R0 - 1,
  y = p/p_b0 - 1 and the ideal-gas temperature) against the oracle's small-amplitude run;
* at fixed radius with no heat transfer, vapour uptake keeps p - p_b0 = gamma_b R_v T0 (m - m_v0)/V0 and
  relaxes at the rate the linearised transfer law gives; condensation under compression.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import workloads as W

C = W.AIR_VAPOUR
R0 = 10e-6
P0 = W.WATER["p0"]
SIG = W.AIR["sigma"]
MU = W.AIR["mu"]


def _eq(pv, R=R0, contents=C):
    """Equilibrium contents of a bubble of equilibrium radius R: p_b0, m_v0, gas mass."""
    V0 = 4.0 / 3.0 * math.pi * R ** 3
    pb0 = P0 + 2.0 * SIG / R
    return pb0, pv * V0 / (contents["Rv"] * contents["T0"]), (pb0 - pv) * V0 / (contents["Rg"] * contents["T0"])


def _one_cell(orc, contents, pv, p_l=P0, alpha=1e-8, rtol=1e-10, mu=MU, r0=R0):
    """One periodic cell in split mode: only the bubble half-steps act, with the liquid frozen."""
    gas = dict(W.AIR, pv=pv, mu=mu)
    pb = orc.problem(1, (1, 1, 1), (1e-4, 1e-4, 1e-4), ((0, 0),) * 3, 1, r0_median=r0, sigma_ln=0.3, gas=gas,
                     split=1, sub_rtol=rtol, max_substeps=10 ** 7, contents=contents)
    q = orc.init_state(pb, np.array([[1000.0], [0.0], [p_l], [alpha]]))
    return pb, q


def _bubble(orc, pb, q):
    n = orc.moments(pb, q)[0, 0]
    R, V = q[4, 0] / n, q[5, 0] / n
    if pb.contents:
        return R, V, q[6, 0] / n, q[7, 0] / n
    return R, V


@pytest.mark.parametrize("pv", [0.0, W.PV_WATER_20C])
def test_equilibrium_rates_vanish(orc, pv):
    gas = dict(W.AIR, pv=pv)
    pb = orc.problem(1, (8, 1, 1), (1e-4,) * 3, ((0, 0),) * 3, 3, gas=gas, contents=C)
    r0, _ = orc.bins(3, 10e-6, 0.3)
    for R in r0:
        pb0, mv0, mg = _eq(pv, R)
        pdot, mdot = orc.contents_rates(pb, R, 0.0, pb0, mv0, mg)
        assert abs(pdot) <= 1e-12 * pb0 * 1e6 and abs(mdot) <= 1e-12 * (mv0 + mg) * 1e6
        assert abs(orc.km_rddot_pb(pb, R, 0.0, pb0, pdot, P0, 1000.0, 1500.0)) < 1e-6
    prim = np.zeros((4, 8))
    prim[0], prim[2], prim[3] = 1000.0, P0, 1e-3
    q = orc.init_state(pb, prim)
    L = orc.rhs(pb, q)
    assert np.all(L[:7] == 0.0)                        # mixture fluxes cancel; n Rdot = 0 at rest
    n = orc.moments(pb, q)[0].max()
    # what is left is rounding in R = nR/n and the mean temperature: against the rates of a 1 us motion
    assert np.abs(L[7:10]).max() <= 1e-12 * n * P0 / (1000.0 * R0) * 1e0
    assert np.abs(L[10:13]).max() <= 1e-12 * n * P0 * 1e6
    assert np.abs(L[13:16]).max() <= 1e-12 * np.abs(q[13:16]).max() * 1e6 + 1e-12 * n * _eq(pv)[2] * 1e6


def test_no_transfer_is_the_polytropic_model(orc):
    """beta_T = beta_c = 0 and no vapour: p_b R^(3 gamma_b) is conserved by the contents equation, so the
    trajectory is the polytropic one with kappa = gamma_b; the gap closes at third order in dt.  A uniform
    bubbly liquid at 2 atm (every cell the same, so only the bubble dynamics and their coupling to the
    mixture act: advection would mix the cells' p_b and R, whose relation is nonlinear, at the scheme's
    spatial error)."""
    case = W.uniform(1, (8,), 1e-4, 3, p=2 * P0, alpha=1e-3)
    adiabatic = dict(C, beta_T=0.0, beta_c=0.0)
    gaps = []
    for k in (1, 2):
        pt = orc.problem_from_case(case, contents=adiabatic)
        pp = orc.problem_from_case(case)                  # air: kappa = 1.4 = gamma_b
        qt, qp = orc.init_state(pt, case.prim), orc.init_state(pp, case.prim)
        dt = 2e-9 / k
        for _ in range(200 * k):
            orc.rk3_step(pt, qt, dt)
            orc.rk3_step(pp, qp, dt)
        nv = qp.shape[0]
        gap = np.abs(qt[:nv] - qp).max(axis=1) / np.maximum(np.abs(qp).max(axis=1), 1e-300)
        gaps.append(gap.max())
        # p_b R^(3 gamma) at every cell and bin of the transfer run equals p_b0 R0^(3 gamma)
        n = orc.moments(pt, qt)[0]
        r0, _ = orc.bins(3, case.r0_median, case.sigma_ln)
        for i in range(3):
            R, p = qt[4 + i] / n, qt[4 + 6 + i] / n
            inv = p * R ** (3 * C["gam_b"]) / ((P0 + 2 * SIG / r0[i]) * r0[i] ** (3 * C["gam_b"]))
            assert np.abs(inv - 1).max() < 1e-7 / k ** 3
    print("no-transfer gap to the polytropic model:", gaps)
    assert gaps[0] < 1e-6 and gaps[0] / gaps[1] > 6.0


def test_strong_heat_transfer_is_isothermal(orc):
    """beta_T large: the contents stay at T0, so p_b R^3 stays at its equilibrium value as the bubble is
    driven by a 3 atm liquid."""
    hot = dict(C, beta_T=2e4, beta_c=0.0)
    pb, q = _one_cell(orc, hot, 0.0, p_l=3 * P0, rtol=1e-8)
    pb0, _, _ = _eq(0.0)
    worst = 0.0
    for _ in range(40):
        orc.bubble_advance(pb, q, 5e-8)
        R, V, p, m = _bubble(orc, pb, q)
        worst = max(worst, abs(p * R ** 3 / (pb0 * R0 ** 3) - 1))
    assert R < 0.9 * R0             # it was compressed
    print("isothermal limit: max |p R^3 / (p0 R0^3) - 1| =", worst)
    assert worst < 2e-3


def test_first_law_with_vapour_transfer(orc):
    """No heat transfer, vapour transfer on: d(p V)/(gamma - 1) = -p dV + gamma/(gamma - 1) R_v T0 dm along
    a driven oscillation (the vapour enters and leaves at the wall temperature).  The work integral is
    taken by the trapezoid rule over 1 ns samples."""
    vap = dict(C, beta_T=0.0, beta_c=5.0, D_v=2.42e-5)
    pb, q = _one_cell(orc, vap, W.PV_WATER_20C, p_l=0.5 * P0)
    g = C["gam_b"]
    samples = [_bubble(orc, pb, q)]
    for _ in range(3000):
        orc.bubble_advance(pb, q, 1e-9)
        samples.append(_bubble(orc, pb, q))
    s = np.array(samples)
    R, p, m = s[:, 0], s[:, 2], s[:, 3]
    V = 4.0 / 3.0 * math.pi * R ** 3
    U = p * V / (g - 1)
    work = np.concatenate([[0.0], np.cumsum(0.5 * (p[1:] + p[:-1]) * np.diff(V))])
    hv = g / (g - 1) * C["Rv"] * C["T0"]
    resid = U - U[0] + work - hv * (m - m[0])
    scale = np.abs(work).max()
    assert abs(m[-1] - m[0]) > 1e-3 * m[0]       # vapour moved
    assert R.max() > 1.2 * R0                     # the bubble grew in the low-pressure liquid
    print("first law: max residual / max work", np.abs(resid).max() / scale)
    assert np.abs(resid).max() < 1e-4 * scale


@pytest.mark.parametrize("r0", [10e-6, 4e-6])
def test_linear_thermal_oscillator(orc, r0):
    """Small free oscillation with heat transfer and no vapour against the linearised model:
       x' = v,
       y' = -3 gamma v - lam (y + 3x),             lam = 3 (gamma - 1) k beta_T T0 / (p_b0 R0^2),
       (R0^2 + 4 mu R0/(rho c)) v' = (p_b0 y + 2 sigma/R0 x - 4 mu v)/rho + R0 (p_b0 y' + 2 sigma/R0 v)/(rho c),
    from Keller--Miksis with p_bw = p_b - 2 sigma/R - 4 mu Rdot/R and the ideal-gas temperature
    T/T0 - 1 = y + 3x at fixed gas mass."""
    eps = 1e-5
    R0 = r0
    pb, q = _one_cell(orc, dict(C, beta_c=0.0), 0.0, r0=r0)
    n = orc.moments(pb, q)[0, 0]
    q[4, 0] *= 1 + eps                               # R = R0 (1 + eps), contents unchanged,
    q[3, 0] *= (1 + eps) ** 3                        # and alpha with it, so that n stays
    g, k, bt, T0 = C["gam_b"], C["k_b"], C["beta_T"], C["T0"]
    pb0 = P0 + 2 * SIG / R0
    rho = 1000.0
    c = math.sqrt(W.WATER["gamma"] * (P0 + W.WATER["pi_inf"]) / rho)
    lam = 3 * (g - 1) * k * bt * T0 / (pb0 * R0 ** 2)
    # v' = a1 x + a2 v + a3 y + a4 y'  with y' = -3 g v - lam y - 3 lam x
    den = R0 ** 2 + 4 * MU * R0 / (rho * c)
    a1, a2, a3 = 2 * SIG / R0 / rho, -4 * MU / rho + R0 * 2 * SIG / R0 / (rho * c), pb0 / rho
    a4 = R0 * pb0 / (rho * c)
    A = np.array([[0.0, 1.0, 0.0],
                  [(a1 - 3 * lam * a4) / den, (a2 - 3 * g * a4) / den, (a3 - lam * a4) / den],
                  [-3 * lam, -3 * g, -lam]])
    x0 = np.array([eps, 0.0, 0.0])
    ev = np.linalg.eigvals(A)
    period = 2 * math.pi / np.abs(ev.imag).max()
    dt = period / 50
    worst = 0.0
    for j in range(1, 151):
        orc.bubble_advance(pb, q, dt)
        R = q[4, 0] / n
        x_lin = (expm(A * j * dt) @ x0)[0]
        worst = max(worst, abs((R / R0 - 1) - x_lin))
    decay = -ev[np.abs(ev.imag).argmax()].real * period
    print(f"linear thermal oscillator: period {period:.3e} s, decay per period {decay:.3f}, max |x - x_lin|/eps "
          f"{worst / eps:.2e}")
    assert decay > 0.05                    # heat transfer damps the oscillation visibly over 3 periods
    assert worst < 2e-3 * eps


def test_vapour_relaxation_at_fixed_radius(orc):
    """R fixed, no heat transfer: the contents equation gives dp = gamma R_v T0 dm / V0 exactly, and the
    vapour relaxes to saturation at the rate of the linearised law
       dm/dt = 4 pi R0 D beta_c rho_w/(1 - chi_w) (dchi_w/dp gamma R_v T0 / V0 - dchibar/dm) (m - m_eq);
    a compressed bubble (p_b above p_b0, same vapour mass) condenses."""
    pb = orc.problem(1, (1, 1, 1), (1e-4,) * 3, ((0, 0),) * 3, 1, r0_median=R0, sigma_ln=0.3,
                     gas=dict(W.AIR, pv=W.PV_WATER_20C), contents=dict(C, beta_T=0.0))
    pv = W.PV_WATER_20C
    pb0, mv0, mg = _eq(pv)
    V0 = 4.0 / 3.0 * math.pi * R0 ** 3
    g, Rg, Rv, T0 = C["gam_b"], C["Rg"], C["Rv"], C["T0"]
    # condensation under compression
    assert orc.contents_rates(pb, R0, 0.0, 1.5 * pb0, mv0, mg)[1] < 0
    assert orc.contents_rates(pb, R0, 0.0, 0.8 * pb0, mv0, mg)[1] > 0

    def f(t, y):
        return orc.contents_rates(pb, R0, 0.0, y[0], y[1], mg)

    m1 = 1.05 * mv0
    p1 = pb0 + g * Rv * T0 * (m1 - mv0) / V0
    sol = solve_ivp(f, (0, 2e-6), [p1, m1], method="LSODA", rtol=1e-11, atol=[1e-9, 1e-30], dense_output=True)
    ts = np.linspace(0, 2e-6, 41)
    p, m = sol.sol(ts)
    inv = p - g * Rv * T0 * m / V0
    assert np.abs(inv - inv[0]).max() < 1e-7 * pb0
    # the linearised rate
    Sw = pv * Rg + (pb0 - pv) * Rv
    chiw = pv * Rg / Sw
    rhow = pb0 / ((chiw * Rv + (1 - chiw) * Rg) * T0)
    dchiw_dp = -pv * Rg * Rv / Sw ** 2
    dchib_dm = mg / (mv0 + mg) ** 2
    rate = 4 * math.pi * R0 * C["D_v"] * C["beta_c"] * rhow / (1 - chiw) * (dchiw_dp * g * Rv * T0 / V0 - dchib_dm)
    # the equilibrium of this closed system is (pb0, mv0); deviations decay as exp(rate t)
    dev = m - mv0
    k = slice(5, 30)
    fit = np.polyfit(ts[k], np.log(np.abs(dev[k])), 1)[0]
    print(f"vapour relaxation: rate {fit:.4e} 1/s, linearised {rate:.4e} 1/s")
    assert rate < 0 and abs(fit / rate - 1) < 2e-3
