"""Pins of the oracle's viscous stress (eq. stressTensor in the fluxes of eq. euler_transport).

The stress T = mu (grad u + grad u^T - 2/3 div(u) I) enters the momentum flux as -T and the energy flux as
-T.u.  Its discretisation is not given by the paper; whatever it is, the viscous part of the right-hand side
must tend to the analytic divergences of T and T.u, and a shear wave must decay as exp(-nu k^2 t).
"""
import math

import numpy as np

import workloads as W

MU = 1.0


def _field(n, U=1.0, V=0.5, L=1e-3):
    """2D periodic, u = U sin(kx) cos(ky), v = V cos(kx) sin(ky), uniform rho_l, p_l and alpha."""
    dx = L / n
    case = W.uniform(2, (n, n), dx, 1)
    x = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x)                       # [y][x]
    k = 2 * math.pi / L
    case.prim[1] = (U * np.sin(k * X) * np.cos(k * Y)).reshape(-1)
    case.prim[2] = (V * np.cos(k * X) * np.sin(k * Y)).reshape(-1)
    return case, X.reshape(-1), Y.reshape(-1), k, U, V


def _analytic(X, Y, k, U, V, mu):
    """div T (x, y components) and div(T.u) of the field of _field, worked out by hand."""
    c1, s1, c2, s2 = np.cos(k * X), np.sin(k * X), np.cos(k * Y), np.sin(k * Y)
    A, B, C = 4 * U / 3 - 2 * V / 3, 4 * V / 3 - 2 * U / 3, U + V
    fx = -mu * k * k * s1 * c2 * (7 * U / 3 + V / 3)
    fy = -mu * k * k * c1 * s2 * (U / 3 + 7 * V / 3)
    fe = mu * k * k * (np.cos(2 * k * X) * (A * U * c2 ** 2 - C * V * s2 ** 2)
                       + np.cos(2 * k * Y) * (-C * U * s1 ** 2 + B * V * c1 ** 2))
    return fx, fy, fe


def test_viscous_rhs_tends_to_the_analytic_stress_divergence(orc):
    errs = []
    for n in (16, 32, 64):
        case, X, Y, k, U, V = _field(n)
        gas = dict(case.gas, mu=MU)
        pb0 = orc.problem_from_case(case)
        pb0.mu = MU
        pb1 = orc.problem_from_case(case, viscous=1)
        pb1.mu = MU
        q = orc.init_state(pb1, case.prim)
        Lv = orc.rhs(pb1, q) - orc.rhs(pb0, q)
        fx, fy, fe = _analytic(X, Y, k, U, V, MU)
        # rows: rho, rho u, rho v, E, alpha, nR, nRdot; the stress touches momentum and energy only
        assert np.abs(Lv[[0, 4, 5, 6]]).max() == 0.0
        e = [np.abs(Lv[1] - fx).max() / np.abs(fx).max(), np.abs(Lv[2] - fy).max() / np.abs(fy).max(),
             np.abs(Lv[3] - fe).max() / np.abs(fe).max()]
        errs.append(e)
        del gas
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    assert orders.min() > 1.8, (errs, orders)
    assert errs[-1].max() < 5e-3, errs


def test_shear_wave_decays_at_the_viscous_rate(orc):
    """v = V sin(kx) in a periodic box (no pressure or density change at first order in V): its amplitude
    decays as exp(-nu k^2 t), nu = mu/rho, and the grid error falls at second order."""
    mu, L, Vamp = 10.0, 1e-3, 1e-2
    k = 2 * math.pi / L
    out = []
    for n in (32, 64):
        dx = L / n
        case = W.uniform(2, (n, 4), dx, 1)
        x = ((np.arange(n * 4) % n) + 0.5) * dx
        case.prim[2] = Vamp * np.sin(k * x)
        pb = orc.problem_from_case(case, viscous=1)
        pb.mu = mu
        q = orc.init_state(pb, case.prim)
        rho = q[0].mean()
        nu = mu / rho
        T = 1.0 / (nu * k * k)
        ns = int(math.ceil(T / orc.cfl_dt(pb, q)))
        for _ in range(ns):
            orc.rk3_step(pb, q, T / ns)
        v = q[2] / q[0]
        amp = 2.0 / v.size * (v * np.sin(k * x)).sum()
        out.append(abs(amp / (Vamp * math.exp(-1.0)) - 1))
    assert out[1] < 1e-3 and out[0] / out[1] > 3.5, out
