"""Pins of the oracle's volume-averaged (Euler--Lagrange) variant, Sec. 2.1."""
import math

import numpy as np

import workloads as W


def _pb(orc, n=16, dx=1e-4, bc=0):
    return orc.problem(3, (n, n, n), (dx, dx, dx), ((bc, bc),) * 3, 1)


def test_kernel_shape(orc):
    h = 1e-4
    peak = 1.0 / (h ** 3 * (2 * math.pi) ** 1.5)
    assert abs(orc.el_kernel(0.0, h) / peak - 1) < 1e-15
    assert abs(orc.el_kernel(h, h) / (peak * math.exp(-0.5)) - 1) < 1e-15
    assert orc.el_kernel(3 * h, h) == 0.0
    assert orc.el_kernel(2.999999 * h, h) > 0.0


def _lattice_mass(x, h, dx, m=6):
    """Brute-force sum of delta * dV over a large lattice (eq. kernel3D written out)."""
    host = np.floor(x / dx).astype(int)
    off = np.arange(-m, m + 1)
    g = [(host[d] + off + 0.5) * dx - x[d] for d in range(3)]
    d2 = g[0][None, None, :] ** 2 + g[1][None, :, None] ** 2 + g[2][:, None, None] ** 2
    d = np.sqrt(d2)
    k = np.where(d < 3 * h, np.exp(-d2 / (2 * h * h)) / (h ** 3 * (2 * math.pi) ** 1.5), 0.0)
    return k.sum() * dx ** 3


def test_smear_total_volume_matches_lattice_sum(orc):
    n, dx = 16, 1e-4
    pb = _pb(orc, n, dx)
    rng = np.random.default_rng(2)
    nb = 20
    pos = rng.uniform(0, n * dx, size=(3, nb))
    r0 = 10e-6 * np.exp(0.3 * rng.standard_normal(nb))
    bub = orc.el_bubbles(pb, pos, r0)
    bub[4] *= rng.uniform(0.8, 1.2, nb)      # non-equilibrium radii
    bub[5] = rng.normal(size=nb)             # and wall velocities
    alpha, dalpha = orc.el_smear(pb, bub)
    vol = 4 / 3 * math.pi * bub[4] ** 3
    rate = 4 * math.pi * bub[4] ** 2 * bub[5]
    K = np.array([_lattice_mass(pos[:, b], dx, dx) for b in range(nb)])
    assert abs(alpha.sum() * dx ** 3 / (vol * K).sum() - 1) < 1e-13
    assert abs(dalpha.sum() * dx ** 3 - (rate * K).sum()) < 1e-13 * np.abs(rate * K).sum()
    # the discrete kernel mass is close to the continuous mass inside 3h (0.9707...)
    cont = math.erf(3 / math.sqrt(2)) - math.sqrt(2 / math.pi) * 3 * math.exp(-4.5)
    assert np.all(np.abs(K / cont - 1) < 0.05)


def test_gather_uniform_field_exact(orc):
    pb = _pb(orc)
    n = 16
    N = n ** 3
    prim = np.zeros((5, N))
    prim[0] = 998.0
    prim[4] = 2.5e5
    ql = orc.el_liquid_state(pb, prim)
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, n * 1e-4, size=(3, 10))
    bub = orc.el_bubbles(pb, pos, np.full(10, 10e-6))
    p, r, c = orc.el_gather(pb, ql, bub)
    assert np.allclose(p, 2.5e5, rtol=1e-14)
    assert np.allclose(r, 998.0, rtol=0)


def test_bubble_at_rest_stays(orc):
    pb = _pb(orc, n=12)
    n = 12
    N = n ** 3
    prim = np.zeros((5, N))
    prim[0] = pb.rho0
    prim[4] = pb.p0
    ql = orc.el_liquid_state(pb, prim)
    bub = orc.el_bubbles(pb, np.full((3, 1), 6e-4 + 1.3e-5), np.array([10e-6]))
    alpha, dalpha = orc.el_smear(pb, bub)
    for _ in range(5):
        orc.el_step(pb, ql, bub, alpha, dalpha)
    assert abs(bub[4, 0] / 10e-6 - 1) < 1e-12
    assert abs(bub[5, 0]) < 1e-9


def test_driven_bubble_follows_km(orc):
    """Uniform overpressure: the gathered forcing is uniform, so each bubble follows KM."""
    pb = _pb(orc, n=12)
    n = 12
    N = n ** 3
    prim = np.zeros((5, N))
    prim[0] = pb.rho0
    prim[4] = 2 * pb.p0
    ql = orc.el_liquid_state(pb, prim)
    R0 = 10e-6
    bub = orc.el_bubbles(pb, np.full((3, 1), 6e-4 + 2e-5), np.array([R0]))
    alpha, dalpha = orc.el_smear(pb, bub)
    dt = 2e-8
    for _ in range(5):
        orc.el_step(pb, ql, bub, alpha, dalpha, dt)
    c = math.sqrt(pb.gamma * (2 * pb.p0 + pb.pi_inf) / pb.rho0)
    R, V, _, _ = orc.km_integrate(pb, R0, bub[6, 0], 2 * pb.p0, pb.rho0, c, R0, 0.0, [5 * dt], rtol=1e-12,
                                  atol_r=1e-22, atol_v=1e-14)
    # a single dilute bubble barely perturbs the liquid: KM with the undisturbed forcing
    assert abs(bub[4, 0] / R[0] - 1) < 1e-4
