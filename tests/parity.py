"""Helpers shared by the GPU parity tests (comparison norms, seeded state perturbation)."""
from __future__ import annotations

import numpy as np


def rel_err(got, ref, floor=1e-300):
    """Per-row max-norm relative error max|got - ref| / max|ref| (rows = fields)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref).max(axis=-1), floor)
    return np.abs(got - ref).max(axis=-1) / scale


def perturb_bins(q, ndim, nb, seed, amp_r=0.05, vel=0.5):
    """Seeded out-of-equilibrium bins: nR_i scaled by (1 + amp_r * noise), nRdot_i = nR_i * vel * noise / R0-scale.

    Acts only on the bin slots of a conserved state and uses plain multiplications,
    so it is an input recipe, not part of the method.
    """
    rng = np.random.default_rng(seed)
    q = q.copy()
    N = q.shape[1]
    i0 = ndim + 3
    for i in range(nb):
        s = 1.0 + amp_r * np.sin(rng.uniform(0, 6.3) + np.linspace(0, rng.uniform(2, 9), N))
        q[i0 + i] *= s
        q[i0 + nb + i] = q[i0 + i] * vel * np.cos(rng.uniform(0, 6.3) + np.linspace(0, rng.uniform(2, 9), N)) / 1e-5
    return q


def flux_scale(orc, pb, q):
    """Per-field size of the face fluxes divided by the spacing.

    Conserved field v has flux ~ (max wave speed) * |q_v|; momentum also carries
    the pressure, so its rows get max|p| / dx as well.
    """
    q = np.asarray(q)
    lam_dx = pb.cfl / orc.cfl_dt(pb, q)
    s = lam_dx * np.abs(q).max(axis=-1)
    dxmin = min(pb.dx[d] for d in range(pb.ndim))
    pmax = np.abs(orc.moments(pb, q)[6]).max()
    mom = slice(1, 1 + pb.ndim)
    s[mom] = lam_dx * np.abs(q[mom]).max() + pmax / dxmin
    return s


def rhs_err(got, ref, scale):
    """RHS error per field relative to max|L| + the flux-divergence scale of that field.

    A rate that is a small difference of large face fluxes carries rounding of the
    size of the fluxes, so its error is measured against that scale.
    """
    got = np.asarray(got)
    ref = np.asarray(ref)
    s = np.abs(ref).max(axis=-1) + scale
    return np.abs(got - ref).max(axis=-1) / np.maximum(s, 1e-300)


def oracle_split_step(orc, pb, q, dt):
    """One split-mode step of the oracle in its three parts, S_b(dt/2) S_f(dt) S_b(dt/2), in place on q.

    Returns the accepted sub-step counts of both bubble half-steps, int32 [2][nb][N].  The flux part is
    the oracle's SSP-RK3 on its flux-only right-hand side with the same operations in the same order as
    the oracle's own step, so the result is bitwise that of orc.rk3_step (a CPU test checks this).
    """
    ns1 = orc.bubble_advance(pb, q, 0.5 * dt)
    L = orc.rhs(pb, q, sources=False)
    u1 = q + dt * L
    L = orc.rhs(pb, u1, sources=False)
    u2 = 0.75 * q + 0.25 * (u1 + dt * L)
    L = orc.rhs(pb, u2, sources=False)
    q[:] = q / 3.0 + 2.0 / 3.0 * (u2 + dt * L)
    ns2 = orc.bubble_advance(pb, q, 0.5 * dt)
    return np.stack([ns1, ns2])

