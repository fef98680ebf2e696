"""Pins of the oracle's one-way acoustic source and non-reflective boundaries.

The paper drives its validation cases with a source-term forcing of the mass, momentum and energy
equations that emits a one-way planar wave (Sec. 2, last paragraph), and bounds them with non-reflective
boundaries after Thompson (Sec. 5.1).  What linear acoustics fixes, independent of the discretisation:

* a right-running pulse leaves through a non-reflective end and leaves the domain quiet (a wall or a
  periodic end sends it back at full amplitude);
* the source emits p'(x, t) = int A(t - (x - x')/c0) g(x' - x_s) dx' on its downstream side, with the
  prescribed amplitude, and nothing upstream;
* in a periodic domain the fluxes cancel in the totals, so the total mass and momentum grow by exactly
  (integral of g) * (SSP-RK3 quadrature of A / c0 and of A), the quadrature being Simpson's rule on
  each step when the stages see the source at t, t + dt and t + dt/2;
* a plane source along y in 2D gives every column the 1D solution;
* Sec. 5.1's isolated bubble (one bin at a trace void fraction) follows Keller-Miksis driven by the
  emitted wave.
"""
import math

import numpy as np

import workloads as W

C0 = W.c0_water()
P0 = W.WATER["p0"]


def _pressure(orc, pb, q):
    return orc.moments(pb, q)[7] - P0


def _run_to(orc, pb, q, T):
    while pb.t < T:
        orc.rk3_step(pb, q)


def test_nonreflective_end_lets_a_pulse_leave(orc):
    res = {}
    for bc in (W.BC_NONREFLECTIVE, W.BC_REFLECTIVE, W.BC_PERIODIC):
        case = W.pulse_tube(bc=bc)
        pb = orc.problem_from_case(case)
        q = orc.init_state(pb, case.prim)
        width = 12 * case.dx[0]
        _run_to(orc, pb, q, (0.4 * 0.1 + 6 * width) / C0)     # the pulse's tail is past the right end
        res[bc] = np.abs(_pressure(orc, pb, q)).max() / 1e3
    assert res[W.BC_NONREFLECTIVE] < 1e-4, res                # measured 9e-6
    assert res[W.BC_REFLECTIVE] > 0.9 and res[W.BC_PERIODIC] > 0.9, res


def _smoothed(A, xs, t, x_s, sig):
    """Exact linear emission: the burst A delayed by the travel time, convolved with the Gaussian g."""
    xp = np.linspace(x_s - 6 * sig, x_s + 6 * sig, 4001)
    g = np.exp(-0.5 * ((xp - x_s) / sig) ** 2) / (math.sqrt(2 * math.pi) * sig)
    return np.array([np.trapezoid(A(t - (x - xp) / C0) * g, xp) for x in xs])


def _burst(src):
    k = 2 * math.pi * src["freq"] / C0
    amp = src["amp"] * math.exp(0.5 * (k * src["width"]) ** 2)
    f, dur = src["freq"], src["ncyc"] / src["freq"]
    return lambda t: np.where((t >= 0) & (t <= dur), amp * np.sin(2 * math.pi * f * t), 0.0)


def _emit(orc, sign):
    case = W.acoustic_tube(1)
    dx = case.dx[0]
    L = case.n[0] * dx
    src = W.source_burst(0, sign, L / 2, dx)
    pb = orc.problem_from_case(case, source=src)
    q = orc.init_state(pb, case.prim)
    _run_to(orc, pb, q, 3 / src["freq"] + 0.3 * L / C0)
    x = (np.arange(case.n[0]) + 0.5) * dx
    return pb, src, x, _pressure(orc, pb, q)


def test_source_emits_the_prescribed_one_way_burst(orc):
    for sign in (1, -1):
        pb, src, x, p = _emit(orc, sign)
        sig, x_s, f = src["width"], src["x"], src["freq"]
        down = (x - x_s) * sign > 6 * sig
        up = (x - x_s) * sign < -6 * sig
        # amplitude: the Gaussian's smoothing takes 7 % off a sinusoid at 3 cells of width; the source
        # restores it
        assert abs(np.abs(p[down]).max() / src["amp"] - 1.0) < 0.01, sign
        # nothing travels upstream
        assert np.abs(p[up]).max() < 1e-3 * src["amp"], sign
        # waveform of the middle cycle against the exact emission (the burst's ends carry the kinks of a
        # switched sine, which the scheme smooths)
        xd = x[down]
        tr = pb.t - sign * (xd - x_s) / C0                     # emission time of each point
        mid = (tr > 1.0 / f) & (tr < 2.0 / f)
        exact = _smoothed(_burst(src), sign * (xd[mid] - x_s) + x_s, pb.t, x_s, sig)
        assert np.abs(p[down][mid] - exact).max() < 0.01 * src["amp"], sign


def test_source_totals_follow_simpson_quadrature(orc):
    """Periodic tube: every flux cancels in the totals, so sum(rho) dx and sum(m) dx grow by exactly the
    integral of g times the step-by-step Simpson quadrature of A/c0 and of sign*A."""
    case = W.acoustic_tube(1, n=200, length=0.05, bc=W.BC_PERIODIC)
    dx = case.dx[0]
    src = W.source_burst(0, -1, 0.02, dx, cycles=0.0)        # continuous, toward -x
    pb = orc.problem_from_case(case, source=src)
    q = orc.init_state(pb, case.prim)
    q0 = q.copy()
    quad = 0.0
    for _ in range(60):
        t = pb.t
        dt = orc.rk3_step(pb, q)
        A = [orc.source_amplitude(pb, t + c * dt) for c in (0.0, 0.5, 1.0)]
        quad += dt * (A[0] + 4 * A[1] + A[2]) / 6
    x = (np.arange(case.n[0]) + 0.5) * dx
    s = x - src["x"]
    g = np.where(np.abs(s) <= 6 * src["width"],
                 np.exp(-0.5 * (s / src["width"]) ** 2) / (math.sqrt(2 * math.pi) * src["width"]), 0.0)
    G = g.sum() * dx
    dmass = (q[0] - q0[0]).sum() * dx
    dmom = (q[1] - q0[1]).sum() * dx
    # rho ~ 1e3 takes increments of ~1e-5 per step, so its totals carry ~1e-8 of rounding; m starts at 0
    assert abs(dmass / (G * quad / C0) - 1) < 2e-7
    assert abs(dmom / (-G * quad) - 1) < 1e-9


def test_plane_source_along_y_gives_every_column_the_1d_solution(orc):
    one = W.acoustic_tube(1, n=240, length=0.06)
    two = W.acoustic_tube(2, n=240, length=0.06, axis=1, ncross=3)
    dx = one.dx[0]
    src1 = W.source_burst(0, 1, 0.03, dx, cycles=1.0)
    src2 = dict(src1, dir=1)
    p1 = orc.problem_from_case(one, source=src1)
    p2 = orc.problem_from_case(two, source=src2)
    q1 = orc.init_state(p1, one.prim)
    q2 = orc.init_state(p2, two.prim)
    for _ in range(80):
        dt = orc.rk3_step(p1, q1)
        orc.rk3_step(p2, q2, dt)
    # 2D slots: rho, mu, mv, E, alpha, ...; column j of the 2D grid holds cells j, j + 3, ...
    for j in range(3):
        np.testing.assert_allclose(q2[0, j::3], q1[0], rtol=1e-13, atol=0)
        np.testing.assert_allclose(q2[2, j::3], q1[1], rtol=1e-10, atol=1e-12 * np.abs(q1[1]).max())
        np.testing.assert_allclose(q2[3, j::3], q1[2], rtol=1e-13, atol=0)
        assert np.abs(q2[1, j::3]).max() == 0.0


def km_driven_by_emission(orc, pb, case, src, probe, ts, plain=False):
    """Keller-Miksis radius of one bubble of the case's radius at the probe cell, at rest at t = 0 and
    driven by the pressure the source emits there in linear acoustics (the burst delayed by the travel
    time and convolved with g; plain: the bare sine burst, delayed); scipy's DOP853 on the oracle's
    Keller-Miksis acceleration."""
    from scipy.integrate import solve_ivp
    R0 = case.r0_median
    pg0 = P0 + 2 * case.gas["sigma"] / R0 - case.gas["pv"]
    xp = (probe + 0.5) * case.dx[0]
    sig = src["width"]
    xg = np.linspace(-6 * sig, 6 * sig, 801)
    g = np.exp(-0.5 * (xg / sig) ** 2) / (math.sqrt(2 * math.pi) * sig)
    A = _burst(src)
    f, dur, delay = src["freq"], src["ncyc"] / src["freq"], (xp - src["x"]) / C0

    def pinf(t):
        if plain:
            tau = t - delay
            return P0 + (src["amp"] * math.sin(2 * math.pi * f * tau) if 0.0 <= tau <= dur else 0.0)
        return P0 + np.trapezoid(A(t - (xp - src["x"] - xg) / C0) * g, xg)

    rho = W.WATER["rho0"]
    sol = solve_ivp(lambda t, y: [y[1], orc.km_rddot(pb, y[0], y[1], R0, pg0, pinf(t), rho, C0)],
                    (0.0, ts[-1]), [R0, 0.0], method="DOP853", rtol=1e-10, atol=[1e-16, 1e-10], t_eval=ts,
                    max_step=0.01 / src["freq"])
    return sol.y[0]


def run_isolated_bubble(orc, case, src, probe):
    """Oracle run of the isolated-bubble set-up in split mode: times, the probe cell's bubble radius and
    the steps taken."""
    pb = orc.problem_from_case(case, source=src, split=1)
    q = orc.init_state(pb, case.prim)
    T = (probe + 0.5 - 0.25 * case.n[0]) * case.dx[0] / C0 + 4.0 / src["freq"]
    ts, Rs, dts = [0.0], [case.r0_median], []
    while pb.t < T:
        dts.append(orc.rk3_step(pb, q))
        ts.append(pb.t)
        Rs.append(q[4, probe] / orc.moments(pb, q)[0][probe])   # 1D slots: rho, m, E, alpha, nR, nRdot
    return pb, np.array(ts), np.array(Rs), dts


def test_isolated_bubble_follows_keller_miksis(orc):
    """Sec. 5.1's first validation set-up (a 50 um bubble, one cycle of 0.2 MPa at 150 kHz, non-reflective
    ends), with the bubble as one bin at a trace void fraction: its radius must follow Keller-Miksis driven
    by the wave the source emits, at 35 and 100 cells per wavelength and CFL 0.2 and 0.6."""
    res = {}
    for ppw, cfl in ((35, 0.2), (100, 0.2), (50, 0.6)):
        case, src, probe = W.isolated_bubble(ppw, cfl)
        pb, ts, Rs, _ = run_isolated_bubble(orc, case, src, probe)
        Rk = km_driven_by_emission(orc, pb, case, src, probe, ts)
        res[(ppw, cfl)] = math.sqrt(np.mean((Rs - Rk) ** 2)) / case.r0_median
        assert Rk.max() > 1.6 * case.r0_median                     # the bubble does respond strongly
        if ppw == 100:
            # against the bare sine of the paper's comparison: the source's support smooths a one-cycle
            # burst's kinks, which costs less the finer the grid; the paper reports at most 2.76 %
            Rp = km_driven_by_emission(orc, pb, case, src, probe, ts, plain=True)
            plain = math.sqrt(np.mean((Rs - Rp) ** 2)) / case.r0_median
            print(f"RMSE / R0 against the bare sine at {ppw} cells per wavelength: {plain:.4f}")
            assert plain < 0.0276                                   # measured 0.009
    print("RMSE / R0:", res)
    assert max(res.values()) < 5e-3                                 # measured 1.6e-3, 3e-4, 5e-4
