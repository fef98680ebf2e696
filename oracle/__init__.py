"""ctypes wrapper of the plain FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``; never by the product package.  It
imports nothing from the GPU package: the seeded inputs come from
``workloads`` and every number is computed by the C oracle in this folder.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (IEEE doubles, OpenMP)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=gnu99", "-Wall", "-fPIC", "-fopenmp", "-shared",
               os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle_el.c"),
               "-o", _SO + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
        ("bc", (ctypes.c_int * 2) * 3),
        ("gamma", ctypes.c_double), ("pi_inf", ctypes.c_double), ("rho0", ctypes.c_double),
        ("p0", ctypes.c_double),
        ("kappa", ctypes.c_double), ("sigma", ctypes.c_double), ("mu", ctypes.c_double),
        ("pv", ctypes.c_double),
        ("nb", ctypes.c_int), ("r0_median", ctypes.c_double), ("sigma_ln", ctypes.c_double),
        ("cfl", ctypes.c_double), ("split", ctypes.c_int), ("sub_rtol", ctypes.c_double),
        ("max_substeps", ctypes.c_int), ("viscous", ctypes.c_int),
        ("t", ctypes.c_double), ("src_on", ctypes.c_int), ("src_dir", ctypes.c_int), ("src_sign", ctypes.c_int),
        ("src_x", ctypes.c_double), ("src_width", ctypes.c_double), ("src_amp", ctypes.c_double),
        ("src_freq", ctypes.c_double), ("src_t0", ctypes.c_double), ("src_ncyc", ctypes.c_double),
        ("contents", ctypes.c_int), ("gam_b", ctypes.c_double), ("Rg", ctypes.c_double), ("Rv", ctypes.c_double),
        ("T0", ctypes.c_double), ("k_b", ctypes.c_double), ("D_v", ctypes.c_double),
        ("beta_T", ctypes.c_double), ("beta_c", ctypes.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER(Problem)
        L.orc_bins.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_init_state.argtypes = [P, _dp, _dp]
        L.orc_moments.argtypes = [P, _dp, _dp]
        L.orc_rhs.argtypes = [P, _dp, _dp]
        L.orc_rhs_flux_only.argtypes = [P, _dp, _dp]
        L.orc_rhs_cells.argtypes = [P, _dp, _lp, ctypes.c_int64, _dp]
        L.orc_cfl_dt.argtypes = [P, _dp]
        L.orc_cfl_dt.restype = ctypes.c_double
        L.orc_rk3_step.argtypes = [P, _dp, ctypes.c_double, _dp]
        L.orc_bubble_advance.argtypes = [P, _dp, ctypes.c_double, _ip]
        L.orc_km_rddot.argtypes = [P] + [ctypes.c_double] * 7
        L.orc_km_rddot.restype = ctypes.c_double
        L.orc_km_rddot_pb.argtypes = [P] + [ctypes.c_double] * 7
        L.orc_km_rddot_pb.restype = ctypes.c_double
        L.orc_contents_rates.argtypes = [P] + [ctypes.c_double] * 5 + [_dp, _dp]
        L.orc_contents_rates.restype = None
        L.orc_weno5.argtypes = [_dp]
        L.orc_weno5.restype = ctypes.c_double
        L.orc_hllc.argtypes = [P, ctypes.c_int, _dp, _dp, _dp]
        L.orc_km_integrate.argtypes = [P] + [ctypes.c_double] * 10 + [ctypes.c_int, _dp, _dp, _dp,
                                                                         ctypes.c_double, _dp]
        L.orc_km_integrate.restype = ctypes.c_int64
        L.orc_source_amplitude.argtypes = [P, ctypes.c_double]
        L.orc_source_amplitude.restype = ctypes.c_double
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_el_kernel.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_el_kernel.restype = ctypes.c_double
        L.orc_el_smear.argtypes = [P, _dp, ctypes.c_int64, _dp, _dp]
        L.orc_el_gather.argtypes = [P, _dp, _dp, ctypes.c_int64, _dp, _dp, _dp]
        L.orc_el_rhs.argtypes = [P, _dp, _dp, _dp, _dp]
        L.orc_el_step.argtypes = [P, _dp, _dp, ctypes.c_int64, ctypes.c_double, _dp, _dp, _ip, _dp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def problem(ndim, n, dx, bc, nb, r0_median=10e-6, sigma_ln=0.3, cfl=0.3, liquid=None, gas=None,
            split=0, sub_rtol=1e-4, max_substeps=10000, viscous=0, source=None, t=0.0, contents=None) -> Problem:
    """source: dict(dir, sign, x, width, amp, freq, t0=0, ncyc=0) of the one-way acoustic source.
    contents: None (polytropic gas) or dict(gam_b, Rg, Rv, T0, k_b, D_v, beta_T, beta_c) of the transfer
    contents (the vapour pressure is the gas dict's pv)."""
    from workloads import WATER, AIR
    liquid = liquid or WATER
    gas = gas or AIR
    pb = Problem()
    pb.ndim = ndim
    for d in range(3):
        pb.n[d] = int(n[d])
        pb.dx[d] = float(dx[d])
        pb.bc[d][0] = int(bc[d][0])
        pb.bc[d][1] = int(bc[d][1])
    pb.gamma, pb.pi_inf, pb.rho0, pb.p0 = liquid["gamma"], liquid["pi_inf"], liquid["rho0"], liquid["p0"]
    pb.kappa, pb.sigma, pb.mu, pb.pv = gas["kappa"], gas["sigma"], gas["mu"], gas["pv"]
    pb.nb = nb
    pb.r0_median = r0_median
    pb.sigma_ln = sigma_ln
    pb.cfl = cfl
    pb.split = int(split)
    pb.sub_rtol = sub_rtol
    pb.max_substeps = int(max_substeps)
    pb.viscous = int(viscous)
    pb.t = float(t)
    if source:
        set_source(pb, **source)
    if contents:
        set_contents(pb, **contents)
    return pb


def set_contents(pb, gam_b, Rg, Rv, T0, k_b, D_v, beta_T, beta_c):
    pb.contents = 1
    pb.gam_b, pb.Rg, pb.Rv, pb.T0 = float(gam_b), float(Rg), float(Rv), float(T0)
    pb.k_b, pb.D_v, pb.beta_T, pb.beta_c = float(k_b), float(D_v), float(beta_T), float(beta_c)


def km_rddot_pb(pb, R, V, p_b, pdot_b, pinf, rho, c):
    return lib().orc_km_rddot_pb(ctypes.byref(pb), R, V, p_b, pdot_b, pinf, rho, c)


def contents_rates(pb, R, V, p_b, m_v, mg):
    """(dp_b/dt, dm_v/dt) of one bubble with transfer contents."""
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_contents_rates(ctypes.byref(pb), R, V, p_b, m_v, mg, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def set_source(pb, dir, sign, x, width, amp, freq, t0=0.0, ncyc=0.0):
    pb.src_on = 1
    pb.src_dir, pb.src_sign = int(dir), int(sign)
    pb.src_x, pb.src_width, pb.src_amp = float(x), float(width), float(amp)
    pb.src_freq, pb.src_t0, pb.src_ncyc = float(freq), float(t0), float(ncyc)


def source_amplitude(pb, t):
    return lib().orc_source_amplitude(ctypes.byref(pb), float(t))


def problem_from_case(case, **kw) -> Problem:
    kw.setdefault("contents", getattr(case, "contents", None))
    return problem(case.ndim, case.n, case.dx, case.bc, case.nb, case.r0_median, case.sigma_ln,
                   case.cfl, case.liquid, case.gas, **kw)


def nvar(pb) -> int:
    return pb.ndim + 3 + (4 if pb.contents else 2) * pb.nb


def ncells(pb) -> int:
    return pb.n[0] * pb.n[1] * pb.n[2]


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    """Threads of later oracle calls (OpenMP)."""
    lib().orc_set_threads(int(n))


def bins(nb, r0_median, sigma_ln):
    r0 = np.zeros(nb)
    w = np.zeros(nb)
    _check(lib().orc_bins(nb, r0_median, sigma_ln, _ptr(r0), _ptr(w)), "bins")
    return r0, w


def init_state(pb, prim):
    prim = _c(prim)
    q = np.zeros((nvar(pb), ncells(pb)))
    _check(lib().orc_init_state(ctypes.byref(pb), _ptr(prim), _ptr(q)), "init_state")
    return q


def rhs(pb, q, sources=True):
    q = _c(q)
    out = np.zeros_like(q)
    f = lib().orc_rhs if sources else lib().orc_rhs_flux_only
    _check(f(ctypes.byref(pb), _ptr(q), _ptr(out)), "rhs")
    return out


def rhs_cells(pb, q, cells):
    q = _c(q)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), nvar(pb)))
    _check(lib().orc_rhs_cells(ctypes.byref(pb), _ptr(q), cells.ctypes.data_as(_lp), len(cells),
                               _ptr(out)), "rhs_cells")
    return out


def moments(pb, q):
    q = _c(q)
    out = np.zeros((8, ncells(pb)))
    _check(lib().orc_moments(ctypes.byref(pb), _ptr(q), _ptr(out)), "moments")
    return out


def cfl_dt(pb, q):
    return lib().orc_cfl_dt(ctypes.byref(pb), _ptr(_c(q)))


def rk3_step(pb, q, dt=0.0):
    """Advance q (float64, C-contiguous, modified in place) and the clock pb.t; return the step used."""
    assert q.dtype == np.float64 and q.flags.c_contiguous
    used = ctypes.c_double(0.0)
    _check(lib().orc_rk3_step(ctypes.byref(pb), _ptr(q), float(dt), ctypes.byref(used)), "rk3_step")
    pb.t += used.value
    return used.value


def bubble_advance(pb, q, dt):
    assert q.dtype == np.float64 and q.flags.c_contiguous
    ns = np.zeros((pb.nb, ncells(pb)), dtype=np.int32)
    rc = lib().orc_bubble_advance(ctypes.byref(pb), _ptr(q), float(dt), ns.ctypes.data_as(_ip))
    _check(rc, "bubble_advance")
    return ns


def km_rddot(pb, R, V, R0, pg0, pinf, rho, c):
    return lib().orc_km_rddot(ctypes.byref(pb), R, V, R0, pg0, pinf, rho, c)


def weno5(v):
    v = _c(v)
    assert v.shape == (5,)
    return lib().orc_weno5(_ptr(v))


def hllc(pb, direction, WL, WR):
    WL, WR = _c(WL), _c(WR)
    F = np.zeros(nvar(pb))
    _check(lib().orc_hllc(ctypes.byref(pb), direction, _ptr(WL), _ptr(WR), _ptr(F)), "hllc")
    return F


def km_integrate(pb, R0, pg0, pinf, rho, c, R_init, V_init, t_out, rtol=1e-10, atol_r=1e-16,
                 atol_v=1e-10, r_stop=0.0):
    t_out = _c(t_out)
    R = np.zeros_like(t_out)
    V = np.zeros_like(t_out)
    ts = ctypes.c_double(-1.0)
    steps = lib().orc_km_integrate(ctypes.byref(pb), R0, pg0, pinf, rho, c, R_init, V_init, rtol,
                                   atol_r, atol_v, len(t_out), _ptr(t_out), _ptr(R), _ptr(V),
                                   r_stop, ctypes.byref(ts))
    if steps < 0:
        raise RuntimeError("km_integrate did not finish")
    return R, V, ts.value, steps


# ---------------------------------------------------------------------------
# Volume-averaged (Euler--Lagrange) variant
# ---------------------------------------------------------------------------

def el_kernel(d, h):
    return lib().orc_el_kernel(float(d), float(h))


def el_bubbles(pb, positions, r0):
    """Bubble SoA [8][nbub] at rest at their equilibrium radius (x, y, z, R0, R, Rdot, pg0, h_sub)."""
    nb = positions.shape[1]
    b = np.zeros((8, nb))
    b[0:3] = positions
    b[3] = r0
    b[4] = r0
    b[5] = 0.0
    b[6] = pb.p0 + 2.0 * pb.sigma / r0 - pb.pv
    b[7] = 0.0
    return b


def el_liquid_state(pb, prim):
    """Liquid conserved [5][N] from primitives [5][N] = rho_l, u, v, w, p_l."""
    rho = prim[0]
    u = prim[1:4]
    p = prim[4]
    q = np.empty_like(prim)
    q[0] = rho
    q[1:4] = rho * u
    q[4] = (p + pb.gamma * pb.pi_inf) / (pb.gamma - 1.0) + 0.5 * rho * (u * u).sum(axis=0)
    return q


def el_smear(pb, bub):
    bub = _c(bub)
    N = ncells(pb)
    a = np.zeros(N)
    d = np.zeros(N)
    _check(lib().orc_el_smear(ctypes.byref(pb), _ptr(bub), bub.shape[1], _ptr(a), _ptr(d)), "el_smear")
    return a, d


def el_gather(pb, ql, bub):
    bub = _c(bub)
    nb = bub.shape[1]
    p, r, c = np.zeros(nb), np.zeros(nb), np.zeros(nb)
    _check(lib().orc_el_gather(ctypes.byref(pb), _ptr(_c(ql)), _ptr(bub), nb, _ptr(p), _ptr(r), _ptr(c)),
           "el_gather")
    return p, r, c


def el_rhs(pb, ql, alpha, dalpha):
    ql = _c(ql)
    out = np.zeros_like(ql)
    _check(lib().orc_el_rhs(ctypes.byref(pb), _ptr(ql), _ptr(_c(alpha)), _ptr(_c(dalpha)), _ptr(out)), "el_rhs")
    return out


def el_step(pb, ql, bub, alpha, dalpha, dt=0.0):
    """One Strang-split Lagrangian step in place (the clock pb.t advances); returns (dt_used, accepted
    sub-steps per bubble)."""
    for a in (ql, bub, alpha, dalpha):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    ns = np.zeros(bub.shape[1], dtype=np.int32)
    used = ctypes.c_double(0.0)
    rc = lib().orc_el_step(ctypes.byref(pb), _ptr(ql), _ptr(bub), bub.shape[1], float(dt), _ptr(alpha),
                           _ptr(dalpha), ns.ctypes.data_as(_ip), ctypes.byref(used))
    _check(rc, "el_step")
    pb.t += used.value
    return used.value, ns
