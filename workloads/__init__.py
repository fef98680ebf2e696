"""Seeded synthetic inputs for the phase-averaged bubbly-flow hot path.

This module is shared by the CPU oracle tests and by the GPU path.  It holds
no arithmetic of the method itself: it only builds the *inputs* -- grids,
physical constants, initial primitive fields (liquid density, velocity,
liquid pressure, void fraction), Lagrangian bubble sets and the serving
request stream -- with the shapes and value ranges of the workloads below.
Conversion of these primitive fields to conserved variables, the bin
quadrature and everything after it is computed independently by each side.

All quantities are SI.  Arrays are float64, structure-of-arrays, laid out
``[field][z][y][x]`` with x fastest (``N = nx*ny*nz`` cells per field).

Workloads (water as a stiffened gas, air bubbles, polytropic contents):

* ``c1``  1D, 400 cells over 0.1 m, reflective ends, 11 bins (lognormal
  sigma 0.3 about 10 um), alpha 1e-4, Gaussian pulse of 0.5 atm (standard
  deviation 2 mm) centred at x = 0.02 m, CFL 0.3, 200 RK3 steps.
* ``c2``  2D 1024^2 periodic, dx = 100 um, 31 bins (sigma 0.5),
  alpha = 1e-4 (1 + 0.5 sin sin), right-running plane sine wave of 1 atm
  with 21 wavelengths across the box (about 302 kHz), 100 RK3 steps.
* ``c3``  3D 256^3 reflective, dx = 100 um, 21 bins (sigma 0.3),
  alpha 1e-4, centred spherical Gaussian overpressure of 10 atm
  (standard deviation 2 mm).
* ``c4``  3D 192^3 periodic Lagrangian case: 1e5 bubbles uniform in the
  central half-box, R0 = 10 um * exp(0.3 Z), plane sine wave of 2 atm
  with 4 wavelengths across the box, 500 steps.
* ``c5``  stream of 512 solves with Poisson arrivals (rate 20/s): 70 % 1D
  (N uniform in 200..4000), 25 % 2D (side 64..512), 5 % 3D 96^3; bins in
  {11, 21, 31}; alpha log-uniform in [1e-5, 1e-3]; amplitude 0.1..5 atm;
  50..500 steps.
* ``acoustic_tube`` / ``pulse_tube``  the validation set-ups of the one-way
  acoustic source and the non-reflective boundaries: water at rest in a tube
  with non-reflective ends, either driven by a planar sine burst of 50 cells
  per wavelength emitted from the middle, or carrying a right-running
  Gaussian pulse (p' = P exp(-((x - x0)/w)^2), u' = p'/(rho0 c0),
  rho' = p'/c0^2) toward the right end.

Every size can be shrunk by argument so that tests run the same recipe on
grids the CPU oracle finishes in seconds.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

ATM = 101325.0

# Water (stiffened gas) and air bubble constants of the workloads.
WATER = dict(gamma=7.1, pi_inf=3.06e8, rho0=1000.0, p0=101325.0)
AIR = dict(kappa=1.4, sigma=0.0728, mu=1.0e-3, pv=0.0)

# Bubble contents with heat and vapour transfer: air and water vapour at 20 C (handbook properties; the
# paper gives none).  The transfer coefficients beta = 5 are those of a parabolic profile inside the bubble
# (f - f_wall proportional to 1 - r^2/R^2 has wall gradient 5 (f_wall - mean)/R), the slow-oscillation
# limit; callers pass their own.  The vapour pressure is the gas dict's pv.
AIR_VAPOUR = dict(gam_b=1.4, Rg=287.06, Rv=461.52, T0=293.15, k_b=0.0257, D_v=2.42e-5, beta_T=5.0, beta_c=5.0)
PV_WATER_20C = 2339.0
AIR_WITH_VAPOUR = dict(AIR, pv=PV_WATER_20C)

# Boundary codes shared by both sides' problem descriptions.
BC_PERIODIC = 0
BC_REFLECTIVE = 1
BC_NONREFLECTIVE = 2


def c0_water() -> float:
    """Small-amplitude sound speed of the undisturbed water (input recipe only)."""
    w = WATER
    return math.sqrt(w["gamma"] * (w["p0"] + w["pi_inf"]) / w["rho0"])


@dataclass
class Case:
    """One ensemble-averaged problem: grid, physics constants, bins, primitives."""
    name: str
    ndim: int
    n: tuple            # (nx, ny, nz), unused dims are 1
    dx: tuple           # (dx, dy, dz) in m
    bc: tuple           # ((lo, hi), (lo, hi), (lo, hi)) boundary codes
    nb: int             # number of equilibrium-radius bins (odd)
    r0_median: float
    sigma_ln: float
    cfl: float
    steps: int
    prim: np.ndarray    # [ndim+3][N]: rho_l, u_1..ndim, p_l, alpha
    liquid: dict = field(default_factory=lambda: dict(WATER))
    gas: dict = field(default_factory=lambda: dict(AIR))
    contents: dict | None = None   # None: polytropic gas; else transfer-contents constants (AIR_VAPOUR)

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def nvar(self) -> int:
        return self.ndim + 3 + (4 if self.contents else 2) * self.nb


def _centres(n: int, dx: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * dx


def _pack(fields, n):
    nx, ny, nz = n
    out = np.empty((len(fields), nz * ny * nx), dtype=np.float64)
    for k, f in enumerate(fields):
        out[k] = np.broadcast_to(f, (nz, ny, nx)).reshape(-1)
    return out


def c1(n: int = 400, length: float = 0.1, nb: int = 11, steps: int = 200,
       amp_atm: float = 0.5, alpha: float = 1e-4) -> Case:
    """1D reflective tube with a Gaussian pressure pulse (the 400-cell workload)."""
    dx = length / n
    x = _centres(n, dx)
    w = WATER
    p = w["p0"] + amp_atm * ATM * np.exp(-(x - 0.2 * length) ** 2 / (2.0 * (2e-3) ** 2))
    rho = np.full(n, w["rho0"])
    u = np.zeros(n)
    a = np.full(n, alpha)
    prim = _pack([rho[None, None, :], u[None, None, :], p[None, None, :], a[None, None, :]], (n, 1, 1))
    return Case("c1", 1, (n, 1, 1), (dx, 1.0, 1.0),
                ((BC_REFLECTIVE, BC_REFLECTIVE), (BC_PERIODIC, BC_PERIODIC), (BC_PERIODIC, BC_PERIODIC)),
                nb, 10e-6, 0.3, 0.3, steps, prim)


def c2(n: int = 1024, dx: float = 1e-4, nb: int = 31, steps: int = 100,
       amp_atm: float = 1.0, waves: int | None = None) -> Case:
    """2D periodic box driven by a right-running plane sine wave (the 1024^2 workload)."""
    length = n * dx
    if waves is None:
        waves = max(1, int(round(21 * n / 1024)))
    x = _centres(n, dx)
    y = _centres(n, dx)
    w = WATER
    c0 = c0_water()
    dp = amp_atm * ATM * np.sin(2 * np.pi * waves * x / length)
    p = (w["p0"] + dp)[None, None, :]
    u = (dp / (w["rho0"] * c0))[None, None, :]
    rho = (w["rho0"] + dp / c0 ** 2)[None, None, :]
    v = np.zeros((1, 1, 1))
    a = 1e-4 * (1.0 + 0.5 * np.sin(2 * np.pi * x / length)[None, None, :]
                * np.sin(2 * np.pi * y / length)[None, :, None])
    prim = _pack([rho, u, v, p, a], (n, n, 1))
    return Case("c2", 2, (n, n, 1), (dx, dx, 1.0),
                ((BC_PERIODIC, BC_PERIODIC), (BC_PERIODIC, BC_PERIODIC), (BC_PERIODIC, BC_PERIODIC)),
                nb, 10e-6, 0.5, 0.3, steps, prim)


def c3(n: int = 256, dx: float = 1e-4, nb: int = 21, steps: int = 100,
       amp_atm: float = 10.0, width: float = 2e-3) -> Case:
    """3D reflective box with a centred spherical Gaussian overpressure (the 256^3 workload)."""
    length = n * dx
    x = _centres(n, dx) - 0.5 * length
    w = WATER
    r2 = x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2
    p = w["p0"] + amp_atm * ATM * np.exp(-r2 / (2.0 * width ** 2))
    rho = np.full((1, 1, 1), w["rho0"])
    z0 = np.zeros((1, 1, 1))
    a = np.full((1, 1, 1), 1e-4)
    prim = _pack([rho, z0, z0, z0, p, a], (n, n, n))
    rb = ((BC_REFLECTIVE, BC_REFLECTIVE),) * 3
    return Case("c3", 3, (n, n, n), (dx, dx, dx), rb, nb, 10e-6, 0.3, 0.3, steps, prim)


def uniform(ndim: int, n: tuple, dx: float, nb: int, *, rho=1000.0, u=(0.0, 0.0, 0.0),
            p=101325.0, alpha=1e-4, sigma_ln=0.3, bc=BC_PERIODIC, cfl=0.3) -> Case:
    """A uniform state (free-stream and 0D tests)."""
    nn = tuple(list(n) + [1] * (3 - len(n)))
    fields = [np.full((1, 1, 1), rho)] + [np.full((1, 1, 1), u[d]) for d in range(ndim)] \
        + [np.full((1, 1, 1), p), np.full((1, 1, 1), alpha)]
    prim = _pack(fields, nn)
    return Case("uniform", ndim, nn, (dx, dx, dx), ((bc, bc),) * 3, nb, 10e-6, sigma_ln, cfl, 1, prim)


def random_smooth(ndim: int, n: tuple, dx: float, nb: int, seed: int, *, bc=BC_PERIODIC,
                  sigma_ln=0.3, amp_atm=0.5, umax=2.0, alpha=1e-4) -> Case:
    """Seeded smooth random field: a few random Fourier modes on each primitive."""
    rng = np.random.default_rng(seed)
    nn = tuple(list(n) + [1] * (3 - len(n)))
    L = [nn[d] * dx for d in range(3)]
    xs = [_centres(nn[d], dx) for d in range(3)]
    X = xs[0][None, None, :]
    Y = xs[1][None, :, None]
    Z = xs[2][:, None, None]

    def modes(scale):
        f = np.zeros((nn[2], nn[1], nn[0]))
        for _ in range(3):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi, size=3)
            term = np.sin(2 * np.pi * k[0] * X / L[0] + ph[0])
            if ndim > 1:
                term = term * np.cos(2 * np.pi * k[1] * Y / L[1] + ph[1])
            if ndim > 2:
                term = term * np.cos(2 * np.pi * k[2] * Z / L[2] + ph[2])
            f = f + rng.uniform(-1, 1) * term
        return scale * f / 3.0

    w = WATER
    rho = w["rho0"] * (1.0 + modes(0.01))
    us = [modes(umax) for _ in range(ndim)]
    p = w["p0"] + modes(amp_atm * ATM)
    a = alpha * (1.0 + 0.5 * modes(1.0))
    prim = _pack([rho] + us + [p, a], nn)
    return Case("random", ndim, nn, (dx, dx, dx), ((bc, bc),) * 3, nb, 10e-6, sigma_ln, 0.3, 1, prim)


# ---------------------------------------------------------------------------
# Lagrangian (volume-averaged) workload
# ---------------------------------------------------------------------------

@dataclass
class LagrangianCase:
    n: tuple
    dx: float
    nbub: int
    bubbles: np.ndarray   # [4][nbub]: x, y, z, R0
    prim: np.ndarray      # [5][N]: rho_l, u, v, w, p_l
    steps: int
    liquid: dict = field(default_factory=lambda: dict(WATER))
    gas: dict = field(default_factory=lambda: dict(AIR))

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


def c4(n: int = 192, dx: float = 1e-4, nbub: int = 100_000, seed: int = 2511,
       amp_atm: float = 2.0, waves: int = 4, steps: int = 500) -> LagrangianCase:
    """3D periodic Lagrangian case: bubbles uniform in the central half-box."""
    rng = np.random.default_rng(seed)
    length = n * dx
    pos = rng.uniform(0.25 * length, 0.75 * length, size=(3, nbub))
    r0 = 10e-6 * np.exp(0.3 * rng.standard_normal(nbub))
    x = _centres(n, dx)
    w = WATER
    c0 = c0_water()
    dp = amp_atm * ATM * np.sin(2 * np.pi * waves * x / length)
    p = (w["p0"] + dp)[None, None, :]
    u = (dp / (w["rho0"] * c0))[None, None, :]
    rho = (w["rho0"] + dp / c0 ** 2)[None, None, :]
    z0 = np.zeros((1, 1, 1))
    prim = _pack([rho, u, z0, z0, p], (n, n, n))
    bub = np.vstack([pos, r0[None, :]])
    return LagrangianCase((n, n, n), dx, nbub, bub, prim, steps)


# ---------------------------------------------------------------------------
# Serving stream
# ---------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival: float
    ndim: int
    n: tuple
    dx: float
    nb: int
    alpha: float
    amp_atm: float
    steps: int


def c5_stream(count: int = 512, seed: int = 21031, rate: float = 20.0,
              scale: float = 1.0) -> list:
    """Seeded request stream; ``scale`` < 1 shrinks grids and step counts for tests."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        kind = rng.uniform()
        if kind < 0.70:
            nd = 1
            nx = int(rng.integers(200, 4001))
            n = (max(16, int(nx * scale)), 1, 1)
            dx = 0.1 / n[0]
        elif kind < 0.95:
            nd = 2
            s = int(rng.integers(64, 513))
            s = max(16, int(s * scale))
            n = (s, s, 1)
            dx = 1e-4
        else:
            nd = 3
            s = max(8, int(96 * scale))
            n = (s, s, s)
            dx = 1e-4
        nb = int(rng.choice([11, 21, 31]))
        alpha = float(10 ** rng.uniform(-5, -3))
        amp = float(rng.uniform(0.1, 5.0))
        steps = max(2, int(int(rng.integers(50, 501)) * scale))
        out.append(Request(rid, t, nd, n, dx, nb, alpha, amp, steps))
    return out


def request_case(r: Request) -> Case:
    """Initial primitives of one serving request: a Gaussian pulse in a reflective box."""
    nn = r.n
    length = [nn[d] * r.dx for d in range(3)]
    width = max(2e-3, 4 * r.dx)
    xs = [_centres(nn[d], r.dx) for d in range(3)]
    w = WATER
    if r.ndim == 1:
        r2 = ((xs[0] - 0.2 * length[0]) ** 2)[None, None, :]
    else:
        r2 = ((xs[0] - 0.5 * length[0]) ** 2)[None, None, :] + ((xs[1] - 0.5 * length[1]) ** 2)[None, :, None]
        if r.ndim == 3:
            r2 = r2 + ((xs[2] - 0.5 * length[2]) ** 2)[:, None, None]
    p = w["p0"] + r.amp_atm * ATM * np.exp(-r2 / (2.0 * width ** 2))
    rho = np.full((1, 1, 1), w["rho0"])
    z0 = np.zeros((1, 1, 1))
    a = np.full((1, 1, 1), r.alpha)
    prim = _pack([rho] + [z0] * r.ndim + [p, a], nn)
    rb = ((BC_REFLECTIVE, BC_REFLECTIVE),) * 3
    return Case(f"req{r.rid}", r.ndim, nn, (r.dx, r.dx, r.dx), rb, r.nb, 10e-6, 0.3, 0.3, r.steps, prim)


# ---------------------------------------------------------------------------
# Acoustic source and non-reflective boundary set-ups
# ---------------------------------------------------------------------------

def source_burst(axis: int, sign: int, x: float, dx: float, *, cells_per_wavelength: float = 50.0,
                 width_cells: float = 3.0, amp: float = 1e3, cycles: float = 3.0, t0: float = 0.0) -> dict:
    """Parameters of a planar sine burst (frequency from the wavelength in cells at the water sound speed)."""
    f = c0_water() / (cells_per_wavelength * dx)
    return dict(dir=axis, sign=sign, x=x, width=width_cells * dx, amp=amp, freq=f, t0=t0, ncyc=cycles)


def acoustic_tube(ndim: int = 1, n: int = 600, length: float = 0.15, nb: int = 1, *, alpha: float = 0.0,
                  axis: int = 0, ncross: int = 4, bc=BC_NONREFLECTIVE, cfl: float = 0.3,
                  r0_median: float = 10e-6) -> Case:
    """Water at rest with the given void fraction; `n` cells of length/n along `axis`, `ncross` periodic
    cells across it (2D and 3D); non-reflective ends along the axis."""
    dx = length / n
    nn = [1, 1, 1]
    for d in range(ndim):
        nn[d] = n if d == axis else ncross
    nn = tuple(nn)
    w = WATER
    fields = [np.full((1, 1, 1), w["rho0"])] + [np.zeros((1, 1, 1))] * ndim \
        + [np.full((1, 1, 1), w["p0"]), np.full((1, 1, 1), alpha)]
    bcs = tuple((bc, bc) if d == axis else (BC_PERIODIC, BC_PERIODIC) for d in range(3))
    return Case("acoustic_tube", ndim, nn, (dx, dx, dx), bcs, nb, r0_median, 0.3, cfl, 1, _pack(fields, nn))


def isolated_bubble(cells_per_wavelength: float = 50.0, cfl: float = 0.2):
    """The isolated-bubble validation set-up: a 50 um air bubble in water (one bin, trace void fraction so
    the bubble does not act on the liquid), driven by one cycle of a 0.2 MPa, 150 kHz plane wave emitted at
    a quarter of a four-wavelength tube with non-reflective ends; returns (case, source, probe cell)."""
    f = 150e3
    dx = c0_water() / f / cells_per_wavelength
    n = int(round(4 * cells_per_wavelength))
    case = acoustic_tube(1, n=n, length=n * dx, nb=1, alpha=1e-8, cfl=cfl, r0_median=50e-6)
    src = source_burst(0, 1, 0.25 * n * dx, dx, cells_per_wavelength=cells_per_wavelength, amp=2e5, cycles=1.0)
    return case, src, int(0.6 * n)


def pulse_tube(n: int = 400, length: float = 0.1, *, amp: float = 1e3, x0_frac: float = 0.6,
               width_cells: float = 12.0, nb: int = 1, alpha: float = 0.0, bc=BC_NONREFLECTIVE) -> Case:
    """1D water tube carrying a right-running Gaussian acoustic pulse (linear acoustics initial data)."""
    dx = length / n
    x = _centres(n, dx)
    c0 = c0_water()
    w = WATER
    pp = amp * np.exp(-((x - x0_frac * length) / (width_cells * dx)) ** 2)
    prim = np.stack([w["rho0"] + pp / c0 ** 2, pp / (w["rho0"] * c0), w["p0"] + pp, np.full(n, alpha)])
    return Case("pulse_tube", 1, (n, 1, 1), (dx, 1.0, 1.0), ((bc, bc), (BC_PERIODIC, BC_PERIODIC),
                (BC_PERIODIC, BC_PERIODIC)), nb, 10e-6, 0.3, 0.3, 1, prim)
