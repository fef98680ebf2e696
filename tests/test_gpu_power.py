"""GPU parity of both compiled forms of the polytropic power p_b = p_g0 (R0/R)^(3 kappa) (eq. keller_miksis).

The kernels take x^(3 kappa) as x^c (x^(-1/5))^d with the fifth root from Newton's iteration when 3 kappa
is a whole number n of fifths (c = ceil(n/5), d = 5c - n), and as exp2(3 kappa log2 x) otherwise; the form
is compiled into the kernels, and the general one has a single stage shape and no fused epilogue.  Against
the FP64 oracle (which calls the C library's pow):

* the fifth-root form at several splits (c, d) of the exponent: kappa = 1 (n = 15, d = 0), 1.2 (n = 18,
  d = 2), 4/3 (n = 20, d = 0), 1.4 (n = 21, d = 4, air), 5/3 (n = 25, d = 0) on the right-hand side, the
  moments, and split-mode bubble sub-steps;
* the general form (kappa = 1.3, 1.37) on the same, on RK3 trajectories at a size where the fifth-root
  form would fuse the primitive pass, and on the Lagrangian bubble sub-steps;
* the general form rejects stage shapes other than 0, and the autotuner keeps shape 0.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from tests.parity import flux_scale, perturb_bins, rel_err, rhs_err

pytestmark = pytest.mark.gpu
FIFTHS = [1.0, 1.2, 4.0 / 3.0, 1.4, 5.0 / 3.0]
GENERAL = [1.3, 1.37]


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def bub(torch):
    import paper_2511_21031_amd as B
    B.lib()
    return B


def _gpu(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _with_kappa(case, kappa):
    return dataclasses.replace(case, gas=dict(W.AIR, kappa=kappa))


def _bubbly_state(orc, pb, case, seed, amp_r=0.05):
    """Bins away from equilibrium (both signs of R - R0), so the power is taken over a range of R0/R."""
    return perturb_bins(orc.init_state(pb, case.prim), case.ndim, case.nb, seed=seed, amp_r=amp_r)


@pytest.mark.parametrize("kappa", FIFTHS + GENERAL)
@pytest.mark.parametrize("ndim", [2, 3])
def test_rhs_and_moments(torch, bub, orc, kappa, ndim):
    base = W.random_smooth(2, (70, 37), 1e-4, 5, seed=41) if ndim == 2 else \
        W.random_smooth(3, (20, 13, 11), 1e-4, 3, seed=42, bc=1)
    case = _with_kappa(base, kappa)
    pb = orc.problem_from_case(case)
    qh = _bubbly_state(orc, pb, case, seed=8, amp_r=0.4)   # R0/R from about 0.7 to 1.7
    ctx = bub.context_from_case(case)
    got = ctx.rhs_stage(_gpu(torch, qh)).cpu().numpy()
    err = rhs_err(got, orc.rhs(pb, qh), flux_scale(orc, pb, qh))
    assert err.max() < 1e-12, (kappa, err.max())
    m = ctx.moments(_gpu(torch, qh)).cpu().numpy()
    assert rel_err(m, orc.moments(pb, qh)).max() < 1e-12
    assert ctx.last_error()[0] == 0


@pytest.mark.parametrize("kappa", [1.2, 5.0 / 3.0, 1.3])
def test_split_bubble_substeps(torch, bub, orc, kappa):
    """Split mode (adaptive sub-steps of Keller--Miksis) over 5 RK3 steps: within ten times the sub-step
    tolerance of the oracle, and the sub-step counts agree on nearly every cell."""
    case = _with_kappa(W.random_smooth(2, (40, 24), 1e-4, 5, seed=43, amp_atm=1.0), kappa)
    pb = orc.problem_from_case(case, split=1)
    qh = _bubbly_state(orc, pb, case, seed=9)
    ctx = bub.context_from_case(case, bubble_mode=bub.BUBBLES_SPLIT)
    q = _gpu(torch, qh)
    work = ctx.new_work()
    q_ref = qh.copy()
    for _ in range(5):
        dt = orc.cfl_dt(pb, q_ref)
        orc.rk3_step(pb, q_ref, dt)
        ctx.rk3_step(q, work, dt)
    assert ctx.last_error()[0] == 0
    err = rel_err(q.cpu().numpy(), q_ref)
    print(f"kappa {kappa:.4f}: split 5 steps, max field err {err.max():.3e}")
    assert err.max() < 10 * 1e-4


@pytest.mark.parametrize("kappa", GENERAL)
def test_general_power_large_grid_steps(torch, bub, orc, kappa):
    """1024 x 512 with 3 bins: the fifth-root form fuses the next stage's primitive pass here, the general
    form takes the separate pass; 2 RK3 steps against the oracle."""
    case = _with_kappa(W.random_smooth(2, (1024, 512), 1e-4, 3, seed=44), kappa)
    pb = orc.problem_from_case(case)
    qh = _bubbly_state(orc, pb, case, seed=10)
    q_ref, q_pert = qh.copy(), qh * (1.0 + 2e-16 * np.random.default_rng(96).standard_normal(qh.shape))
    ctx = bub.context_from_case(case)
    q = _gpu(torch, qh)
    work = ctx.new_work()
    for _ in range(2):
        dt = orc.cfl_dt(pb, q_ref)
        orc.rk3_step(pb, q_ref, dt)
        orc.rk3_step(pb, q_pert, dt)
        ctx.rk3_step(q, work, dt)
    assert ctx.last_error()[0] == 0
    err, env = rel_err(q.cpu().numpy(), q_ref), rel_err(q_pert, q_ref)
    print(f"kappa {kappa}: 1024x512 x 3 bins, 2 steps: max field err {err.max():.3e} (drift {env.max():.3e})")
    assert np.all(err <= np.maximum(1e-10, 10 * env))


def test_general_power_has_one_stage_shape(torch, bub, orc):
    case = _with_kappa(W.random_smooth(2, (70, 37), 1e-4, 5, seed=41), 1.3)
    pb = orc.problem_from_case(case)
    ctx = bub.context_from_case(case)
    assert len(ctx.tiles()) > 1
    with pytest.raises(bub.BubblyError):
        ctx.tile = 1
    ctx.tile = 0
    q = _gpu(torch, _bubbly_state(orc, pb, case, seed=11))
    best, ms = ctx.autotune(q, reps=2)
    assert best == 0 and ctx.tile == 0 and ms[0] > 0 and all(m == -1.0 for m in ms[1:])


@pytest.mark.parametrize("kappa", [1.2, 1.3])
def test_lagrangian_substeps(torch, bub, orc, kappa):
    """Lagrangian bubbles (Dormand--Prince sub-steps of Keller--Miksis) over 6 steps: within ten times the
    sub-step tolerance of the oracle's radii (1e-8 where every sub-step count agrees)."""
    lc = W.c4(n=16, nbub=80, seed=5, amp_atm=2.0, waves=1)
    gas = dict(W.AIR, kappa=kappa)
    pb = orc.problem(3, lc.n, (lc.dx,) * 3, ((0, 0),) * 3, 1, gas=gas)
    ctx = bub.Context(3, lc.n, (lc.dx,) * 3, ((0, 0),) * 3, 1, gas=gas)
    ql_ref = orc.el_liquid_state(pb, lc.prim)
    b_ref = orc.el_bubbles(pb, lc.bubbles[:3], lc.bubbles[3])
    b_ref[4] *= np.linspace(0.8, 1.25, lc.nbub)     # start away from equilibrium
    a_ref, d_ref = orc.el_smear(pb, b_ref)
    ql, bg = _gpu(torch, ql_ref), _gpu(torch, b_ref)
    aD = ctx.lagrangian_smear(bg)
    work = ctx.lagrangian_work(lc.nbub)
    ns = torch.zeros(lc.nbub, dtype=torch.int32, device="cuda")
    diverged = 0
    for _ in range(6):
        dt, ns_ref = orc.el_step(pb, ql_ref, b_ref, a_ref, d_ref)
        ctx.lagrangian_step(ql, bg, aD, work, dt, nsub=ns)
        diverged += int((ns.cpu().numpy() != ns_ref).sum())
    assert ctx.last_error()[0] == 0
    bq = bg.cpu().numpy()
    tol = 1e-8 if diverged == 0 else 10 * 1e-4
    print(f"kappa {kappa}: EL 6 steps, diverging counts {diverged}, R err {rel_err(bq[4], b_ref[4]):.3e}")
    assert rel_err(bq[4], b_ref[4]) < tol and rel_err(bq[5], b_ref[5]) < tol
