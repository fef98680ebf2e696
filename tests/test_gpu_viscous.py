"""GPU parity of the viscous stress (eq. stressTensor in eq. euler_transport) against the FP64 oracle.

The GPU adds the stress in a pass after each stage kernel; the oracle adds it to each face flux.  With a
viscosity large enough that the stress is comparable to the pressure flux, the right-hand sides must agree to
the rounding bar of the inviscid tests, and the viscous part alone (viscous minus inviscid right-hand side on
each side) to 1e-9 of its size.  Through the C ABI.
"""
import numpy as np
import pytest

import workloads as W
from tests.parity import flux_scale, perturb_bins, rel_err, rhs_err

pytestmark = pytest.mark.gpu
MU = 5.0   # Pa s: stress ~ mu u/dx ~ 1e5 Pa, the size of the pressure (right-hand sides only)
# Trajectories take the acoustic CFL step, which must stay inside the explicit viscous limit
# rho dx^2 / (2 ndim mu): at dx = 1e-4 m that is 5e-10 s for MU but 5e-8 s for 0.05 Pa s, above the
# acoustic step of about 2e-8 s.
MU_STEPS = 0.05


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


def _case(kind, mu=MU):
    if kind == "1d_reflective":
        c = W.random_smooth(1, (61,), 1e-4, 3, seed=51, bc=1)
    elif kind == "2d_ragged_periodic":
        c = W.random_smooth(2, (70, 37), 1e-4, 5, seed=52)
    elif kind == "2d_reflective":
        c = W.random_smooth(2, (33, 20), 1e-4, 3, seed=53, bc=1)
    else:
        c = W.random_smooth(3, (20, 13, 11), 1e-4, 3, seed=54, bc=1)
    c.gas = dict(c.gas, mu=mu)
    return c


def _pair(orc, bub, case, viscous, **kw):
    pb = orc.problem_from_case(case, viscous=viscous)
    return pb, bub.context_from_case(case, viscous=viscous, **kw)


KINDS = ["1d_reflective", "2d_ragged_periodic", "2d_reflective", "3d_ragged_reflective"]


@pytest.mark.parametrize("kind", KINDS)
def test_viscous_rhs_matches_oracle(torch, bub, orc, kind):
    case = _case(kind)
    pb1, ctx1 = _pair(orc, bub, case, 1)
    pb0, ctx0 = _pair(orc, bub, case, 0)
    qh = perturb_bins(orc.init_state(pb1, case.prim), case.ndim, case.nb, seed=2)
    q = torch.from_numpy(qh).cuda()
    ref1, ref0 = orc.rhs(pb1, qh), orc.rhs(pb0, qh)
    got1, got0 = ctx1.rhs_stage(q).cpu().numpy(), ctx0.rhs_stage(q).cpu().numpy()
    assert rhs_err(got1, ref1, flux_scale(orc, pb1, qh)).max() < 1e-12
    mom_e = list(range(1, case.ndim + 2))                   # momentum and energy rows
    dv_ref, dv_got = (ref1 - ref0)[mom_e], (got1 - got0)[mom_e]
    # the viscous part stands far enough above the rounding of the inviscid rates it is taken from that
    # the 1e-9 bar below measures it
    assert np.abs(dv_ref).max() > 1e-6 * np.abs(ref0[mom_e]).max()
    err = np.abs(dv_got - dv_ref).max(axis=1) / np.abs(dv_ref).max(axis=1)
    print(f"{kind}: viscous part, max rel err per row {err}")
    assert err.max() < 1e-9
    others = [r for r in range(ref1.shape[0]) if r not in mom_e]
    assert np.array_equal(got1[others], got0[others])        # mass, alpha and bins do not see the stress


def test_viscous_rhs_tile_shapes_identical(torch, bub, orc):
    case = _case("2d_ragged_periodic")
    pb, ctx = _pair(orc, bub, case, 1)
    q = torch.from_numpy(perturb_bins(orc.init_state(pb, case.prim), 2, case.nb, seed=3)).cuda()
    outs = []
    for v in range(len(ctx.tiles())):
        ctx.tile = v
        outs.append(ctx.rhs_stage(q).cpu().numpy())
    assert all(np.array_equal(o, outs[0]) for o in outs[1:])


@pytest.mark.parametrize("kind", ["2d_reflective", "3d_ragged_reflective"])
def test_viscous_trajectory_matches_oracle(torch, bub, orc, kind):
    case = _case(kind, MU_STEPS)
    pb, ctx = _pair(orc, bub, case, 1)
    q_ref = orc.init_state(pb, case.prim)
    q_pert = q_ref * (1.0 + 2e-16 * np.random.default_rng(96).standard_normal(q_ref.shape))
    q = ctx.init_state(torch.from_numpy(case.prim).cuda())
    work = ctx.new_work()
    for _ in range(10):
        dt = orc.cfl_dt(pb, q_ref)
        orc.rk3_step(pb, q_ref, dt)
        orc.rk3_step(pb, q_pert, dt)
        ctx.rk3_step(q, work, dt)
    assert ctx.last_error()[0] == 0
    err, env = rel_err(q.cpu().numpy(), q_ref), rel_err(q_pert, q_ref)
    print(f"{kind} viscous, 10 steps: max field err {err.max():.3e} (oracle drift {env.max():.3e})")
    assert np.all(err <= np.maximum(1e-10, 10 * env))
