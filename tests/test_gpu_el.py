"""GPU parity of the volume-averaged (Euler--Lagrange) entry points against the CPU oracle.

The smear uses FP64 atomic adds, so sums may be formed in a different order
than the oracle's sequential loop: fields agree to rounding (1e-12 relative).
Adaptive Dormand--Prince sub-steps: bubbles with equal sub-step counts agree to
1e-8, the others to 10 * rtol.
"""
import numpy as np
import pytest

import workloads as W
from tests.parity import rel_err

pytestmark = pytest.mark.gpu
RTOL = 1e-4


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


def _setup(orc, bub, n=16, nbub=60, bc=0, seed=3, amp_atm=2.0, near_walls=True):
    lc = W.c4(n=n, nbub=nbub, seed=seed, amp_atm=amp_atm, waves=1)
    if near_walls:   # some bubbles whose kernel support crosses the domain edge
        lc.bubbles[0, :4] = [0.3e-4, n * 1e-4 - 0.2e-4, 1.5e-4, 5e-4]
        lc.bubbles[1, :4] = [2e-4, 0.1e-4, n * 1e-4 - 0.4e-4, 5e-4]
    pb = orc.problem(3, lc.n, (lc.dx,) * 3, ((bc, bc),) * 3, 1)
    ctx = bub.Context(3, lc.n, (lc.dx,) * 3, ((bc, bc),) * 3, 1)
    return lc, pb, ctx


def _check_forcing(pb, f, f_ref):
    """Gathered p_l: the stiffened-gas pressure is a difference of terms of size gamma*pi_inf,
    so its rounding is measured against max|p| + gamma*pi_inf; rho_l and c directly."""
    scale = np.abs(f_ref[0]).max() + pb.gamma * pb.pi_inf
    assert np.abs(f[0] - f_ref[0]).max() / scale < 1e-15 * 10
    assert rel_err(f[1], f_ref[1]) < 1e-14 and rel_err(f[2], f_ref[2]) < 1e-13


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("n", [16, 8, 18])
def test_smear_and_gather(torch, bub, orc, bc, n):
    """Grids of 16, 8 and 18 cells a side: on the smaller ones the wide supports wrap around the
    periodic box more often, or lie further outside the reflective one."""
    lc, pb, ctx = _setup(orc, bub, n=n, bc=bc)
    bub_h = orc.el_bubbles(pb, lc.bubbles[:3], lc.bubbles[3])
    bub_h[4] *= np.linspace(0.9, 1.3, lc.nbub)
    bub_h[5] = np.linspace(-2, 2, lc.nbub)
    # large bubbles (kernel width h = R > dx): supports 11 and 19 cells wide, more (x, y) columns
    # than a wavefront has lanes, and 67 cells wide, more z planes than lanes (wrapping around the
    # periodic box several times, or mostly outside the reflective one)
    bub_h[4, 2:5] = [1.5e-4, 2.9e-4, 11.0e-4]
    a_ref, d_ref = orc.el_smear(pb, bub_h)
    b_g = _gpu(torch, bub_h)
    aD = ctx.lagrangian_smear(b_g).cpu().numpy()
    assert rel_err(aD[0], a_ref) < 1e-12 and rel_err(aD[1], d_ref) < 1e-12
    ql = orc.el_liquid_state(pb, lc.prim)
    f_ref = orc.el_gather(pb, ql, bub_h)
    f = ctx.lagrangian_gather(_gpu(torch, ql), b_g).cpu().numpy()
    _check_forcing(pb, f, f_ref)
    # the bubble records built on the device match the oracle's
    b0 = ctx.lagrangian_bubbles(_gpu(torch, lc.bubbles)).cpu().numpy()
    assert rel_err(b0, orc.el_bubbles(pb, lc.bubbles[:3], lc.bubbles[3])).max() < 1e-15


@pytest.mark.parametrize("bc", [0, 1])
def test_liquid_rhs(torch, bub, orc, bc):
    lc, pb, ctx = _setup(orc, bub, bc=bc)
    bub_h = orc.el_bubbles(pb, lc.bubbles[:3], lc.bubbles[3])
    bub_h[5] = np.linspace(-3, 3, lc.nbub)
    a, d = orc.el_smear(pb, bub_h)
    ql = orc.el_liquid_state(pb, lc.prim)
    ref = orc.el_rhs(pb, ql, a, d)
    got = ctx.lagrangian_rhs(_gpu(torch, ql), _gpu(torch, np.vstack([a, d]))).cpu().numpy()
    lam_dx = 1.0 / 1e-4 * 1500.0
    scale = np.abs(ref).max(axis=1) + lam_dx * np.abs(ql).max(axis=1)
    scale[1:4] += np.abs(lc.prim[4]).max() / 1e-4
    err = np.abs(got - ref).max(axis=1) / scale
    assert err.max() < 1e-12, err


def test_step_trajectory(torch, bub, orc):
    lc, pb, ctx = _setup(orc, bub, n=16, nbub=80)
    ql_ref = orc.el_liquid_state(pb, lc.prim)
    b_ref = orc.el_bubbles(pb, lc.bubbles[:3], lc.bubbles[3])
    a_ref, d_ref = orc.el_smear(pb, b_ref)
    ql = _gpu(torch, ql_ref)
    bg = _gpu(torch, b_ref)
    aD = ctx.lagrangian_smear(bg)
    work = ctx.lagrangian_work(lc.nbub)
    ns = torch.zeros(lc.nbub, dtype=torch.int32, device="cuda")
    diverged = 0
    for _ in range(10):
        dt, ns_ref = orc.el_step(pb, ql_ref, b_ref, a_ref, d_ref)
        ctx.lagrangian_step(ql, bg, aD, work, dt, nsub=ns)
        diverged += int((ns.cpu().numpy() != ns_ref).sum())
    assert ctx.last_error()[0] == 0
    bq = bg.cpu().numpy()
    same = True if diverged == 0 else False
    tol = 1e-8 if same else 10 * RTOL
    print("EL 10 steps: diverging sub-step counts", diverged, "R err", rel_err(bq[4], b_ref[4]),
          "ql err", rel_err(ql.cpu().numpy(), ql_ref).max())
    assert rel_err(bq[4], b_ref[4]) < tol and rel_err(bq[5], b_ref[5]) < tol
    assert rel_err(ql.cpu().numpy(), ql_ref).max() < tol
    assert rel_err(aD.cpu().numpy()[0], a_ref) < tol


def test_multi_step_call(torch, bub, orc):
    """lagrangian_steps(10), which makes only the last step's closing smear, against ten single-step calls
    and ten oracle steps, all with the CFL step size; zero steps change nothing."""
    lc, pb, ctx = _setup(orc, bub, n=16, nbub=80)
    ql0 = orc.el_liquid_state(pb, lc.prim)
    b0 = orc.el_bubbles(pb, lc.bubbles[:3], lc.bubbles[3])
    b0[4] *= np.linspace(0.9, 1.2, lc.nbub)     # away from equilibrium
    ql_ref, b_ref = ql0.copy(), b0.copy()
    a_ref, d_ref = orc.el_smear(pb, b_ref)
    for _ in range(10):
        orc.el_step(pb, ql_ref, b_ref, a_ref, d_ref)
    runs = []
    for multi in (True, False):
        ql, bg = _gpu(torch, ql0), _gpu(torch, b0)
        aD = ctx.lagrangian_smear(bg)
        work = ctx.lagrangian_work(lc.nbub)
        if multi:
            before = ql.clone()
            ctx.lagrangian_steps(ql, bg, aD, work, 0)
            assert torch.equal(ql, before)
            ctx.lagrangian_steps(ql, bg, aD, work, 10)
        else:
            for _ in range(10):
                ctx.lagrangian_step(ql, bg, aD, work)
        assert ctx.last_error()[0] == 0
        runs.append((ql.cpu().numpy(), bg.cpu().numpy(), aD.cpu().numpy()))
    (qm, bm, am), (qs, bs, as_) = runs
    print("multi vs single: ql", rel_err(qm, qs).max(), "R", rel_err(bm[4], bs[4]),
          "; multi vs oracle: ql", rel_err(qm, ql_ref).max(), "R", rel_err(bm[4], b_ref[4]))
    tol = 10 * RTOL   # the smears' atomic order may move a bubble's sub-step count
    for q, b, a in runs:
        assert rel_err(q, ql_ref).max() < tol
        assert rel_err(b[4], b_ref[4]) < tol and rel_err(b[5], b_ref[5]) < tol
        assert rel_err(a[0], a_ref) < tol and rel_err(a[1], d_ref) < tol
    assert rel_err(qm, qs).max() < tol and rel_err(bm[4], bs[4]) < tol


def test_full_size_smear_gather_and_steps(torch, bub, orc):
    """192^3 with 1e5 bubbles: full smear and gather against the oracle, then two whole steps on the GPU."""
    lc = W.c4()
    pb = orc.problem(3, lc.n, (lc.dx,) * 3, ((0, 0),) * 3, 1)
    ctx = bub.Context(3, lc.n, (lc.dx,) * 3, ((0, 0),) * 3, 1)
    b_ref = orc.el_bubbles(pb, lc.bubbles[:3], lc.bubbles[3])
    bg = ctx.lagrangian_bubbles(_gpu(torch, lc.bubbles))
    a_ref, d_ref = orc.el_smear(pb, b_ref)
    aD = ctx.lagrangian_smear(bg)
    assert rel_err(aD[0].cpu().numpy(), a_ref) < 1e-12
    ql_ref = orc.el_liquid_state(pb, lc.prim)
    ql = ctx.lagrangian_init(_gpu(torch, lc.prim))
    assert rel_err(ql.cpu().numpy(), ql_ref).max() < 1e-15
    f_ref = orc.el_gather(pb, ql_ref, b_ref)
    f = ctx.lagrangian_gather(ql, bg).cpu().numpy()
    _check_forcing(pb, f, f_ref)
    work = ctx.lagrangian_work(lc.nbub)
    for _ in range(2):
        ctx.lagrangian_step(ql, bg, aD, work)
    assert ctx.last_error()[0] == 0
    assert torch.isfinite(ql).all().item() and torch.isfinite(bg).all().item()
