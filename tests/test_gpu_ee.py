"""GPU parity of the ensemble-averaged hot path against the FP64 CPU oracle.

Every GPU result goes through the C ABI (libbubbly.so) via the binding.  The
tolerance for plain FP64 is 1e-10 max-norm relative per field (rounding-order
differences only: the two sides share no code).
"""
import numpy as np
import pytest

import workloads as W
from tests.parity import flux_scale, perturb_bins, rel_err, rhs_err

pytestmark = pytest.mark.gpu
TOL = 1e-10       # states: max-norm relative per field
RHS_TOL = 1e-12   # rates: relative to the flux-divergence scale (see tests/parity.py)


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


def _case_grid(kind):
    if kind == "c1":
        return W.c1()
    if kind == "2d_ragged_periodic":
        return W.random_smooth(2, (70, 37), 1e-4, 5, seed=21)
    if kind == "2d_reflective":
        return W.random_smooth(2, (33, 20), 1e-4, 3, seed=22, bc=1)
    if kind == "2d_nb31":
        return W.random_smooth(2, (40, 24), 1e-4, 31, seed=23, sigma_ln=0.5)
    if kind == "3d_ragged_reflective":
        return W.random_smooth(3, (20, 13, 11), 1e-4, 3, seed=24, bc=1)
    if kind == "3d_periodic_mono":
        return W.random_smooth(3, (16, 9, 10), 1e-4, 1, seed=25)
    if kind == "tiny_2d_periodic":
        return W.random_smooth(2, (7, 2), 1e-4, 3, seed=26)
    if kind == "tiny_2d_reflective":
        return W.random_smooth(2, (5, 3), 1e-4, 3, seed=27, bc=1)
    if kind == "tiny_1d_reflective":
        return W.random_smooth(1, (3,), 1e-4, 3, seed=28, bc=1)
    raise KeyError(kind)


CASES = ["c1", "2d_ragged_periodic", "2d_reflective", "2d_nb31", "3d_ragged_reflective", "3d_periodic_mono",
         "tiny_2d_periodic", "tiny_2d_reflective", "tiny_1d_reflective"]


@pytest.mark.parametrize("kind", ["c1", "2d_ragged_periodic", "3d_ragged_reflective"])
def test_init_state(torch, bub, orc, kind):
    case = _case_grid(kind)
    pb = orc.problem_from_case(case)
    q_ref = orc.init_state(pb, case.prim)
    ctx = bub.context_from_case(case)
    q = ctx.init_state(_gpu(torch, case.prim))
    assert rel_err(q.cpu().numpy(), q_ref).max() < 1e-14


@pytest.mark.parametrize("kind", CASES)
def test_moments(torch, bub, orc, kind):
    case = _case_grid(kind)
    pb = orc.problem_from_case(case)
    q = perturb_bins(orc.init_state(pb, case.prim), case.ndim, case.nb, seed=1)
    ref = orc.moments(pb, q)
    ctx = bub.context_from_case(case)
    got = ctx.moments(_gpu(torch, q)).cpu().numpy()
    err = rel_err(got, ref)
    assert err.max() < 1e-12, err
    assert ctx.last_error()[0] == 0


@pytest.mark.parametrize("kind", CASES)
def test_rhs_stage(torch, bub, orc, kind):
    case = _case_grid(kind)
    pb = orc.problem_from_case(case)
    q = perturb_bins(orc.init_state(pb, case.prim), case.ndim, case.nb, seed=2)
    ref = orc.rhs(pb, q)
    ctx = bub.context_from_case(case)
    got = ctx.rhs_stage(_gpu(torch, q)).cpu().numpy()
    err = rhs_err(got, ref, flux_scale(orc, pb, q))
    print(kind, "max err per field", err.max())
    assert err.max() < RHS_TOL, err
    assert ctx.last_error()[0] == 0


def test_cfl_dt(torch, bub, orc):
    case = W.c2(n=48, nb=5)
    pb = orc.problem_from_case(case)
    q_ref = orc.init_state(pb, case.prim)
    dt_ref = orc.cfl_dt(pb, q_ref)
    ctx = bub.context_from_case(case)
    q = ctx.init_state(_gpu(torch, case.prim))
    work = ctx.new_work()
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.rk3_step(q, work, 0.0, dt_dev)
    assert abs(dt_dev.item() / dt_ref - 1) < 1e-14


def _run_both(torch, bub, orc, case, steps):
    """GPU and oracle trajectories from the same primitives, plus the oracle's own rounding envelope.

    The envelope is the per-field drift of the oracle when its initial state is
    perturbed at the 2e-16 relative level: how far rounding alone moves this
    trajectory.  Long runs are held to a multiple of it (see trajectory tests).
    """
    pb = orc.problem_from_case(case)
    q_ref = orc.init_state(pb, case.prim)
    rng = np.random.default_rng(99)
    q_pert = q_ref * (1.0 + 2e-16 * rng.standard_normal(q_ref.shape))
    ctx = bub.context_from_case(case)
    q = ctx.init_state(_gpu(torch, case.prim))
    work = ctx.new_work()
    dts = []
    for _ in range(steps):
        dt = orc.cfl_dt(pb, q_ref)
        dts.append(dt)
        orc.rk3_step(pb, q_ref, dt)
        orc.rk3_step(pb, q_pert, dt)
        ctx.rk3_step(q, work, 0.0)      # the GPU computes its own CFL step on the device
    assert ctx.last_error()[0] == 0
    envelope = rel_err(q_pert, q_ref)
    return q.cpu().numpy(), q_ref, pb, envelope


def _assert_within_rounding(got, ref, envelope):
    err = rel_err(got, ref)
    bound = np.maximum(10.0 * envelope, 1e-12)
    assert np.all(err <= bound), (err / bound).max()
    return err


def test_rk3_c1_full_trajectory(torch, bub, orc):
    """The 400-cell 1D workload, all 200 CFL steps."""
    case = W.c1()
    got, ref, pb, env = _run_both(torch, bub, orc, case, case.steps)
    err = _assert_within_rounding(got, ref, env)
    print("c1 200 steps: max rel err", err.max(), "oracle rounding envelope", env.max())
    assert err.max() < 1e-8
    m_got = orc.moments(pb, got)
    m_ref = orc.moments(pb, ref)
    assert rel_err(m_got[[1, 6, 7]], m_ref[[1, 6, 7]]).max() < TOL   # alpha, p_mix, p_l


def test_rk3_2d_plane_wave(torch, bub, orc):
    case = W.c2(n=64, nb=11)
    got, ref, _, env = _run_both(torch, bub, orc, case, 10)
    _assert_within_rounding(got, ref, env)


def test_rk3_3d_pulse(torch, bub, orc):
    case = W.random_smooth(3, (24, 20, 16), 1e-4, 3, seed=31, bc=1, amp_atm=0.3)
    got, ref, _, env = _run_both(torch, bub, orc, case, 5)
    _assert_within_rounding(got, ref, env)


def test_full_size_2d_sampled_rhs(torch, bub, orc):
    """1024^2 with 31 bins (the benchmark workload): RHS at sampled cells, incl. tile and domain edges."""
    case = W.c2()
    pb = orc.problem_from_case(case)
    ctx = bub.context_from_case(case)
    # seeded off-equilibrium bins (input recipe) so every source term is exercised; both sides get this state
    qh = perturb_bins(orc.init_state(pb, case.prim), case.ndim, case.nb, seed=3)
    rhs = ctx.rhs_stage(_gpu(torch, qh))
    rng = np.random.default_rng(5)
    n = 1024
    pick = list(rng.integers(0, n * n, 200))
    for x, y in [(0, 0), (n - 1, n - 1), (31, 7), (32, 8), (0, 517), (1023, 300), (511, 0)]:
        pick.append(y * n + x)
    cells = np.array(pick, dtype=np.int64)
    ref = orc.rhs_cells(pb, qh, cells)
    got = rhs.cpu().numpy()[:, cells].T
    err = rhs_err(got.T, ref.T, flux_scale(orc, pb, qh))
    assert err.max() < RHS_TOL, err


def test_full_size_2d_conservation(torch, bub, orc):
    case = W.c2()
    ctx = bub.context_from_case(case)
    q = ctx.init_state(_gpu(torch, case.prim))
    work = ctx.new_work()
    tot0 = q[:4].sum(dim=1)
    for _ in range(3):
        ctx.rk3_step(q, work)
    tot = q[:4].sum(dim=1)
    scale = q[:4].abs().sum(dim=1)
    assert ((tot - tot0).abs() / scale).max().item() < 1e-13
    assert ctx.last_error()[0] == 0


def test_error_word_nonfinite_and_negative_radius(torch, bub, orc):
    case = W.c1(n=64, length=64 * 2.5e-4, nb=3)
    ctx = bub.context_from_case(case)
    q = ctx.init_state(_gpu(torch, case.prim))
    work = ctx.new_work()
    q[2, 17] = float("nan")          # energy of cell 17 (1D slots: rho, m, E, alpha, nR.., nRdot..)
    ctx.rk3_step(q, work, 1e-9)
    code, cell, _ = ctx.last_error()
    assert code == -4 and cell == 17
    assert ctx.last_error()[0] == 0  # cleared
    q = ctx.init_state(_gpu(torch, case.prim))
    q[4 + 1, 40] = -q[4 + 1, 40]    # nR of bin 1 at cell 40
    ctx.moments(q)
    code, cell, b = ctx.last_error()
    assert code == -5 and cell == 40 and b == 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["c1", "2d_ragged_periodic", "3d_ragged_reflective"])
def test_tile_shapes_give_identical_results(torch, bub, orc, kind, prec):
    """Every compiled tile shape (the autotuner's candidates, in both precisions) computes each face
    flux with the same arithmetic: bitwise equal right-hand sides and RK3 steps."""
    case = _case_grid(kind)
    pb = orc.problem_from_case(case)
    q0 = _gpu(torch, perturb_bins(orc.init_state(pb, case.prim), case.ndim, case.nb, seed=4))
    P = bub.PREC_FP64 if prec == "fp64" else bub.PREC_MIXED
    ctx = bub.context_from_case(case, precision=P)
    work = ctx.new_work()
    outs = []
    for v in range(len(ctx.tiles())):
        ctx.tile = v
        q = q0.clone()
        rhs = ctx.rhs_stage(q)
        for _ in range(3):
            ctx.rk3_step(q, work)
        assert ctx.last_error()[0] == 0
        outs.append((rhs.cpu().numpy(), q.cpu().numpy()))
    for v, (r, st) in enumerate(outs[1:], 1):
        assert np.array_equal(r, outs[0][0]), (prec, ctx.tiles()[v])
        assert np.array_equal(st, outs[0][1]), (prec, ctx.tiles()[v])
    best, ms = ctx.autotune(q0, reps=2)
    assert ctx.tile == best and 0 <= best < len(ms) and all(m > 0 for m in ms)


@pytest.mark.timeout(900)
def test_c2_shaped_fp64_trajectory(torch, bub, orc):
    """The benchmark's recipe at 256^2 (31 bins, sigma 0.5, periodic, 1 atm plane wave), 100 RK3 steps of
    plain FP64 with the device's own CFL step: every field within 1e-10 (max-norm relative) of the oracle,
    or within 10x the oracle's own drift under a 2e-16 perturbation of its start where that is larger."""
    case = W.c2(n=256)
    pb = orc.problem_from_case(case)
    q_ref = orc.init_state(pb, case.prim)
    q_pert = q_ref * (1.0 + 2e-16 * np.random.default_rng(98).standard_normal(q_ref.shape))
    ctx = bub.context_from_case(case)
    q = ctx.init_state(_gpu(torch, case.prim))
    work = ctx.new_work()
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(100):
        dt = orc.cfl_dt(pb, q_ref)
        orc.rk3_step(pb, q_ref, dt)
        orc.rk3_step(pb, q_pert, dt)
        ctx.rk3_step(q, work, 0.0, dt_dev)
        assert abs(dt_dev.item() / dt - 1) < 1e-12
    assert ctx.last_error()[0] == 0
    got = q.cpu().numpy()
    err, env = rel_err(got, q_ref), rel_err(q_pert, q_ref)
    print(f"256^2 x 31 bins, 100 steps: max field err {err.max():.3e} (oracle drift {env.max():.3e})")
    assert np.all(err <= np.maximum(1e-10, 10 * env)), (err.max(), env.max())
    mg, mr = orc.moments(pb, got), orc.moments(pb, q_ref)
    assert rel_err(mg[[1, 6]], mr[[1, 6]]).max() < 1e-10   # alpha and the mixture pressure


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["c1", "2d_ragged_periodic", "3d_ragged_reflective"])
def test_bin_groups_give_identical_results(torch, bub, orc, kind, prec):
    """Splitting a tile's bins over several workgroups leaves every result bitwise unchanged."""
    case = _case_grid(kind)
    pb = orc.problem_from_case(case)
    q0 = _gpu(torch, perturb_bins(orc.init_state(pb, case.prim), case.ndim, case.nb, seed=4))
    P = bub.PREC_FP64 if prec == "fp64" else bub.PREC_MIXED
    outs = []
    for groups in (1, 0, 2, 3, case.nb):
        ctx = bub.context_from_case(case, precision=P)
        ctx.set_bin_groups(groups)
        q = q0.clone()
        work = ctx.new_work()
        rhs = ctx.rhs_stage(q)
        for _ in range(2):
            ctx.rk3_step(q, work)
        assert ctx.last_error()[0] == 0
        outs.append((rhs.cpu().numpy(), q.cpu().numpy()))
    for r, s in outs[1:]:
        assert np.array_equal(r, outs[0][0]) and np.array_equal(s, outs[0][1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(1024, 512, 1), (84, 84, 84)])
def test_fused_primitive_pass_is_bitwise_the_separate_pass(torch, bub, orc, shape, prec):
    """From 2^19 cells on, stages 1 and 2 write the next stage's primitives from their epilogue (not in
    3D FP64, which always takes the separate pass); two workgroups per tile (forced) take the
    separate primitive pass instead.  Same arithmetic, same bin
    order: the steps must agree bit for bit (right-hand sides and states)."""
    ndim = 2 if shape[2] == 1 else 3
    n = shape[:ndim]
    case = W.random_smooth(ndim, n, 1e-4, 5, seed=31, bc=1 if ndim == 3 else 0)
    pb = orc.problem_from_case(case)
    q0 = _gpu(torch, perturb_bins(orc.init_state(pb, case.prim), ndim, 5, seed=5))
    P = bub.PREC_FP64 if prec == "fp64" else bub.PREC_MIXED
    outs = []
    for groups in (0, 2):
        ctx = bub.context_from_case(case, precision=P)
        ctx.set_bin_groups(groups)
        q = q0.clone()
        work = ctx.new_work()
        for _ in range(2):
            ctx.rk3_step(q, work)
        assert ctx.last_error()[0] == 0
        outs.append(q.cpu().numpy())
        del ctx, work
    assert np.array_equal(outs[0], outs[1])


def test_fused_steps_match_oracle(torch, bub, orc):
    """Fused stages at 1024 x 512 (5 bins, periodic, perturbed bins): 3 RK3 steps against the oracle."""
    case = W.random_smooth(2, (1024, 512), 1e-4, 5, seed=32)
    pb = orc.problem_from_case(case)
    qh = perturb_bins(orc.init_state(pb, case.prim), 2, 5, seed=6)
    q_ref, q_pert = qh.copy(), qh * (1.0 + 2e-16 * np.random.default_rng(97).standard_normal(qh.shape))
    ctx = bub.context_from_case(case)
    q = _gpu(torch, qh)
    work = ctx.new_work()
    for _ in range(3):
        dt = orc.cfl_dt(pb, q_ref)
        orc.rk3_step(pb, q_ref, dt)
        orc.rk3_step(pb, q_pert, dt)
        ctx.rk3_step(q, work, dt)
    assert ctx.last_error()[0] == 0
    err, env = rel_err(q.cpu().numpy(), q_ref), rel_err(q_pert, q_ref)
    print(f"fused 1024x512 x 5 bins, 3 steps: max field err {err.max():.3e} (oracle drift {env.max():.3e})")
    assert np.all(err <= np.maximum(1e-10, 10 * env))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rk3_steps_is_bitwise_repeated_steps(torch, bub, orc, prec):
    """rk3_steps(n) carries the primitives and wave speeds of each step's result to the next step from
    the third stage's epilogue; the states and time steps must be those of n separate calls, bit for bit."""
    case = W.random_smooth(2, (1024, 520), 1e-4, 3, seed=33)
    pb = orc.problem_from_case(case)
    q0 = _gpu(torch, perturb_bins(orc.init_state(pb, case.prim), 2, 3, seed=7))
    P = bub.PREC_FP64 if prec == "fp64" else bub.PREC_MIXED
    ctx = bub.context_from_case(case, precision=P)
    work = ctx.new_work()
    dts = torch.zeros(4, dtype=torch.float64, device="cuda")
    qa = q0.clone()
    for k in range(4):
        ctx.rk3_step(qa, work, 0.0, dts[k:k + 1])
    qb = q0.clone()
    dtb = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.rk3_steps(qb, work, 4, 0.0, dtb)
    assert ctx.last_error()[0] == 0
    assert torch.equal(qa, qb)
    assert dtb.item() == dts[3].item() and dts.min().item() > 0
