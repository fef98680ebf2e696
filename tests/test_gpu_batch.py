"""Batches of resident problems and the continuous-batching server on the GPU.

A batch member runs the arithmetic of bub_rk3_step on its own buffers (its own
kernels on one of the batch's lanes; only the stream, the block order and the
tile shape the class autotuner picks may differ, and results depend on none of
them), so its state after k batched steps must be bitwise the state after k
bub_rk3_step calls on its own context, whatever the other members are and
whenever the member joined.  The server's
results must likewise be bitwise the results of each request solved alone, and
stay within the split-mode bound of the FP64 oracle run on its own.
"""
import numpy as np
import pytest

import workloads as W
from tests.parity import rel_err

pytestmark = pytest.mark.gpu
TOL_SPLIT = 10 * 1e-4     # ten times the bubble sub-step tolerance


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


def _members():
    """Uneven 1D/2D/3D problems, unsplit and split, ragged tiles (name, case, split)."""
    req = W.c5_stream(count=4, seed=3, scale=0.05)
    return [
        ("c1", W.c1(), False),
        ("2d_periodic", W.random_smooth(2, (70, 37), 1e-4, 5, seed=41), False),
        ("3d_reflective", W.random_smooth(3, (20, 13, 11), 1e-4, 3, seed=42, bc=1), False),
        ("3d_collapse_split", W.c3(n=12, nb=5, width=6e-4), True),
        ("request_split", W.request_case(req[0]), True),
    ]


def _alone(torch, bub, case, split, prec, steps):
    ctx = bub.context_from_case(case, precision=prec, bubble_mode=bub.BUBBLES_SPLIT if split else bub.BUBBLES_UNSPLIT)
    q = ctx.init_state(_gpu(torch, case.prim))
    work = ctx.new_work()
    for _ in range(steps):
        ctx.rk3_step(q, work)
    assert ctx.last_error()[0] == 0
    return q


def _fresh(torch, bub, case, split, prec):
    ctx = bub.context_from_case(case, precision=prec, bubble_mode=bub.BUBBLES_SPLIT if split else bub.BUBBLES_UNSPLIT)
    q = ctx.init_state(_gpu(torch, case.prim))
    return ctx, q, ctx.new_work()


def _join(torch, bub, batch, case, split, prec):
    ctx, q, work = _fresh(torch, bub, case, split, prec)
    return batch.add(ctx, q, work), (ctx, q, work)


GROUPED_OFF = ("the grouped launches of bub_batch_run are switched off in the library: on the GPU they once "
               "returned corrupted member states and once faulted the device; run block by block on the host "
               "they reproduce every member bitwise, and the device-side cause is not found yet")


@pytest.mark.skip(reason=GROUPED_OFF)
@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_grouped_batch_members_bitwise_equal_alone(torch, bub, prec, graphs):
    """bub_batch_run in its grouped form: one launch per phase and kernel class for every member (one
    graph launch per chunk)."""
    _run_members_join_leave(torch, bub, prec, graphs)


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_run_members_bitwise_equal_alone(torch, bub, prec, graphs):
    """bub_batch_run: members with their own step counts join and leave; each ends bitwise equal to its
    problem stepped alone, and bub_batch_poll reports every member once, after its last step has
    completed."""
    _run_members_join_leave(torch, bub, prec, graphs)


def _run_members_join_leave(torch, bub, prec, graphs):
    P = bub.PREC_FP64 if prec == "fp64" else bub.PREC_MIXED
    mem = _members()
    want = {"c1": 5, "2d_periodic": 3, "3d_reflective": 6, "3d_collapse_split": 4, "request_split": 2}
    batch = bub.Batch(P, max_cases=8)
    batch.set_graphs(graphs)
    slots, held = {}, {}
    for name, case, split in mem[:4]:
        ctx, q, work = _fresh(torch, bub, case, split, P)
        slots[name] = batch.add(ctx, q, work, steps=want[name])
        held[name] = (ctx, q, work)
    assert batch.run(10) == 3                       # never past the member with the fewest steps left
    torch.cuda.synchronize()
    assert batch.poll() == [slots["2d_periodic"]]
    assert batch.poll() == []
    batch.remove(slots["2d_periodic"])
    name, case, split = mem[4]
    ctx, q, work = _fresh(torch, bub, case, split, P)
    slots[name] = batch.add(ctx, q, work, steps=want[name])
    held[name] = (ctx, q, work)
    reported, chunks = [], []
    while True:
        n = batch.run(10)
        if n == 0:
            break
        chunks.append(n)
        reported += batch.poll()
    assert chunks == [1, 1, 1] and sum(chunks) + 3 == want["3d_reflective"]
    torch.cuda.synchronize()
    reported += batch.poll()
    assert sorted(reported) == sorted(slots[k] for k in want if k != "2d_periodic")
    assert all(batch.remaining(slots[k]) == 0 for k in want if k != "2d_periodic")
    diffs = {}
    for name, case, split in mem:
        ctx, q, _ = held[name]
        assert ctx.last_error()[0] == 0, name
        ref = _alone(torch, bub, case, split, P, want[name])
        diffs[name] = [] if torch.equal(q, ref) else (q - ref).abs().amax(dim=1).tolist()
    print("members differing from their problem alone (max |diff| per row):",
          {k: v for k, v in diffs.items() if v})
    assert not any(diffs.values())
    batch.close()


def test_batch_run_open_members_and_budget(torch, bub):
    """Open-ended members (steps = 0) take every chunk and are never reported; the byte budget refuses a
    member that does not fit and takes one again after a removal."""
    P = bub.PREC_FP64
    mem = _members()
    a = _fresh(torch, bub, mem[0][1], False, P)
    b = _fresh(torch, bub, mem[1][1], False, P)
    need_a = 3 * a[0].state_bytes + bub.ctx_buffer_bytes(a[0].ndim, a[0].n, a[0].nb)
    need_b = 3 * b[0].state_bytes + bub.ctx_buffer_bytes(b[0].ndim, b[0].n, b[0].nb)
    batch = bub.Batch(P, max_cases=4, hbm_budget=need_a + need_b - 1)
    sa = batch.add(*a)
    with pytest.raises(bub.BubblyError) as e:
        batch.add(*b)
    assert e.value.code == -2
    assert batch.run(4) == 4 and batch.run(3) == 3
    torch.cuda.synchronize()
    assert batch.poll() == [] and batch.remaining(sa) == -1
    assert torch.equal(a[1], _alone(torch, bub, mem[0][1], False, P, 7))
    batch.remove(sa)
    sb = batch.add(*b, steps=2)
    assert batch.run(4) == 2
    torch.cuda.synchronize()
    assert batch.poll() == [sb]
    assert torch.equal(b[1], _alone(torch, bub, mem[1][1], False, P, 2))
    batch.close()


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_stream_batch_members_bitwise_equal_alone(torch, bub, prec, graphs):
    """Members join and leave a running batch; each ends bitwise equal to its problem stepped alone."""
    P = bub.PREC_FP64 if prec == "fp64" else bub.PREC_MIXED
    mem = _members()
    batch = bub.Batch(P, max_cases=8)
    batch.set_graphs(graphs)
    slots, held, steps = {}, {}, {}
    for name, case, split in mem[:4]:
        slots[name], held[name] = _join(torch, bub, batch, case, split, P)
        steps[name] = 0
    batch.step(3)
    for name in slots:
        steps[name] += 3
    batch.remove(slots.pop("2d_periodic"))
    name, case, split = mem[4]
    slots[name], held[name] = _join(torch, bub, batch, case, split, P)
    steps[name] = 0
    n, cells, cb = batch.info()
    assert n == 4 and cells == sum(held[k][0].ncells for k in slots)
    batch.step(2)
    for name in slots:
        steps[name] += 2
    torch.cuda.synchronize()
    for name, case, split in mem:
        ctx, q, _ = held[name]
        assert ctx.last_error()[0] == 0, name
        ref = _alone(torch, bub, case, split, P, steps[name])
        assert torch.equal(q, ref), (name, (q - ref).abs().max().item())
    batch.close()


def test_stream_batch_class_autotune(torch, bub):
    """One tuned tile per (ndim, nb) class, applied to members present and joining later; states untouched."""
    P = bub.PREC_FP64
    mem = _members()
    batch = bub.Batch(P, max_cases=8)
    held = {name: _join(torch, bub, batch, case, split, P)[1] for name, case, split in mem[:4]}
    before = {k: v[1].clone() for k, v in held.items()}
    classes = batch.autotune(reps=2)
    assert classes == len({(c.ndim, c.nb) for _, c, _ in mem[:4]})
    for k, v in held.items():
        assert torch.equal(v[1], before[k])
        assert 0 <= v[0].tile < len(v[0].tiles())
    # a later member of an already tuned class gets the class's tile
    late_name, late_case, late_split = mem[0]
    _, late = _join(torch, bub, batch, late_case, late_split, P)
    assert late[0].tile == held[late_name][0].tile
    batch.step(2)
    torch.cuda.synchronize()
    for name, case, split in mem[:4]:
        assert torch.equal(held[name][1], _alone(torch, bub, case, split, P, 2)), name
    assert torch.equal(late[1], _alone(torch, bub, late_case, late_split, P, 2))
    batch.close()


def test_autotune_cache_persists_choices(torch, bub, tmp_path):
    """bub_autotune_cached: a miss tunes and appends one line keyed by (arch, ndim, nb, precision,
    floor(log2 N)); a later context of the same key takes the stored shape without timing; lines that do
    not parse or name no valid shape are ignored; the batch's class autotuner reads the same file."""
    case = W.random_smooth(2, (70, 37), 1e-4, 5, seed=41)
    path = tmp_path / "tiles.txt"
    path.write_text("not an entry\ngfx950 2 5 0 11 99\n")
    ctx = bub.context_from_case(case)
    q = ctx.init_state(_gpu(torch, case.prim))
    best, hit = ctx.autotune_cached(str(path), q, reps=2)
    assert not hit and ctx.tile == best
    lines = path.read_text().splitlines()
    assert len(lines) == 3
    arch, nd, nb, prec, sc, tile = lines[-1].split()
    assert (int(nd), int(nb), int(prec), int(sc), int(tile)) == (2, 5, 0, 11, best)   # 70 x 37 = 2590 cells
    # the same key again: the cached shape, no new line
    path.write_text(path.read_text() + f"{arch} 2 5 0 11 {(best + 1) % len(ctx.tiles())}\n"
                    + f"{arch} 2 5 0 11 {best}\n")                                      # the last match wins
    ctx2 = bub.context_from_case(case)
    ctx2.tile = (best + 2) % len(ctx2.tiles())
    best2, hit2 = ctx2.autotune_cached(str(path), q)
    assert hit2 and best2 == best and ctx2.tile == best
    assert len(path.read_text().splitlines()) == 5
    # another size class or precision is a miss
    mixed = bub.context_from_case(case, precision=bub.PREC_MIXED)
    _, hit3 = mixed.autotune_cached(str(path), q, reps=2)
    assert not hit3 and len(path.read_text().splitlines()) == 6
    # the batch's class autotuner takes the cached shape of a member's class
    batch = bub.Batch(bub.PREC_FP64, max_cases=2)
    batch.set_tune_cache(str(path))
    ctx3, q3, w3 = _fresh(torch, bub, case, False, bub.PREC_FP64)
    ctx3.tile = (best + 1) % len(ctx3.tiles())
    batch.add(ctx3, q3, w3)
    assert batch.autotune(reps=2) == 1
    assert ctx3.tile == best and len(path.read_text().splitlines()) == 6
    batch.close()


def test_graph_replays_match_eager_steps(torch, bub):
    """Every replay of the captured member steps, with eager work and host syncs in between,
    matches a twin of each member stepped eagerly, bitwise."""
    P = bub.PREC_FP64
    mem = _members()
    batch = bub.Batch(P, max_cases=8)
    held = [_join(torch, bub, batch, case, split, P)[1] for _, case, split in mem]
    twins = [_fresh(torch, bub, case, split, P) for _, case, split in mem]
    for rnd in range(4):
        batch.step(1)
        torch.cuda.synchronize()
        for (ctx, q, work) in twins:          # eager work between the replays
            ctx.rk3_step(q, work)
        torch.cuda.synchronize()
        for (_, q, _), (_, qt, _) in zip(held, twins):
            assert torch.equal(q, qt), rnd
    batch.close()


def test_batch_error_word_stays_with_its_member(torch, bub):
    P = bub.PREC_FP64
    bad = W.c1(n=64, length=64 * 2.5e-4, nb=3)
    good = W.c1()
    batch = bub.Batch(P, max_cases=4)
    _, (cb, qb, _) = _join(torch, bub, batch, bad, False, P)
    _, (cg, qg, _) = _join(torch, bub, batch, good, False, P)
    qb[2, 17] = float("nan")            # energy of cell 17
    batch.step(2)
    err = torch.zeros((2, 3), dtype=torch.int64, device="cuda")
    cb.error_copy(err[0])
    cg.error_copy(err[1])
    e = err.cpu().tolist()
    assert e[0][0] == -4 and e[0][1] == 17
    assert e[1] == [0, -1, -1]
    assert torch.equal(qg, _alone(torch, bub, good, False, P, 2))
    batch.close()


def _moment_errors(orc, pb, got, ref):
    mg, mr = orc.moments(pb, got), orc.moments(pb, ref)
    return {"p": rel_err(mg[6], mr[6]), "alpha": rel_err(mg[1], mr[1])}


@pytest.mark.parametrize("use_run", [True, False])
def test_server_results_equal_alone_and_match_oracle(torch, bub, orc, use_run):
    from paper_2511_21031_amd.serve import Server, footprint_bytes
    reqs = W.c5_stream(count=24, seed=7, scale=0.05)
    cases = {r.rid: W.request_case(r) for r in reqs}
    fps = [footprint_bytes(c) for c in cases.values()]
    budget = 3 * max(fps)
    srv = Server(budget, max_slots=6, precision=bub.PREC_MIXED, bubble_mode=bub.BUBBLES_SPLIT, chunk=4,
                 keep_results=True, use_run=use_run)
    recs = srv.run(reqs, lambda r: cases[r.rid], time_scale=0.0)
    print(f"peak resident {srv.peak_active} problems, {srv.peak_used} of {budget} B; {len(srv.chunks)} step calls")
    assert srv.peak_used <= budget and srv.peak_active >= 2 and srv.used == 0
    assert len(srv.chunks) < sum(r.steps for r in reqs)      # step calls were shared
    for r, rec in zip(reqs, recs):
        assert rec.error == 0, (r.rid, rec.error, rec.error_cell, rec.error_bin)
        ref = _alone(torch, bub, cases[r.rid], True, bub.PREC_MIXED, r.steps).cpu().numpy()
        assert np.array_equal(rec.result, ref), r.rid
    # Served results against the FP64 oracle run on its own: each side takes its own CFL step and
    # its own adaptive bubble sub-steps, so where an accept/reject decision falls the other way the
    # two differ by up to the sub-step tolerance; the bar here is that bound (10 * rtol).  The
    # mixed-precision error proper (same steps on both sides, 1e-5) is tested in test_gpu_mixed.
    checked, worst = 0, 0.0
    for r, rec in zip(reqs, recs):
        case = cases[r.rid]
        if case.ncells * case.nb > 4000:
            continue
        pb = orc.problem_from_case(case, split=1)
        q = orc.init_state(pb, case.prim)
        for _ in range(r.steps):
            orc.rk3_step(pb, q, orc.cfl_dt(pb, q))
        e = _moment_errors(orc, pb, rec.result, q)
        worst = max(worst, *e.values())
        assert max(e.values()) < TOL_SPLIT, (r.rid, e)
        checked += 1
    print(f"requests checked against the oracle: {checked}, worst p/alpha error {worst:.2e}")
    assert checked >= 3


def test_batch_mixes_bubble_contents(torch, bub):
    """Members with polytropic contents and with gas and vapour contents (heat and vapour transfer, four
    fields per bin), unsplit and split, in one batch run: each ends bitwise equal to its problem stepped
    alone."""
    import dataclasses
    gas = dict(W.AIR, pv=W.PV_WATER_20C)
    tr = dict(W.AIR_VAPOUR)
    mem = [("c1", W.c1(), False),
           ("2d_transfer", dataclasses.replace(W.random_smooth(2, (70, 37), 1e-4, 5, seed=43), gas=gas, contents=tr),
            False),
           ("1d_transfer_split", dataclasses.replace(W.c1(n=64, length=64 * 2.5e-4, nb=5, amp_atm=3.0), gas=gas,
                                                    contents=tr), True)]
    batch = bub.Batch(bub.PREC_FP64, max_cases=4)
    held = {}
    for name, case, split in mem:
        ctx, q, work = _fresh(torch, bub, case, split, bub.PREC_FP64)
        batch.add(ctx, q, work, steps=4)
        held[name] = (ctx, q, work)
    while batch.run(10):
        pass
    torch.cuda.synchronize()
    for name, case, split in mem:
        ctx, q, _ = held[name]
        assert ctx.last_error()[0] == 0, name
        assert torch.equal(q, _alone(torch, bub, case, split, bub.PREC_FP64, 4)), name
