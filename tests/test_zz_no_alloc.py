"""The allocation-free right-hand side (bub_rhs_stage_noalloc) against bub_rhs_stage on a context.

Both run the same kernels, so the results must be bitwise equal; two calls in a row, the second on a
smaller problem of another dimensionality, check that the static scratch is rebound and its leftovers
do not leak into the next call.  Everything goes through the C ABI.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.parity import perturb_bins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def B(torch):
    import paper_2511_21031_amd._binding as B
    B.lib()
    return B


def _structs(B, case, precision=0, bubble_mode=0):
    g = B._Grid()
    g.ndim = case.ndim
    for d in range(3):
        g.n[d] = int(case.n[d])
        g.dx[d] = float(case.dx[d]) if d < case.ndim else 1.0
        g.bc[d][0], g.bc[d][1] = int(case.bc[d][0]), int(case.bc[d][1])
    lq = B._Liquid(case.liquid["gamma"], case.liquid["pi_inf"], case.liquid["rho0"], case.liquid["p0"])
    gs = B._Gas(case.gas["kappa"], case.gas["sigma"], case.gas["mu"], case.gas["pv"])
    bn = B._Bins(case.nb, case.r0_median, case.sigma_ln)
    op = B._Opts(case.cfl, precision, bubble_mode, 1e-4, 10000)
    return g, lq, gs, bn, op


def _noalloc(torch, B, case, q, precision=0, bubble_mode=0):
    L = B.lib()
    L.bub_rhs_stage_noalloc.argtypes = [ctypes.c_void_p] * 9
    L.bub_rhs_stage_noalloc.restype = ctypes.c_int
    g, lq, gs, bn, op = _structs(B, case, precision, bubble_mode)
    rhs = torch.full_like(q, float("nan"))
    err = torch.full((3,), 7, dtype=torch.int64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.bub_rhs_stage_noalloc(ctypes.byref(g), ctypes.byref(lq), ctypes.byref(gs), ctypes.byref(bn),
                                 ctypes.byref(op), ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(rhs.data_ptr()),
                                 ctypes.c_void_p(err.data_ptr()), stream)
    return rc, rhs, err


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_rhs_equals_context_rhs_twice(torch, B, orc, precision):
    cases = [W.random_smooth(2, (70, 37), 1e-4, 5, seed=41),          # first call
             W.random_smooth(1, (53,), 1e-4, 3, seed=42, bc=1)]       # second call: smaller, 1D, reflective
    for case in cases:
        pb = orc.problem_from_case(case)
        q = torch.from_numpy(perturb_bins(orc.init_state(pb, case.prim), case.ndim, case.nb, seed=3)).cuda()
        ctx = B.context_from_case(case, precision=precision)
        ref = ctx.rhs_stage(q)
        rc, got, err = _noalloc(torch, B, case, q, precision)
        assert rc == 0
        torch.cuda.synchronize()
        assert torch.equal(got, ref), case.n
        assert err.tolist() == [0, -1, -1]


def test_noalloc_reports_the_error_word_and_rejects_oversized_grids(torch, B, orc):
    case = W.random_smooth(2, (40, 24), 1e-4, 3, seed=43)
    pb = orc.problem_from_case(case)
    qh = orc.init_state(pb, case.prim)
    qh[5 + 1, 77] = -qh[5 + 1, 77]                  # nR of bin 1 at cell 77 (2D slots: rho, mu, mv, E, alpha, nR..)
    q = torch.from_numpy(qh).cuda()
    rc, _, err = _noalloc(torch, B, case, q)
    assert rc == 0
    assert err.tolist() == [-5, 77, 1]
    # a clean call afterwards starts from a cleared error word
    rc, _, err = _noalloc(torch, B, case, torch.from_numpy(orc.init_state(pb, case.prim)).cuda())
    assert rc == 0 and err.tolist() == [0, -1, -1]
    # 724^2 cells need 11520 + 64 * 524176 bytes > 32 MiB: refused before anything is launched
    big = W.uniform(2, (724, 724), 1e-4, 3)
    qb = torch.empty((2 + 3 + 6, 1), dtype=torch.float64, device="cuda")
    rc, _, _ = _noalloc(torch, B, big, qb)
    assert rc == -2
