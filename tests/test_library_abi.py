"""The C-ABI library loads and exports every entry point include/bubbly.h declares.

Runs without a GPU: only symbol lookup and argument checks that return before
any device call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bubbly.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bub_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    pkg = pytest.importorskip("paper_2511_21031_amd")
    return pkg.lib()


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ("bub_ctx_create", "bub_init_state", "bub_rhs_stage", "bub_rk3_step", "bub_moments",
                     "bub_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_strerror(L):
    assert L.bub_strerror(0) == b"ok"
    assert L.bub_strerror(-1) == b"invalid argument"


def test_invalid_arguments_rejected_before_device_use(L):
    from paper_2511_21031_amd import _binding as B
    g = B._Grid()
    g.ndim = 4
    lq = B._Liquid(7.1, 3.06e8, 1000.0, 101325.0)
    gs = B._Gas(1.4, 0.0728, 1e-3, 0.0)
    bn = B._Bins(11, 10e-6, 0.3)
    op = B._Opts(0.3, 0, 0, 1e-4, 10000)
    h = ctypes.c_void_p()
    args = (ctypes.byref(g), ctypes.byref(lq), ctypes.byref(gs), ctypes.byref(bn), ctypes.byref(op), ctypes.byref(h))
    assert L.bub_ctx_create(*args) == -1
    g.ndim = 1
    g.n[0], g.n[1], g.n[2] = 100, 1, 1
    g.dx[0] = 1e-4
    g.bc[0][0], g.bc[0][1] = 1, 0          # mixed periodic/reflective is invalid
    assert L.bub_ctx_create(*args) == -1
    g.bc[0][1] = 1
    bn.nb = 10                              # even bin count is invalid
    assert L.bub_ctx_create(*args) == -1
    bn.nb = 11
    op.cfl = 0.0
    assert L.bub_ctx_create(*args) == -1
    assert L.bub_ctx_create(None, None, None, None, None, None) == -1
    assert L.bub_rk3_step(None, None, None, 0.0, None, None) == -1
    assert L.bub_layout(None, None, None, None, None, None) == -1
    assert L.bub_lagrangian_step(None, None, None, 0, None, None, 0.0, None, None, None) == -1
    assert L.bub_lagrangian_steps(None, None, None, 0, None, None, 3, 0.0, None, None, None) == -1


def test_ctx_buffer_bytes_host_only(L):
    """The device footprint of a context is computed on the host: bin table (six fields of up to 63
    bins), scalars (with the partial wave-speed maxima, 8 KiB) and the primitive scratch of ndim + 6
    fields, each part 256-byte aligned."""
    from paper_2511_21031_amd import _binding as B
    g = B._Grid()
    bn = B._Bins(21, 10e-6, 0.3)
    out = ctypes.c_size_t()
    g.ndim = 2
    g.n[0], g.n[1], g.n[2] = 70, 37, 1
    assert L.bub_ctx_buffer_bytes(ctypes.byref(g), ctypes.byref(bn), ctypes.byref(out)) == 0
    n = 70 * 37
    scratch = 8 * (2 + 6) * n
    assert scratch <= out.value <= scratch + 8 * 6 * 63 + 8192 + 512 + 3 * 256
    assert out.value % 256 == 0
    assert B.ctx_buffer_bytes(2, (70, 37, 1), 21) == out.value
    g.n[1] = 0
    assert L.bub_ctx_buffer_bytes(ctypes.byref(g), ctypes.byref(bn), ctypes.byref(out)) == -1
    g.n[1] = 37
    g.ndim = 0
    assert L.bub_ctx_buffer_bytes(ctypes.byref(g), ctypes.byref(bn), ctypes.byref(out)) == -1
    assert L.bub_ctx_buffer_bytes(None, ctypes.byref(bn), ctypes.byref(out)) == -1


def test_serving_footprint_counts_three_states_the_context_and_the_primitives(L):
    import workloads as W
    from paper_2511_21031_amd import ctx_buffer_bytes
    from paper_2511_21031_amd.serve import footprint_bytes
    case = W.request_case(W.c5_stream(count=1, seed=3)[0])
    fp = footprint_bytes(case)
    state = 8 * case.nvar * case.ncells
    prim = 8 * (case.ndim + 3) * case.ncells      # the initial primitives, alive until the problem retires
    ctxb = ctx_buffer_bytes(case.ndim, case.n, case.nb)
    assert 3 * state + prim + ctxb <= fp <= 3 * state + prim + ctxb + 256


def test_context_buffer_holds_a_second_primitive_scratch_from_2_19_cells(L):
    from paper_2511_21031_amd import ctx_buffer_bytes
    small, big = ctx_buffer_bytes(2, (724, 724, 1), 5), ctx_buffer_bytes(2, (725, 725, 1), 5)
    p_small, p_big = 8 * 8 * 724 * 724, 8 * 8 * 725 * 725          # (ndim + 6) fields
    assert p_small < small < p_small + 16384                          # 524176 cells: one scratch
    assert 2 * p_big < big < 2 * p_big + 16384                        # 525625 cells: two
