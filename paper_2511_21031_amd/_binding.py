"""ctypes binding of libbubbly.so: same entry points as include/bubbly.h, torch tensors in."""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime that libbubbly.so then binds to (same soname)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libbubbly.so")

BC_PERIODIC, BC_REFLECTIVE = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
BUBBLES_UNSPLIT, BUBBLES_SPLIT = 0, 1
CONTENTS_POLYTROPIC, CONTENTS_TRANSFER = 0, 1


class BubblyError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = _lib.bub_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} (code {code})")


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
                ("bc", (ctypes.c_int * 2) * 3)]


class _Liquid(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("pi_inf", ctypes.c_double), ("rho0", ctypes.c_double),
                ("p0", ctypes.c_double)]


class _Gas(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("sigma", ctypes.c_double), ("mu", ctypes.c_double),
                ("pv", ctypes.c_double)]


class _Bins(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("r0_median", ctypes.c_double), ("sigma_ln", ctypes.c_double)]


class _Transfer(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("gam_b", "Rg", "Rv", "T0", "k_b", "D_v", "beta_T", "beta_c")]


class _Opts(ctypes.Structure):
    _fields_ = [("cfl", ctypes.c_double), ("precision", ctypes.c_int), ("bubble_mode", ctypes.c_int),
                ("sub_rtol", ctypes.c_double), ("max_substeps", ctypes.c_int), ("viscous", ctypes.c_int),
                ("contents", ctypes.c_int), ("transfer", _Transfer)]


class _Source(ctypes.Structure):
    _fields_ = [("dir", ctypes.c_int), ("sign", ctypes.c_int), ("x", ctypes.c_double), ("width", ctypes.c_double),
                ("amp", ctypes.c_double), ("freq", ctypes.c_double), ("t0", ctypes.c_double),
                ("ncycles", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)

# entry point -> argtypes (all return int unless noted)
_SIGS = {
    "bub_ctx_create": [ctypes.POINTER(_Grid), ctypes.POINTER(_Liquid), ctypes.POINTER(_Gas),
                       ctypes.POINTER(_Bins), ctypes.POINTER(_Opts), ctypes.POINTER(_vp)],
    "bub_ctx_destroy": [_vp],
    "bub_ctx_buffer_bytes": [ctypes.POINTER(_Grid), ctypes.POINTER(_Bins), ctypes.POINTER(ctypes.c_size_t)],
    "bub_ctx_create_on": [ctypes.POINTER(_Grid), ctypes.POINTER(_Liquid), ctypes.POINTER(_Gas),
                          ctypes.POINTER(_Bins), ctypes.POINTER(_Opts), _vp, ctypes.c_size_t, _vp,
                          ctypes.POINTER(_vp)],
    "bub_layout": [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64),
                   ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
    "bub_bins_get": [_vp, _dp, _dp],
    "bub_init_state": [_vp, _vp, _vp, _vp],
    "bub_rhs_stage": [_vp, _vp, _vp, _vp],
    "bub_rk3_step": [_vp, _vp, _vp, ctypes.c_double, _vp, _vp],
    "bub_set_source": [_vp, ctypes.POINTER(_Source)],
    "bub_set_time": [_vp, ctypes.c_double, _vp],
    "bub_get_time": [_vp, ctypes.POINTER(ctypes.c_double)],
    "bub_rk3_steps": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double, _vp, _vp],
    "bub_moments": [_vp, _vp, _vp, _vp],
    "bub_last_error": [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_int),
                       _vp],
    "bub_error_copy": [_vp, _vp, _vp],
    "bub_bubble_advance": [_vp, _vp, ctypes.c_double, _vp, _vp],
    "bub_lagrangian_layout": [_vp, _i64, ctypes.POINTER(ctypes.c_size_t)],
    "bub_lagrangian_bubbles": [_vp, _vp, _vp, _i64, _vp],
    "bub_lagrangian_init": [_vp, _vp, _vp, _vp],
    "bub_lagrangian_smear": [_vp, _vp, _i64, _vp, _vp],
    "bub_lagrangian_gather": [_vp, _vp, _vp, _i64, _vp, _vp],
    "bub_lagrangian_rhs": [_vp, _vp, _vp, _vp, _vp],
    "bub_lagrangian_step": [_vp, _vp, _vp, _i64, _vp, _vp, ctypes.c_double, _vp, _vp, _vp],
    "bub_lagrangian_steps": [_vp, _vp, _vp, _i64, _vp, _vp, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp],
    "bub_tile_count": [_vp, ctypes.POINTER(ctypes.c_int)],
    "bub_tile_info": [_vp, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 4,
    "bub_tile_set": [_vp, ctypes.c_int],
    "bub_tile_get": [_vp, ctypes.POINTER(ctypes.c_int)],
    "bub_bin_groups": [_vp, ctypes.c_int],
    "bub_substep_counts": [_vp, _vp],
    "bub_autotune": [_vp, _vp, _vp, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int), _vp],
    "bub_autotune_cached": [_vp, ctypes.c_char_p, _vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_int), _vp],
    "bub_batch_tune_cache": [_vp, ctypes.c_char_p],
    "bub_batch_create": [ctypes.c_int, ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_vp)],
    "bub_batch_destroy": [_vp],
    "bub_batch_add": [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "bub_batch_run": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _vp],
    "bub_batch_poll": [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
    "bub_batch_remaining": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "bub_batch_remove": [_vp, ctypes.c_int],
    "bub_batch_step": [_vp, ctypes.c_int, _vp],
    "bub_batch_info": [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "bub_batch_autotune": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _vp],
    "bub_batch_lanes": [_vp, ctypes.c_int],
    "bub_batch_graphs": [_vp, ctypes.c_int],
    "bub_profile": [_vp, ctypes.c_int],
    "bub_profile_read": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)],
}

K_STAGE, K_PRIM, K_OTHER = 0, 1, 2


def library_path() -> str:
    return _SO


def lib():
    """Load libbubbly.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise ImportError(f"{_SO} is missing: build it with `python -m paper_2511_21031_amd.build`")
        L = ctypes.CDLL(_SO)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.bub_strerror.argtypes = [ctypes.c_int]
        L.bub_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise BubblyError(rc, what)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _ptr(t: torch.Tensor):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 tensor on the GPU")
    return _vp(t.data_ptr())


class Context:
    """One problem (grid, physics, bins, options) on the current device."""

    def __init__(self, ndim, n, dx, bc, nb, r0_median=10e-6, sigma_ln=0.3, liquid=None, gas=None, cfl=0.3,
                 precision=PREC_FP64, bubble_mode=BUBBLES_UNSPLIT, sub_rtol=1e-4, max_substeps=10000,
                 torch_buffer=False, stream=None, viscous=0, source=None, contents=None):
        """torch_buffer=True: the context's device memory is a torch tensor and it is initialised on
        `stream` (bub_ctx_create_on): no allocation call and no host synchronisation.  contents: None for
        polytropic gas, or dict(gam_b, Rg, Rv, T0, k_b, D_v, beta_T, beta_c) for gas and vapour with heat
        and vapour transfer (the vapour pressure is gas['pv'])."""
        L = lib()
        liquid = liquid or dict(gamma=7.1, pi_inf=3.06e8, rho0=1000.0, p0=101325.0)
        gas = gas or dict(kappa=1.4, sigma=0.0728, mu=1e-3, pv=0.0)
        g = _Grid()
        g.ndim = ndim
        for d in range(3):
            g.n[d] = int(n[d]) if d < len(n) else 1
            g.dx[d] = float(dx[d]) if d < len(dx) else 1.0
            b = bc[d] if d < len(bc) else (0, 0)
            g.bc[d][0], g.bc[d][1] = int(b[0]), int(b[1])
        lq = _Liquid(liquid["gamma"], liquid["pi_inf"], liquid["rho0"], liquid["p0"])
        gs = _Gas(gas["kappa"], gas["sigma"], gas["mu"], gas["pv"])
        bn = _Bins(nb, r0_median, sigma_ln)
        op = _Opts(cfl, precision, bubble_mode, sub_rtol, max_substeps, int(viscous))
        if contents:
            op.contents = CONTENTS_TRANSFER
            op.transfer = _Transfer(*(float(contents[k]) for k, _ in _Transfer._fields_))
        h = _vp()
        self._buf = None
        if torch_buffer:
            nbytes = ctypes.c_size_t()
            _check(L.bub_ctx_buffer_bytes(ctypes.byref(g), ctypes.byref(bn), ctypes.byref(nbytes)),
                   "bub_ctx_buffer_bytes")
            self._buf = torch.empty((nbytes.value + 256,), dtype=torch.uint8, device="cuda")
            addr = (self._buf.data_ptr() + 255) & ~255
            _check(L.bub_ctx_create_on(ctypes.byref(g), ctypes.byref(lq), ctypes.byref(gs), ctypes.byref(bn),
                                       ctypes.byref(op), _vp(addr), nbytes.value, _stream(stream), ctypes.byref(h)),
                   "bub_ctx_create_on")
        else:
            _check(L.bub_ctx_create(ctypes.byref(g), ctypes.byref(lq), ctypes.byref(gs), ctypes.byref(bn),
                                    ctypes.byref(op), ctypes.byref(h)), "bub_ctx_create")
        self._h = h
        self.ndim = ndim
        self.n = tuple(g.n)
        self.nb = nb
        self.precision = precision
        self.bubble_mode = bubble_mode
        nv, npr, nc = ctypes.c_int(), ctypes.c_int(), _i64()
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(L.bub_layout(h, ctypes.byref(nv), ctypes.byref(npr), ctypes.byref(nc), ctypes.byref(sb),
                            ctypes.byref(wb)), "bub_layout")
        self.nvar, self.nprim, self.ncells = nv.value, npr.value, nc.value
        self.state_bytes, self.work_bytes = sb.value, wb.value
        if source is not None:
            self.set_source(source)

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().bub_ctx_destroy(self._h)
            self._h = None
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers ----------------------------------------------------------------
    def new_state(self, device="cuda"):
        return torch.empty((self.nvar, self.ncells), dtype=torch.float64, device=device)

    def new_work(self, device="cuda"):
        return torch.empty((self.work_bytes // 8,), dtype=torch.float64, device=device)

    def bins(self):
        r0 = (ctypes.c_double * self.nb)()
        w = (ctypes.c_double * self.nb)()
        _check(lib().bub_bins_get(self._h, r0, w), "bub_bins_get")
        return list(r0), list(w)

    # -- entry points ---------------------------------------------------------------
    def init_state(self, prim: torch.Tensor, q: torch.Tensor | None = None, stream=None):
        if prim.shape != (self.ndim + 3, self.ncells):
            raise ValueError(f"prim must be [{self.ndim + 3}][{self.ncells}]")
        q = self.new_state(prim.device) if q is None else q
        _check(lib().bub_init_state(self._h, _ptr(prim), _ptr(q), _stream(stream)), "bub_init_state")
        return q

    def rhs_stage(self, q: torch.Tensor, rhs: torch.Tensor | None = None, stream=None):
        rhs = torch.empty_like(q) if rhs is None else rhs
        _check(lib().bub_rhs_stage(self._h, _ptr(q), _ptr(rhs), _stream(stream)), "bub_rhs_stage")
        return rhs

    def set_source(self, src: dict | None):
        """One-way planar acoustic source: dict(dir, sign, x, width, amp, freq, t0=0, ncyc=0), or None."""
        if src is None:
            _check(lib().bub_set_source(self._h, None), "bub_set_source")
            return
        so = _Source(int(src["dir"]), int(src["sign"]), float(src["x"]), float(src["width"]), float(src["amp"]),
                     float(src["freq"]), float(src.get("t0", 0.0)), float(src.get("ncyc", 0.0)))
        _check(lib().bub_set_source(self._h, ctypes.byref(so)), "bub_set_source")

    def set_time(self, t: float, stream=None):
        _check(lib().bub_set_time(self._h, float(t), _stream(stream)), "bub_set_time")

    def time(self) -> float:
        """The context's clock (waits for the device)."""
        v = ctypes.c_double()
        _check(lib().bub_get_time(self._h, ctypes.byref(v)), "bub_get_time")
        return v.value

    def rk3_step(self, q: torch.Tensor, work: torch.Tensor, dt: float = 0.0, dt_dev: torch.Tensor | None = None,
                 stream=None):
        if work.numel() * 8 < self.work_bytes:
            raise ValueError("work buffer too small")
        _check(lib().bub_rk3_step(self._h, _ptr(q), _ptr(work), float(dt), _ptr(dt_dev), _stream(stream)),
               "bub_rk3_step")

    def rk3_steps(self, q: torch.Tensor, work: torch.Tensor, nsteps: int, dt: float = 0.0,
                  dt_dev: torch.Tensor | None = None, stream=None):
        """nsteps RK3 steps in one call (bitwise nsteps calls of rk3_step)."""
        if work.numel() * 8 < self.work_bytes:
            raise ValueError("work buffer too small")
        _check(lib().bub_rk3_steps(self._h, _ptr(q), _ptr(work), int(nsteps), float(dt), _ptr(dt_dev),
                                   _stream(stream)), "bub_rk3_steps")

    def moments(self, q: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        out = torch.empty((8, self.ncells), dtype=torch.float64, device=q.device) if out is None else out
        _check(lib().bub_moments(self._h, _ptr(q), _ptr(out), _stream(stream)), "bub_moments")
        return out

    def bubble_advance(self, q: torch.Tensor, tau: float, nsub: torch.Tensor | None = None, stream=None):
        """Bubble half of the Strang splitting over tau, in place; nsub (int32 [nb][N]) gets sub-step counts."""
        if nsub is not None and (nsub.dtype != torch.int32 or not nsub.is_cuda or nsub.numel() != self.nb * self.ncells):
            raise ValueError("nsub must be an int32 GPU tensor of nb*N entries")
        _check(lib().bub_bubble_advance(self._h, _ptr(q), float(tau),
                                        None if nsub is None else _vp(nsub.data_ptr()), _stream(stream)),
               "bub_bubble_advance")

    def substep_counts(self, nsub: torch.Tensor | None):
        """Record the sub-step counts of both bubble half-steps of later split-mode steps in nsub
        (int32 [2][nb][N] on the GPU, kept alive by the caller), or stop recording (None)."""
        if nsub is not None and (nsub.dtype != torch.int32 or not nsub.is_cuda or not nsub.is_contiguous()
                                 or nsub.numel() != 2 * self.nb * self.ncells):
            raise ValueError("nsub must be a contiguous int32 GPU tensor of 2*nb*N entries")
        self._nsub = nsub
        _check(lib().bub_substep_counts(self._h, None if nsub is None else _vp(nsub.data_ptr())),
               "bub_substep_counts")

    # -- volume-averaged (Euler--Lagrange) variant ------------------------------
    def lagrangian_work(self, nbub: int, device="cuda"):
        wb = ctypes.c_size_t()
        _check(lib().bub_lagrangian_layout(self._h, int(nbub), ctypes.byref(wb)), "bub_lagrangian_layout")
        return torch.empty((wb.value // 8,), dtype=torch.float64, device=device)

    def lagrangian_bubbles(self, xyzr0: torch.Tensor, stream=None):
        """Bubble records [8][nbub] at rest at R0 from [4][nbub] = x, y, z, R0."""
        nb = xyzr0.shape[1]
        out = torch.empty((8, nb), dtype=torch.float64, device=xyzr0.device)
        _check(lib().bub_lagrangian_bubbles(self._h, _ptr(xyzr0), _ptr(out), nb, _stream(stream)),
               "bub_lagrangian_bubbles")
        return out

    def lagrangian_init(self, prim: torch.Tensor, stream=None):
        ql = torch.empty((5, self.ncells), dtype=torch.float64, device=prim.device)
        _check(lib().bub_lagrangian_init(self._h, _ptr(prim), _ptr(ql), _stream(stream)), "bub_lagrangian_init")
        return ql

    def lagrangian_smear(self, bubbles: torch.Tensor, alpha_D: torch.Tensor | None = None, stream=None):
        aD = torch.empty((2, self.ncells), dtype=torch.float64, device=bubbles.device) if alpha_D is None else alpha_D
        _check(lib().bub_lagrangian_smear(self._h, _ptr(bubbles), bubbles.shape[1], _ptr(aD), _stream(stream)),
               "bub_lagrangian_smear")
        return aD

    def lagrangian_gather(self, ql: torch.Tensor, bubbles: torch.Tensor, stream=None):
        out = torch.empty((3, bubbles.shape[1]), dtype=torch.float64, device=ql.device)
        _check(lib().bub_lagrangian_gather(self._h, _ptr(ql), _ptr(bubbles), bubbles.shape[1], _ptr(out),
                                           _stream(stream)), "bub_lagrangian_gather")
        return out

    def lagrangian_rhs(self, ql: torch.Tensor, alpha_D: torch.Tensor, stream=None):
        rhs = torch.empty_like(ql)
        _check(lib().bub_lagrangian_rhs(self._h, _ptr(ql), _ptr(alpha_D), _ptr(rhs), _stream(stream)),
               "bub_lagrangian_rhs")
        return rhs

    def lagrangian_step(self, ql, bubbles, alpha_D, work, dt=0.0, dt_dev=None, nsub=None, stream=None):
        _check(lib().bub_lagrangian_step(self._h, _ptr(ql), _ptr(bubbles), bubbles.shape[1], _ptr(alpha_D),
                                         _ptr(work), float(dt), _ptr(dt_dev),
                                         None if nsub is None else _vp(nsub.data_ptr()), _stream(stream)),
               "bub_lagrangian_step")

    def lagrangian_steps(self, ql, bubbles, alpha_D, work, nsteps, dt=0.0, dt_dev=None, nsub=None, stream=None):
        """nsteps Lagrangian steps in one call (only the last one's closing smear is made)."""
        _check(lib().bub_lagrangian_steps(self._h, _ptr(ql), _ptr(bubbles), bubbles.shape[1], _ptr(alpha_D),
                                          _ptr(work), int(nsteps), float(dt), _ptr(dt_dev),
                                          None if nsub is None else _vp(nsub.data_ptr()), _stream(stream)),
               "bub_lagrangian_steps")

    def tiles(self):
        """List of (tx, ty, tz, block) stage-kernel tile shapes for this dimensionality."""
        n = ctypes.c_int()
        _check(lib().bub_tile_count(self._h, ctypes.byref(n)), "bub_tile_count")
        out = []
        for i in range(n.value):
            v = [ctypes.c_int() for _ in range(4)]
            _check(lib().bub_tile_info(self._h, i, *[ctypes.byref(x) for x in v]), "bub_tile_info")
            out.append(tuple(x.value for x in v))
        return out

    @property
    def tile(self) -> int:
        v = ctypes.c_int()
        _check(lib().bub_tile_get(self._h, ctypes.byref(v)), "bub_tile_get")
        return v.value

    @tile.setter
    def tile(self, idx: int):
        _check(lib().bub_tile_set(self._h, int(idx)), "bub_tile_set")

    def set_bin_groups(self, groups: int):
        """Stage-kernel workgroups per tile (0: automatic)."""
        _check(lib().bub_bin_groups(self._h, int(groups)), "bub_bin_groups")

    def autotune(self, q: torch.Tensor, scratch: torch.Tensor | None = None, reps: int = 5, stream=None):
        """Time every tile shape on q, keep the fastest; returns (best index, ms per launch per shape)."""
        scratch = torch.empty_like(q) if scratch is None else scratch
        n = len(self.tiles())
        ms = (ctypes.c_double * n)()
        best = ctypes.c_int()
        _check(lib().bub_autotune(self._h, _ptr(q), _ptr(scratch), int(reps), ms, ctypes.byref(best),
                                  _stream(stream)), "bub_autotune")
        return best.value, list(ms)

    def autotune_cached(self, cache_path: str, q: torch.Tensor, scratch: torch.Tensor | None = None, reps: int = 5,
                        stream=None):
        """Tile shape from the cache file if it holds this context's key, else tuned and stored;
        returns (best index, whether the cache held it)."""
        scratch = torch.empty_like(q) if scratch is None else scratch
        best, hit = ctypes.c_int(), ctypes.c_int()
        _check(lib().bub_autotune_cached(self._h, str(cache_path).encode(), _ptr(q), _ptr(scratch), int(reps),
                                         ctypes.byref(best), ctypes.byref(hit), _stream(stream)),
               "bub_autotune_cached")
        return best.value, bool(hit.value)

    def profile(self, enable: bool):
        _check(lib().bub_profile(self._h, 1 if enable else 0), "bub_profile")

    def profile_read(self, kind: int):
        """(total milliseconds, launches) of one kernel kind since the last read."""
        ms, n = ctypes.c_double(), _i64()
        _check(lib().bub_profile_read(self._h, kind, ctypes.byref(ms), ctypes.byref(n)), "bub_profile_read")
        return ms.value, n.value

    def last_error(self, stream=None):
        code, cell, b = ctypes.c_int(), _i64(), ctypes.c_int()
        _check(lib().bub_last_error(self._h, ctypes.byref(code), ctypes.byref(cell), ctypes.byref(b),
                                    _stream(stream)), "bub_last_error")
        return code.value, cell.value, b.value

    def error_copy(self, dst: torch.Tensor, stream=None):
        """Enqueue a copy of the error word (code, cell, bin) into the int64 device tensor dst[3]."""
        if not dst.is_cuda or dst.dtype != torch.int64 or dst.numel() < 3 or not dst.is_contiguous():
            raise ValueError("dst must be a contiguous int64 GPU tensor of at least 3 elements")
        _check(lib().bub_error_copy(self._h, _vp(dst.data_ptr()), _stream(stream)), "bub_error_copy")


def ctx_buffer_bytes(ndim, n, nb) -> int:
    """Device bytes of a context's own buffers (bin table, scalars, primitive scratch)."""
    g = _Grid()
    g.ndim = ndim
    for d in range(3):
        g.n[d] = int(n[d]) if d < len(n) else 1
        g.dx[d] = 1.0
    bn = _Bins(nb, 1e-5, 0.3)
    nbytes = ctypes.c_size_t()
    _check(lib().bub_ctx_buffer_bytes(ctypes.byref(g), ctypes.byref(bn), ctypes.byref(nbytes)),
           "bub_ctx_buffer_bytes")
    return nbytes.value


class Batch:
    """Resident problems advanced together (bub_batch_*).  run(): a chunk of steps for the members that
    still have steps to take, completion read by poll(); step(): every member's steps.  Both step each
    member with its own kernels, overlapping over the batch's internal streams."""

    def __init__(self, precision=PREC_FP64, max_cases=64, hbm_budget=0):
        h = _vp()
        _check(lib().bub_batch_create(int(precision), int(max_cases), int(hbm_budget), ctypes.byref(h)),
               "bub_batch_create")
        self._h = h
        self.precision = precision
        self.max_cases = int(max_cases)
        self._members = {}     # slot -> (ctx, q, work): keeps buffers alive while resident

    def close(self):
        if getattr(self, "_h", None):
            lib().bub_batch_destroy(self._h)
            self._h = None
            self._members.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, ctx: Context, q: torch.Tensor, work: torch.Tensor, steps: int = 0) -> int:
        """Add a member needing `steps` steps from run() (0: open-ended); returns its slot."""
        if q.numel() * 8 < ctx.state_bytes or work.numel() * 8 < ctx.work_bytes:
            raise ValueError("state or work buffer too small")
        slot = ctypes.c_int()
        _check(lib().bub_batch_add(self._h, ctx._h, _ptr(q), _ptr(work), int(steps), ctypes.byref(slot)),
               "bub_batch_add")
        self._members[slot.value] = (ctx, q, work)
        return slot.value

    def run(self, max_steps: int, stream=None) -> int:
        """Grouped chunk of at most max_steps steps (never past the member with the fewest left);
        returns the steps taken."""
        n = ctypes.c_int()
        _check(lib().bub_batch_run(self._h, int(max_steps), ctypes.byref(n), _stream(stream)), "bub_batch_run")
        return n.value

    def poll(self):
        """Slots whose last step has completed on the device since the last poll (no synchronisation)."""
        buf = (ctypes.c_int * self.max_cases)()
        n = ctypes.c_int()
        _check(lib().bub_batch_poll(self._h, buf, ctypes.byref(n)), "bub_batch_poll")
        return [buf[i] for i in range(n.value)]

    def remaining(self, slot: int) -> int:
        v = ctypes.c_int()
        _check(lib().bub_batch_remaining(self._h, int(slot), ctypes.byref(v)), "bub_batch_remaining")
        return v.value

    def remove(self, slot: int):
        _check(lib().bub_batch_remove(self._h, int(slot)), "bub_batch_remove")
        self._members.pop(slot, None)

    def step(self, nsteps: int = 1, stream=None):
        _check(lib().bub_batch_step(self._h, int(nsteps), _stream(stream)), "bub_batch_step")

    def info(self):
        """(members, cells, cell-bins)."""
        n, c, cb = ctypes.c_int(), _i64(), _i64()
        _check(lib().bub_batch_info(self._h, ctypes.byref(n), ctypes.byref(c), ctypes.byref(cb)), "bub_batch_info")
        return n.value, c.value, cb.value

    def set_graphs(self, enable: bool):
        """Replay each member's step as a captured graph (default) or launch its kernels directly."""
        _check(lib().bub_batch_graphs(self._h, int(bool(enable))), "bub_batch_graphs")

    def set_lanes(self, lanes: int):
        """Internal streams the members are dealt over (1..16)."""
        _check(lib().bub_batch_lanes(self._h, int(lanes)), "bub_batch_lanes")

    def set_tune_cache(self, cache_path: str | None):
        """Tile-shape cache file of the class autotuner (None: none)."""
        _check(lib().bub_batch_tune_cache(self._h, str(cache_path).encode() if cache_path else None),
               "bub_batch_tune_cache")

    def autotune(self, reps: int = 3, stream=None) -> int:
        """Tune the stage tile shape of every new (ndim, nb) class; returns the number of tuned classes."""
        k = ctypes.c_int()
        _check(lib().bub_batch_autotune(self._h, int(reps), ctypes.byref(k), _stream(stream)), "bub_batch_autotune")
        return k.value


def context_from_case(case, **kw) -> Context:
    """Context for a ``workloads.Case`` (grid, bins, physics, contents and CFL of the case)."""
    kw.setdefault("contents", getattr(case, "contents", None))
    return Context(case.ndim, case.n, case.dx, case.bc, case.nb, case.r0_median, case.sigma_ln, case.liquid,
                   case.gas, case.cfl, **kw)
