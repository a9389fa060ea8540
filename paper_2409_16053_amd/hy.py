"""Thin ctypes binding of the C ABI in ``include/hy.h`` (``libhy.so``).

Argument marshalling only: every step of the hydro update runs in the gfx950
kernels of the library. PyTorch provides device memory (each problem's
workspace is a ``torch.uint8`` CUDA tensor owned here) and streams. There is
no CPU fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhy.so")

HY_OK, HY_ERR_ARG, HY_ERR_NOMEM, HY_ERR_HIP, HY_ERR_STATE, HY_ERR_BUDGET = range(6)
PERIODIC, OUTFLOW = 0, 1
PLM, PPM4, WENOZ, PPMX = 0, 1, 2, 3
FP64, MIXED = 0, 1
MAX_REFINE_BOXES = 8  # HY_MAX_REFINE_BOXES of include/hy.h
HOST, DEVICE, HOST_PINNED = 0, 1, 2

# (name, argtypes, restype) of every entry point declared in include/hy.h
_c = ctypes
_vp = _c.c_void_p
_dp = _c.POINTER(_c.c_double)


class HyConfig(_c.Structure):
    _fields_ = [
        ("n", _c.c_int32 * 3),
        ("block", _c.c_int32 * 3),
        ("lo", _c.c_double * 3),
        ("hi", _c.c_double * 3),
        ("bc", (_c.c_int32 * 2) * 3),
        ("gamma", _c.c_double),
        ("cfl", _c.c_double),
        ("recon", _c.c_int32),
        ("precision", _c.c_int32),
        ("fofc", _c.c_int32),
        ("rk", _c.c_int32),
        ("rho_floor", _c.c_double),
        ("p_floor", _c.c_double),
        ("nrefine", _c.c_int32),
        ("refine", ((_c.c_int32 * 3) * 2) * MAX_REFINE_BOXES),
    ]


_CP = _c.POINTER(HyConfig)
_i32p = _c.POINTER(_c.c_int32)
_i64p = _c.POINTER(_c.c_int64)

SIGNATURES = {
    "hy_workspace_bytes": ([_CP], _c.c_size_t),
    "hy_leaves": ([_CP, _i32p], _c.c_int32),
    "hy_create": ([_CP, _vp, _c.c_size_t, _c.POINTER(_vp)], _c.c_int),
    "hy_set_state": ([_vp, _vp, _c.c_int, _vp], _c.c_int),
    "hy_get_state": ([_vp, _vp, _c.c_int, _vp], _c.c_int),
    "hy_advance": ([_vp, _c.c_int32, _vp], _c.c_int),
    "hy_batch_advance": ([_c.POINTER(_vp), _i32p, _c.c_int32, _vp], _c.c_int),
    "hy_batch_advance_graph": ([_c.POINTER(_vp), _i32p, _c.c_int32, _vp], _c.c_int),
    "hy_query": ([_vp, _dp, _dp, _i64p, _i64p, _i64p], _c.c_int),
    "hy_set_time": ([_vp, _c.c_double], _c.c_int),
    "hy_destroy": ([_vp], _c.c_int),
    "hy_last_error": ([], _c.c_char_p),
    "hy_num_variants": ([], _c.c_int32),
    "hy_variant_info": ([_c.c_int32, _i32p, _i32p, _i32p], _c.c_int),
    "hy_set_launch": ([_vp, _c.c_int32, _c.c_int32], _c.c_int),
    "hy_get_launch": ([_vp, _i32p, _i32p], _c.c_int),
    "hy_autotune": ([_vp, _vp, _c.c_int32, _i32p, _i32p, _dp], _c.c_int),
    "hy_copy_probe": ([_vp, _vp, _c.c_size_t, _vp], _c.c_int),
    "hy_advance_timed": ([_vp, _c.c_int32, _vp, _dp, _dp], _c.c_int),
    "hy_advance_noalloc": ([_CP, _vp, _c.c_int32, _c.c_double, _vp, _vp], _c.c_int),
}

_lib = None


class HydroError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hy status {status}: {msg}")
        self.status = status


def lib():
    """Load libhy.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2409_16053_amd.build` (or __graft_entry__.build())")
        L = _c.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return lib().hy_last_error().decode()


def _check(st):
    if st != HY_OK:
        raise HydroError(st, last_error())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the hydro library needs a ROCm GPU; none is visible")
    return torch


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


def _enter(stream, *tensors):
    """Before the library works on ``stream`` with tensors produced on torch's
    current stream: order ``stream`` after that work and tell the caching
    allocator that the tensors are in use there."""
    torch = _torch()
    if stream is None:
        return
    cur = torch.cuda.current_stream()
    if stream != cur:
        stream.wait_stream(cur)
        for t in tensors:
            t.record_stream(stream)


def _leave(stream):
    """After enqueuing work on ``stream`` whose results torch's current stream
    will read: order the current stream after it."""
    torch = _torch()
    if stream is not None and stream != torch.cuda.current_stream():
        torch.cuda.current_stream().wait_stream(stream)


def make_config(pb) -> HyConfig:
    """HyConfig from a ``problems.Problem``."""
    c = HyConfig()
    block = pb.block if pb.block is not None else pb.n
    for d in range(3):
        c.n[d] = int(pb.n[d])
        c.block[d] = int(block[d])
        c.lo[d] = float(pb.lo[d])
        c.hi[d] = float(pb.hi[d])
        c.bc[d][0] = int(pb.bc[d][0])
        c.bc[d][1] = int(pb.bc[d][1])
    c.gamma = float(pb.gamma)
    c.cfl = float(pb.cfl)
    c.recon = int(pb.recon)
    c.precision = int(pb.precision)
    c.fofc = int(getattr(pb, "fofc", 0))
    c.rk = int(getattr(pb, "rk", 2))
    c.rho_floor = float(pb.rho_floor)
    c.p_floor = float(pb.p_floor)
    from .problems import refine_boxes
    boxes = refine_boxes(getattr(pb, "refine", None))
    if len(boxes) > MAX_REFINE_BOXES:
        raise HydroError(HY_ERR_ARG, f"at most {MAX_REFINE_BOXES} refined boxes")
    c.nrefine = len(boxes)
    for b, (lo, hi) in enumerate(boxes):
        for d in range(3):
            c.refine[b][0][d] = int(lo[d])
            c.refine[b][1][d] = int(hi[d])
    return c


def leaves(pb) -> np.ndarray:
    """Leaf blocks of the problem's mesh as int32 [leaf][level, x, y, z]
    (the order of a refined problem's leaf-major state)."""
    c = make_config(pb)
    n = lib().hy_leaves(_c.byref(c), None)
    if n < 0:
        raise HydroError(HY_ERR_ARG, last_error())
    out = np.zeros((n, 4), dtype=np.int32)
    lib().hy_leaves(_c.byref(c), out.ctypes.data_as(_i32p))
    return out


def workspace_bytes(pb) -> int:
    c = make_config(pb)
    n = lib().hy_workspace_bytes(_c.byref(c))
    if n == 0:
        raise HydroError(HY_ERR_ARG, last_error())
    return int(n)


def variants_full():
    """Compiled stage-kernel variants as (tx, ty, waves per SIMD)."""
    out = []
    for v in range(lib().hy_num_variants()):
        tx, ty, w = _c.c_int32(), _c.c_int32(), _c.c_int32()
        _check(lib().hy_variant_info(v, _c.byref(tx), _c.byref(ty), _c.byref(w)))
        out.append((tx.value, ty.value, w.value))
    return out


def variants():
    """Tile shapes (tx, ty) of the compiled stage-kernel variants."""
    return [(a, b) for a, b, _ in variants_full()]


class Problem:
    """One hydro problem resident on the GPU (state, counters, launch shape)."""

    def __init__(self, pb, device=None):
        torch = _torch()
        self.pb = pb
        self.cfg = make_config(pb)
        self.nbytes = workspace_bytes(pb)
        dev = torch.device("cuda" if device is None else device)
        # 256-byte aligned workspace carved from a torch allocation
        self._buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=dev)
        base = self._buf.data_ptr()
        self._off = (-base) % 256
        self.ws_ptr = base + self._off
        self.device = dev
        h = _vp()
        with torch.cuda.device(dev):
            _check(lib().hy_create(_c.byref(self.cfg), _vp(self.ws_ptr), self.nbytes, _c.byref(h)))
        self.h = h
        if getattr(pb, "refine", None) is not None:  # leaf-major state
            bx, by, bz = (int(b) for b in pb.block)
            self.shape = (len(leaves(pb)), 5, bz, by, bx)
        else:
            self.shape = (5, int(pb.n[2]), int(pb.n[1]), int(pb.n[0]))

    # -- state ---------------------------------------------------------
    def set_state(self, U=None, stream=None):
        """Load a state from a numpy array (pageable host) or a CUDA tensor."""
        torch = _torch()
        U = self.pb.U if U is None else U
        if isinstance(U, torch.Tensor) and U.is_cuda:
            t = U.to(torch.float64).contiguous()
            assert tuple(t.shape) == self.shape
            _enter(stream, t)
            _check(lib().hy_set_state(self.h, _vp(t.data_ptr()), DEVICE, _stream(stream)))
            self._keep = t
        else:
            a = np.ascontiguousarray(U, dtype=np.float64)
            assert a.shape == self.shape
            _check(lib().hy_set_state(self.h, _vp(a.ctypes.data), HOST, _stream(stream)))
        return self

    def set_state_pinned(self, t, stream=None):
        """Enqueue a load from a page-locked float64 CPU tensor; the caller keeps
        ``t`` alive and unchanged until the stream has passed this point."""
        assert t.is_pinned() and t.dtype == _torch().float64 and tuple(t.shape) == self.shape
        _check(lib().hy_set_state(self.h, _vp(t.data_ptr()), HOST_PINNED, _stream(stream)))
        return self

    def get_state(self, device=False, stream=None):
        torch = _torch()
        if device:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
            _enter(stream, out)
            _check(lib().hy_get_state(self.h, _vp(out.data_ptr()), DEVICE, _stream(stream)))
            _leave(stream)
            return out
        out = np.empty(self.shape, dtype=np.float64)
        _check(lib().hy_get_state(self.h, _vp(out.ctypes.data), HOST, _stream(stream)))
        return out

    def get_state_pinned(self, out, stream=None):
        """Enqueue a store into a page-locked float64 CPU tensor (check the
        bad-state flag later with ``query``)."""
        assert out.is_pinned() and out.dtype == _torch().float64 and tuple(out.shape) == self.shape
        _check(lib().hy_get_state(self.h, _vp(out.data_ptr()), HOST_PINNED, _stream(stream)))
        return out

    def get_state_status(self, stream=None):
        """(status, U) without raising on a device-flagged bad state."""
        out = np.empty(self.shape, dtype=np.float64)
        st = lib().hy_get_state(self.h, _vp(out.ctypes.data), HOST, _stream(stream))
        return st, out

    # -- time stepping ---------------------------------------------------
    def advance(self, nsteps, stream=None):
        _check(lib().hy_advance(self.h, int(nsteps), _stream(stream)))
        return self

    def advance_timed(self, nsteps, stream=None):
        a, b = _c.c_double(), _c.c_double()
        _check(lib().hy_advance_timed(self.h, int(nsteps), _stream(stream), _c.byref(a), _c.byref(b)))
        return a.value, b.value

    def query(self, raise_on_state=True):
        t, dt = _c.c_double(), _c.c_double()
        steps, fh, fc = _c.c_int64(), _c.c_int64(), _c.c_int64()
        st = lib().hy_query(self.h, _c.byref(t), _c.byref(dt), _c.byref(steps), _c.byref(fh),
                            _c.byref(fc))
        if st != HY_OK and (raise_on_state or st != HY_ERR_STATE):
            _check(st)
        return dict(t=t.value, dt=dt.value, steps=steps.value, floor_hits=fh.value,
                    fofc_cells=fc.value, status=st)

    def set_time(self, t):
        _check(lib().hy_set_time(self.h, float(t)))

    # -- launch shape ------------------------------------------------------
    def set_launch(self, variant, kc):
        _check(lib().hy_set_launch(self.h, int(variant), int(kc)))

    def get_launch(self):
        v, k = _c.c_int32(), _c.c_int32()
        _check(lib().hy_get_launch(self.h, _c.byref(v), _c.byref(k)))
        return v.value, k.value

    def autotune(self, full_steps=0, stream=None):
        """Pick the fastest compiled variant and z-chunk (see hy_autotune).
        full_steps > 0 times whole RK steps and advances the state."""
        v, k, us = _c.c_int32(), _c.c_int32(), _c.c_double()
        _check(lib().hy_autotune(self.h, _stream(stream), int(full_steps), _c.byref(v), _c.byref(k),
                                 _c.byref(us)))
        return v.value, k.value, us.value

    def autotune_steps(self, full_steps=2):
        """Tune on whole RK steps using a scratch copy of this problem, then
        apply the choice here (this problem's state is left unchanged)."""
        scratch = Problem(self.pb, device=self.device)
        scratch.set_state(self.get_state(device=True))
        res = scratch.autotune(full_steps=full_steps)
        scratch.close()
        self.set_launch(res[0], res[1])
        return res

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().hy_destroy(self.h)
            self.h = _vp()
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_advance(problems, nsteps, stream=None):
    """Advance several problems together (one launch per stage and kernel)."""
    n = len(problems)
    hs = (_vp * n)(*[p.h for p in problems])
    if np.isscalar(nsteps):
        nsteps = [int(nsteps)] * n
    ns = (_c.c_int32 * n)(*[int(x) for x in nsteps])
    _check(lib().hy_batch_advance(hs, ns, n, _stream(stream)))


def batch_advance_graph(problems, nsteps, stream):
    """Like ``batch_advance`` but captured once into a HIP graph and replayed
    (``stream`` must be a non-default torch.cuda.Stream)."""
    n = len(problems)
    hs = (_vp * n)(*[p.h for p in problems])
    if np.isscalar(nsteps):
        nsteps = [int(nsteps)] * n
    ns = (_c.c_int32 * n)(*[int(x) for x in nsteps])
    _check(lib().hy_batch_advance_graph(hs, ns, n, _stream(stream)))


def copy_probe(dst, src, nbytes=None, stream=None):
    """Plain device-to-device streaming copy with the library's probe kernel."""
    nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
    _check(lib().hy_copy_probe(_vp(dst.data_ptr()), _vp(src.data_ptr()), int(nbytes), _stream(stream)))


NOALLOC_MAX_BYTES = 256 << 20  # HY_NOALLOC_MAX_BYTES of include/hy.h


def advance_noalloc(pb, U, nsteps, t0=0.0, out=None, stream=None):
    """hy_advance_noalloc: advance the device state ``U`` (a contiguous
    float64 CUDA tensor of shape (5, nz, ny, nx)) in place by ``nsteps`` steps
    of problem ``pb`` without any device allocation; ``out`` (a float64 CUDA
    tensor of 3, or None) receives (t, dt_next, error flag)."""
    torch = _torch()
    c = make_config(pb)
    if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.float64
            and U.is_contiguous() and U.numel() == 5 * int(np.prod(pb.n))):
        raise ValueError("U must be a contiguous float64 CUDA tensor of 5 * cells elements")
    if out is not None and not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= 3):
        raise ValueError("out must be a float64 CUDA tensor of at least 3 elements")
    optr = _vp(out.data_ptr()) if out is not None else None
    _enter(stream, U, *([out] if out is not None else []))
    _check(lib().hy_advance_noalloc(_c.byref(c), _vp(U.data_ptr()), int(nsteps), float(t0), optr,
                                    _stream(stream)))
    _leave(stream)
