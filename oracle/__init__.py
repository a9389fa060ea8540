"""Python access to the plain FP64 CPU reference solver in ``oracle/oracle.c``.

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the benchmark's
CPU-baseline leg use it. The product path (``paper_2409_16053_amd``) never
imports it, and the two share no code. This wrapper only marshals arguments;
all arithmetic is in the C file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_NOMEM, ERR_STATE = 0, 1, 2, 4


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc: FP64, -O2, no FP contraction, OpenMP."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC,
               "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("recon", ctypes.c_int32),
        ("fofc", ctypes.c_int32),
        ("rk", ctypes.c_int32),
        ("dx", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("rho_floor", ctypes.c_double),
        ("p_floor", ctypes.c_double),
    ]


MAX_BOXES = 8


class Smr(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32 * 3),
        ("nbox", ctypes.c_int32),
        ("box", ((ctypes.c_int32 * 3) * 2) * MAX_BOXES),
    ]


def _boxes(refine):
    """The refined boxes of ``Problem.refine``: one box ((lo), (hi)) or a
    sequence of them."""
    if refine is None:
        return []
    if len(refine) == 2 and all(np.isscalar(x) for x in refine[0]):
        return [refine]
    return list(refine)


def smr_params(pb) -> Smr:
    """ctypes refinement block (block size and refined boxes) of a problem."""
    S = Smr()
    boxes = _boxes(pb.refine)
    if len(boxes) > MAX_BOXES:
        raise ValueError(f"at most {MAX_BOXES} refined boxes")
    S.nbox = len(boxes)
    for d in range(3):
        S.block[d] = int(pb.block[d])
    for b, (lo, hi) in enumerate(boxes):
        for d in range(3):
            S.box[b][0][d] = int(lo[d])
            S.box[b][1][d] = int(hi[d])
    return S


def _bind(L):
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(Params)
    L.or_advance.argtypes = [pp, dp, ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_longlong),
                             ctypes.POINTER(ctypes.c_longlong)]
    L.or_advance.restype = ctypes.c_int
    L.or_new_dt.argtypes = [pp, dp]
    L.or_new_dt.restype = ctypes.c_double
    L.or_divergence.argtypes = [pp, dp, dp, ctypes.POINTER(ctypes.c_longlong)]
    L.or_divergence.restype = ctypes.c_int
    L.or_fill_ghosts.argtypes = [pp, dp, dp]
    L.or_fill_ghosts.restype = ctypes.c_int
    L.or_c2p.argtypes = [pp, dp, dp, ctypes.POINTER(ctypes.c_int)]
    L.or_c2p.restype = ctypes.c_int
    L.or_plm_cell.argtypes = [ctypes.c_double] * 3 + [dp, dp]
    L.or_plm_cell.restype = None
    L.or_ppm4_cell.argtypes = [dp, dp, dp]
    L.or_ppm4_cell.restype = None
    L.or_wenoz_cell.argtypes = [dp, dp, dp]
    L.or_wenoz_cell.restype = None
    L.or_ppmx_cell.argtypes = [dp, dp, dp]
    L.or_ppmx_cell.restype = None
    L.or_hllc.argtypes = [ctypes.c_double, dp, dp, dp]
    L.or_hllc.restype = None
    L.or_llf.argtypes = [ctypes.c_double, dp, dp, dp]
    L.or_llf.restype = None
    L.or_nghost.argtypes = [ctypes.c_int]
    L.or_nghost.restype = ctypes.c_int
    L.or_set_threads.argtypes = [ctypes.c_int]
    L.or_set_threads.restype = None
    L.or_get_threads.argtypes = []
    L.or_get_threads.restype = ctypes.c_int
    sp = ctypes.POINTER(Smr)
    L.or_smr_leaves.argtypes = [pp, sp, ctypes.POINTER(ctypes.c_int32)]
    L.or_smr_leaves.restype = ctypes.c_int
    L.or_smr_new_dt.argtypes = [pp, sp, dp]
    L.or_smr_new_dt.restype = ctypes.c_double
    L.or_smr_advance.argtypes = [pp, sp, dp, ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_longlong),
                                 ctypes.POINTER(ctypes.c_longlong)]
    L.or_smr_advance.restype = ctypes.c_int
    L.or_smr_fill_ghosts.argtypes = [pp, sp, dp, dp]
    L.or_smr_fill_ghosts.restype = ctypes.c_int
    L.or_smr_divergence.argtypes = [pp, sp, dp, dp, ctypes.POINTER(ctypes.c_longlong)]
    L.or_smr_divergence.restype = ctypes.c_int
    return L


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params(pb) -> Params:
    """ctypes parameter block from a ``problems.Problem``."""
    P = Params()
    for d in range(3):
        P.n[d] = int(pb.n[d])
        P.bc[d][0] = int(pb.bc[d][0])
        P.bc[d][1] = int(pb.bc[d][1])
        P.dx[d] = float(pb.dx[d])
    P.recon = int(pb.recon)
    P.fofc = int(getattr(pb, "fofc", 0))
    P.rk = int(getattr(pb, "rk", 2))
    P.gamma = float(pb.gamma)
    P.cfl = float(pb.cfl)
    P.rho_floor = float(pb.rho_floor)
    P.p_floor = float(pb.p_floor)
    return P


class Oracle:
    """The reference solver bound to one compiled library (default: the
    committed source built as liboracle.so)."""

    def __init__(self, handle=None):
        self._L = handle if handle is not None else lib()

    @classmethod
    def from_path(cls, path):
        return cls(_bind(ctypes.CDLL(path)))

    def set_threads(self, n: int) -> None:
        self._L.or_set_threads(int(n))

    def get_threads(self) -> int:
        return int(self._L.or_get_threads())

    def new_dt(self, pb, U=None) -> float:
        """CFL time step of a state (Sec. 3, Eq. 3)."""
        U = np.ascontiguousarray(pb.U if U is None else U, dtype=np.float64)
        P = params(pb)
        if pb.refine is not None:
            S = smr_params(pb)
            return float(self._L.or_smr_new_dt(ctypes.byref(P), ctypes.byref(S), _dp(U)))
        return float(self._L.or_new_dt(ctypes.byref(P), _dp(U)))

    def smr_leaves(self, pb):
        """Leaves of a refined mesh as int32 [leaf][level, lx, ly, lz]."""
        P, S = params(pb), smr_params(pb)
        n = self._L.or_smr_leaves(ctypes.byref(P), ctypes.byref(S), None)
        if n < 0:
            raise ValueError(f"bad refined mesh (status {-n})")
        out = np.zeros((n, 4), dtype=np.int32)
        self._L.or_smr_leaves(ctypes.byref(P), ctypes.byref(S),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return out

    def smr_fill_ghosts(self, pb, U=None):
        """Ghosted leaves [leaf][5][bz+2g][by+2g][bx+2g]: face ghosts from the
        level representation, edges and corners 0."""
        U = np.ascontiguousarray(pb.U if U is None else U, dtype=np.float64)
        g = self._L.or_nghost(int(pb.recon))
        bx, by, bz = pb.block
        out = np.zeros((U.shape[0], 5, bz + 2 * g, by + 2 * g, bx + 2 * g))
        P, S = params(pb), smr_params(pb)
        st = self._L.or_smr_fill_ghosts(ctypes.byref(P), ctypes.byref(S), _dp(U), _dp(out))
        if st != OK:
            raise ValueError(f"or_smr_fill_ghosts status {st}")
        return out

    def smr_divergence(self, pb, U=None):
        U = np.ascontiguousarray(pb.U if U is None else U, dtype=np.float64)
        L = np.empty_like(U)
        P, S = params(pb), smr_params(pb)
        fh = ctypes.c_longlong(0)
        st = self._L.or_smr_divergence(ctypes.byref(P), ctypes.byref(S), _dp(U), _dp(L),
                                       ctypes.byref(fh))
        return L, st, fh.value

    def advance(self, pb, nsteps: int, U=None, t: float = 0.0, dt: float | None = None):
        """Run ``nsteps`` RK2 steps from state U (default ``pb.U``).

        Returns a dict with the final U, t, the dt for the next step, the floor
        hits and the status code. The first step uses ``dt`` or, if None, the CFL
        step of the initial state.
        """
        U = np.array(pb.U if U is None else U, dtype=np.float64, order="C", copy=True)
        P = params(pb)
        if dt is None:
            dt = self.new_dt(pb, U)
        tt = ctypes.c_double(t)
        dd = ctypes.c_double(dt)
        fh = ctypes.c_longlong(0)
        fc = ctypes.c_longlong(0)
        if pb.refine is not None:  # statically refined mesh, leaf-major U
            S = smr_params(pb)
            st = self._L.or_smr_advance(ctypes.byref(P), ctypes.byref(S), _dp(U), int(nsteps),
                                        ctypes.byref(tt), ctypes.byref(dd), ctypes.byref(fh),
                                        ctypes.byref(fc))
            return dict(U=U, t=tt.value, dt=dd.value, floor_hits=fh.value, fofc_cells=fc.value,
                        status=st)
        st = self._L.or_advance(ctypes.byref(P), _dp(U), int(nsteps), ctypes.byref(tt),
                                ctypes.byref(dd), ctypes.byref(fh), ctypes.byref(fc))
        return dict(U=U, t=tt.value, dt=dd.value, floor_hits=fh.value, fofc_cells=fc.value,
                    status=st)

    def divergence(self, pb, U=None):
        U = np.ascontiguousarray(pb.U if U is None else U, dtype=np.float64)
        L = np.empty_like(U)
        P = params(pb)
        fh = ctypes.c_longlong(0)
        st = self._L.or_divergence(ctypes.byref(P), _dp(U), _dp(L), ctypes.byref(fh))
        return L, st, fh.value

    def fill_ghosts(self, pb, U=None):
        U = np.ascontiguousarray(pb.U if U is None else U, dtype=np.float64)
        g = self._L.or_nghost(int(pb.recon))
        nx, ny, nz = pb.n
        out = np.full((5, nz + 2 * g, ny + 2 * g, nx + 2 * g), np.nan)
        P = params(pb)
        self._L.or_fill_ghosts(ctypes.byref(P), _dp(U), _dp(out))
        return out

    def c2p(self, pb, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.empty(5)
        bad = ctypes.c_int(0)
        P = params(pb)
        hit = self._L.or_c2p(ctypes.byref(P), _dp(u), _dp(w), ctypes.byref(bad))
        return w, hit, bad.value

    def plm_cell(self, wm, w0, wp):
        l = ctypes.c_double()
        r = ctypes.c_double()
        self._L.or_plm_cell(float(wm), float(w0), float(wp), ctypes.byref(l), ctypes.byref(r))
        return l.value, r.value

    def ppm4_cell(self, w5):
        w = np.ascontiguousarray(w5, dtype=np.float64)
        l = ctypes.c_double()
        r = ctypes.c_double()
        self._L.or_ppm4_cell(_dp(w), ctypes.byref(l), ctypes.byref(r))
        return l.value, r.value

    def ppmx_cell(self, w5):
        w = np.ascontiguousarray(w5, dtype=np.float64)
        l, r = ctypes.c_double(), ctypes.c_double()
        self._L.or_ppmx_cell(_dp(w), ctypes.byref(l), ctypes.byref(r))
        return l.value, r.value

    def wenoz_cell(self, w5):
        w = np.ascontiguousarray(w5, dtype=np.float64)
        l, r = ctypes.c_double(), ctypes.c_double()
        self._L.or_wenoz_cell(_dp(w), ctypes.byref(l), ctypes.byref(r))
        return l.value, r.value

    def llf(self, gamma, wl, wr):
        """LLF flux for primitive states [rho, u_n, u_t1, u_t2, p]."""
        a = np.ascontiguousarray(wl, dtype=np.float64)
        b = np.ascontiguousarray(wr, dtype=np.float64)
        f = np.empty(5)
        self._L.or_llf(float(gamma), _dp(a), _dp(b), _dp(f))
        return f

    def hllc(self, gamma, wl, wr):
        """HLLC flux for primitive states [rho, u_n, u_t1, u_t2, p]."""
        a = np.ascontiguousarray(wl, dtype=np.float64)
        b = np.ascontiguousarray(wr, dtype=np.float64)
        f = np.empty(5)
        self._L.or_hllc(float(gamma), _dp(a), _dp(b), _dp(f))
        return f


_default = None


def _inst():
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def set_threads(n):
    return _inst().set_threads(n)


def get_threads():
    return _inst().get_threads()


def new_dt(pb, U=None):
    return _inst().new_dt(pb, U)


def advance(pb, nsteps, U=None, t=0.0, dt=None):
    return _inst().advance(pb, nsteps, U=U, t=t, dt=dt)


def divergence(pb, U=None):
    return _inst().divergence(pb, U)


def fill_ghosts(pb, U=None):
    return _inst().fill_ghosts(pb, U)


def c2p(pb, u):
    return _inst().c2p(pb, u)


def plm_cell(wm, w0, wp):
    return _inst().plm_cell(wm, w0, wp)


def ppm4_cell(w5):
    return _inst().ppm4_cell(w5)


def ppmx_cell(w5):
    return _inst().ppmx_cell(w5)


def wenoz_cell(w5):
    return _inst().wenoz_cell(w5)


def hllc(gamma, wl, wr):
    return _inst().hllc(gamma, wl, wr)


def llf(gamma, wl, wr):
    return _inst().llf(gamma, wl, wr)


def smr_leaves(pb):
    return _inst().smr_leaves(pb)


def smr_fill_ghosts(pb, U=None):
    return _inst().smr_fill_ghosts(pb, U)


def smr_divergence(pb, U=None):
    return _inst().smr_divergence(pb, U)
