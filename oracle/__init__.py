"""CPU oracle for the basket shape queries and the simple navigator.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The product path
(the HIP library and its binding) never does.

Thin ctypes wrapper over ``liboracle.so`` (plain C, built from ``oracle.c``
by :func:`build`). Each call takes the same numpy arrays the GPU path reads:
tracks as a (6, n) float64 array of rows x, y, z, ux, uy, uz.

``prec`` selects the build: ``"d"`` (double) or ``"ld"`` (x87 long double,
the higher-precision rerun).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "oracle_body.h")]

BOX, TUBE, CONE, TUBS, CONS, PCON = 0, 1, 2, 3, 4, 5
CONTAINS, SAFETY, DIST_IN, DIST_OUT = 0, 1, 2, 3
BIG = 1e30

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fused multiply-add, no fast-math)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-Wno-unused-function", "-o", LIB + ".tmp", SRC[0], "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or any(os.path.getmtime(s) > os.path.getmtime(LIB) for s in SRC):
            build()
        lib = C.CDLL(LIB)
        P = C.c_void_p
        for sfx in ("_d", "_ld"):
            f = getattr(lib, "or_shape_query" + sfx)
            f.argtypes = [C.c_int, P, C.c_int, C.c_int64] + [P] * 6 + [P, P]
            f.restype = None
            f = getattr(lib, "or_navigate" + sfx)
            f.argtypes = [C.c_int, P, C.c_int, P, P, P, P, P, C.c_int64] + [P] * 6 + [P, P, P]
            f.restype = None
            f = getattr(lib, "or_navigate_fd" + sfx)
            f.argtypes = ([C.c_int, P, C.c_int, P, P, P, P, P, C.c_int64] + [P] * 6 +
                          [P, P, C.c_double, C.c_double, C.c_double, C.c_double] + [P] * 5)
            f.restype = None
            f = getattr(lib, "or_navigate_safety" + sfx)
            f.argtypes = [C.c_int, P, C.c_int, P, P, P, P, P, C.c_int64, P, P, P, P]
            f.restype = None
            f = getattr(lib, "or_locate" + sfx)
            f.argtypes = [C.c_int, P, C.c_int, P, P, P, P, P, C.c_int64, P, P, P, P]
            f.restype = None
        lib.or_max_daughters.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


NPAR = 27      # 3 + 3 x 8 polycone planes


def _parn(par):
    """Shape parameters padded with zeros to the NPAR the library reads."""
    p = np.zeros(NPAR)
    v = np.asarray(par, np.float64).reshape(-1)
    p[:v.size] = v
    return p


def _tracks(t):
    t = _f64(t)
    if t.ndim != 2 or t.shape[0] not in (3, 6):
        raise ValueError("tracks must be (6, n) or (3, n) float64")
    if t.shape[0] == 3:
        t = np.ascontiguousarray(np.concatenate([t, np.zeros_like(t)]))
    return t


def shape_query(kind: int, par, query: int, tracks, prec: str = "d"):
    """One query for every track. Returns uint8 (Contains) or float64."""
    lib = _load()
    t = _tracks(tracks)
    n = t.shape[1]
    par = _parn(par)
    vals = np.zeros(n, np.float64)
    ins = np.zeros(n, np.uint8)
    rows = [t[i] for i in range(6)]
    getattr(lib, "or_shape_query_" + prec)(int(kind), _ptr(par), int(query), n,
                                           *[_ptr(r) for r in rows], _ptr(vals), _ptr(ins))
    return ins if query == CONTAINS else vals


def contains(kind, par, tracks, prec="d"):
    return shape_query(kind, par, CONTAINS, tracks, prec)


def safety(kind, par, tracks, prec="d"):
    return shape_query(kind, par, SAFETY, tracks, prec)


def dist_in(kind, par, tracks, prec="d"):
    return shape_query(kind, par, DIST_IN, tracks, prec)


def dist_out(kind, par, tracks, prec="d"):
    return shape_query(kind, par, DIST_OUT, tracks, prec)


def _vol_args(vol):
    v = vol.normalized() if hasattr(vol, "normalized") else vol
    if v.nd > _load().or_max_daughters():
        raise ValueError("too many daughters for the oracle")
    return v, (int(v.mother_kind), _ptr(v.mother_par), v.nd, _ptr(v.kinds), _ptr(v.pars),
               _ptr(v.rots), _ptr(v.trs))


def navigate(vol, tracks, offsets=None, prec: str = "d"):
    """Navigator of Fig. 1 for every track.
    Returns (step float64[n], hit int32[n] (-1 = mother), gap float64[n])."""
    lib = _load()
    v, args = _vol_args(vol)
    t = _tracks(tracks)
    n = t.shape[1]
    offs = None if offsets is None else _f64(offsets, (v.nd, 3))
    step = np.zeros(n)
    hit = np.zeros(n, np.int32)
    gap = np.zeros(n)
    getattr(lib, "or_navigate_" + prec)(*args, _ptr(offs), n, *[_ptr(t[i]) for i in range(6)],
                                        _ptr(step), _ptr(hit), _ptr(gap))
    return step, hit, gap


def navigate_fd(vol, tracks, offsets=None, gstep=None, ghit=None, h: float = 1e-6,
                min_gap: float = 1e-4, kink_tol: float = 1e-3, fd_tol: float = 1e-7,
                prec: str = "ld"):
    """Central finite differences (step h) of phi = gstep*s + ghit.(o + s d).

    Returns dict with g_o (3, n), g_d (3, n), g_off_hit (3, n) (gradient with
    respect to the offset of the hit daughter; 0 for mother hits), hit (n,)
    and mask (n,) (1 = smooth within the stencil, usable as a reference).
    """
    lib = _load()
    v, args = _vol_args(vol)
    t = _tracks(tracks)
    n = t.shape[1]
    offs = None if offsets is None else _f64(offsets, (v.nd, 3))
    gs = None if gstep is None else _f64(gstep, (n,))
    gh = None if ghit is None else _f64(ghit, (3, n))
    g_o = np.zeros((3, n))
    g_d = np.zeros((3, n))
    g_off = np.zeros((3, n))
    hit = np.zeros(n, np.int32)
    mask = np.zeros(n, np.uint8)
    getattr(lib, "or_navigate_fd_" + prec)(*args, _ptr(offs), n, *[_ptr(t[i]) for i in range(6)],
                                           _ptr(gs), _ptr(gh), float(h), float(min_gap),
                                           float(kink_tol), float(fd_tol), _ptr(g_o), _ptr(g_d),
                                           _ptr(g_off), _ptr(hit), _ptr(mask))
    return {"g_o": g_o, "g_d": g_d, "g_off_hit": g_off, "hit": hit, "mask": mask.astype(bool)}


def navigate_safety(vol, points, offsets=None, prec: str = "d"):
    """Safe distance to the volume's boundaries: min of the mother's Safety
    and every daughter's Safety in its frame. points: (3, n) or (6, n)."""
    lib = _load()
    v, args = _vol_args(vol)
    t = _tracks(points)
    n = t.shape[1]
    offs = None if offsets is None else _f64(offsets, (v.nd, 3))
    out = np.zeros(n)
    getattr(lib, "or_navigate_safety_" + prec)(*args, _ptr(offs), n, _ptr(t[0]), _ptr(t[1]), _ptr(t[2]),
                                               _ptr(out))
    return out


def locate(vol, points, offsets=None, prec: str = "d"):
    """Index of the daughter holding each point (lowest index), -1 for the
    mother's own part, -2 outside the mother."""
    lib = _load()
    v, args = _vol_args(vol)
    t = _tracks(points)
    n = t.shape[1]
    offs = None if offsets is None else _f64(offsets, (v.nd, 3))
    out = np.zeros(n, np.int32)
    getattr(lib, "or_locate_" + prec)(*args, _ptr(offs), n, _ptr(t[0]), _ptr(t[1]), _ptr(t[2]), _ptr(out))
    return out
