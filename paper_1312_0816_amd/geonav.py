"""Python binding of libgeonav.so (ctypes, argument marshalling only).

Every computation runs in the HIP library; this module checks tensor
dtype/device/layout, passes raw device pointers and the current HIP stream,
and maps nonzero status codes to exceptions. There is no fallback path: if
the library is not built, importing or calling raises.

Tracks are float64 CUDA tensors of shape (6, n) (rows x, y, z, ux, uy, uz),
or separate (3, n) origin and direction tensors. Outputs are allocated with
torch on the tracks' device.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import build as _build

# the in-tree build; GEONAV_LIBRARY may name another build of the same sources
LIB_PATH = os.environ.get("GEONAV_LIBRARY", _build.LIB)

GEO_BOX, GEO_TUBE, GEO_CONE, GEO_TUBS, GEO_CONS, GEO_PCON = 0, 1, 2, 3, 4, 5
CENSUS_SLOTS, CENSUS_CULL, CENSUS_TRACKS = 16, 14, 15
GEO_CONTAINS, GEO_SAFETY, GEO_DIST_IN, GEO_DIST_OUT = 0, 1, 2, 3
GEO_BIG = 1e30
GEO_MAX_DAUGHTERS = 1024
GEO_PCON_MAX_PLANES = 8
NPAR = 3 + 3 * GEO_PCON_MAX_PLANES   # parameters per shape (GEO_NPAR)


class GeoTracks(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("ux", C.c_void_p), ("uy", C.c_void_p), ("uz", C.c_void_p),
                ("n", C.c_int64)]


class GeoShape(C.Structure):
    _fields_ = [("kind", C.c_int32), ("_pad", C.c_int32), ("par", C.c_double * NPAR)]


def make_shape(kind: int, par) -> "GeoShape":
    """GeoShape from a kind and up to NPAR parameters (zero-padded)."""
    p = [float(v) for v in np.asarray(par, np.float64).reshape(-1)]
    if len(p) > NPAR:
        raise ValueError(f"at most {NPAR} shape parameters")
    p += [0.0] * (NPAR - len(p))
    return GeoShape(int(kind), 0, (C.c_double * NPAR)(*p))


class GeoPlacement(C.Structure):
    _fields_ = [("rot", C.c_double * 9), ("tr", C.c_double * 3)]


class GeoVolumeDesc(C.Structure):
    _fields_ = [("mother", GeoShape), ("ndaughters", C.c_int32), ("_pad", C.c_int32),
                ("daughters", C.POINTER(GeoShape)), ("placements", C.POINTER(GeoPlacement))]


class GeoBasket(C.Structure):
    _fields_ = [("volume", C.c_int32), ("_pad", C.c_int32), ("offset", C.c_int64),
                ("n", C.c_int64)]


EXPORTS = ("geo_geometry_create", "geo_geometry_destroy", "geo_shape_query",
           "geo_navigate_basket", "geo_navigate_batched", "geo_navigate_backward",
           "geo_autotune", "geo_get_launch_config", "geo_set_launch_config", "geo_get_batched_graph",
           "geo_set_batched_graph", "geo_set_culling",
           "geo_get_culling", "geo_navigate_batched_census", "geo_navigate_safety",
           "geo_locate", "geo_set_kernel_timing", "geo_batched_kernel_ms", "geo_navigate_backward_noalloc",
           "geo_strerror")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgeonav.so and declare its signatures. Raises OSError if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libgeonav.so is not built ({path}); run __graft_entry__.build()")
    lib = C.CDLL(path)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    lib.geo_geometry_create.argtypes = [C.POINTER(GeoVolumeDesc), I32, C.POINTER(P)]
    lib.geo_geometry_destroy.argtypes = [P]
    lib.geo_shape_query.argtypes = [C.POINTER(GeoShape), I32, GeoTracks, P, P]
    lib.geo_navigate_basket.argtypes = [P, I32, GeoTracks, P, P, P, P, P]
    lib.geo_navigate_batched.argtypes = [P, C.POINTER(GeoBasket), I32, GeoTracks, P, P, P]
    lib.geo_navigate_backward.argtypes = [P, I32, GeoTracks, P, P, P, P, P, P, P]
    lib.geo_navigate_backward_noalloc.argtypes = [P, I32, GeoTracks, P, P, P, P, P, P, P]
    lib.geo_autotune.argtypes = [P, C.POINTER(GeoBasket), I32, GeoTracks, P]
    lib.geo_get_launch_config.argtypes = [P, C.POINTER(I32), C.POINTER(I32)]
    lib.geo_set_launch_config.argtypes = [P, I32, I32]
    lib.geo_get_batched_graph.argtypes = [P, C.POINTER(I32)]
    lib.geo_set_batched_graph.argtypes = [P, I32]
    lib.geo_set_culling.argtypes = [P, I32]
    lib.geo_navigate_safety.argtypes = [P, I32, GeoTracks, P, P, P]
    lib.geo_locate.argtypes = [P, I32, GeoTracks, P, P, P]
    lib.geo_navigate_batched_census.argtypes = [P, C.POINTER(GeoBasket), I32, GeoTracks, P, P,
                                                C.POINTER(C.c_uint64), P]
    lib.geo_get_culling.argtypes = [P, C.POINTER(I32)]
    lib.geo_set_kernel_timing.argtypes = [P, I32]
    lib.geo_batched_kernel_ms.argtypes = [P, C.POINTER(C.c_float)]
    lib.geo_strerror.argtypes = [C.c_int]
    lib.geo_strerror.restype = C.c_char_p
    for name in EXPORTS:
        if name != "geo_strerror":
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class GeoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"geonav status {status}: {msg}")
        self.status = status


def _check(rc: int):
    if rc != 0:
        raise GeoError(rc, _lib.geo_strerror(rc).decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, name: str, shape=None, dtype=torch.float64):
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a CUDA (HIP) device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def tracks_struct(o: torch.Tensor, d: torch.Tensor | None = None) -> GeoTracks:
    """GeoTracks over a (6, n) tensor, or over (3, n) origins and (3, n)
    directions (d may be None for Contains/Safety)."""
    if d is None and o.dim() == 2 and o.shape[0] == 6:
        _need(o, "tracks")
        n = o.shape[1]
        if n == 0:
            return GeoTracks(None, None, None, None, None, None, 0)
        b, s = o.data_ptr(), 8 * n
        return GeoTracks(b, b + s, b + 2 * s, b + 3 * s, b + 4 * s, b + 5 * s, n)
    if o.dim() != 2 or o.shape[0] != 3:
        raise ValueError("origins must have shape (3, n) (or tracks (6, n))")
    _need(o, "origins")
    n = o.shape[1]
    if d is not None:
        _need(d, "directions", (3, n))
    if n == 0:
        return GeoTracks(None, None, None, None, None, None, 0)
    b = o.data_ptr()
    if d is None:
        return GeoTracks(b, b + 8 * n, b + 16 * n, None, None, None, n)
    e = d.data_ptr()
    return GeoTracks(b, b + 8 * n, b + 16 * n, e, e + 8 * n, e + 16 * n, n)


def _has_dirs(o: torch.Tensor, d: torch.Tensor | None) -> bool:
    return d is not None or (o.dim() == 2 and o.shape[0] == 6)


# ------------------------------------------------------------ shape queries

def geo_shape_query(kind: int, par, query: int, tracks: torch.Tensor, out: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """One shape query (section 3.1) over every track of a (6, n) or (3, n)
    basket; returns uint8 (Contains) or float64."""
    lib = load_library()
    shape = make_shape(kind, par)
    t = tracks_struct(tracks)
    if query in (GEO_DIST_IN, GEO_DIST_OUT) and tracks.shape[0] != 6:
        raise ValueError("distance queries need (6, n) tracks")
    n = t.n
    if out is None:
        out = torch.empty(n, dtype=torch.uint8 if query == GEO_CONTAINS else torch.float64,
                          device=tracks.device)
    else:
        _need(out, "out", (n,), torch.uint8 if query == GEO_CONTAINS else torch.float64)
    _check(lib.geo_shape_query(C.byref(shape), int(query), t, _ptr(out), _stream(stream)))
    return out


# ------------------------------------------------------------- geometry

class Geometry:
    """Owns a geo_geometry handle built from workload ``Volume`` objects
    (mother_kind, mother_par, kinds, pars, rots, trs)."""

    def __init__(self, volumes):
        lib = load_library()
        vols = list(volumes)
        descs = (GeoVolumeDesc * len(vols))()
        self._keep = []
        self.nd = []
        for i, v in enumerate(vols):
            nd = int(len(v.kinds))
            sh = (GeoShape * max(nd, 1))()
            pl = (GeoPlacement * max(nd, 1))()
            for k in range(nd):
                sh[k] = make_shape(v.kinds[k], v.pars[k])
                pl[k] = GeoPlacement((C.c_double * 9)(*map(float, np.asarray(v.rots[k]).reshape(9))),
                                     (C.c_double * 3)(*map(float, v.trs[k])))
            descs[i].mother = make_shape(v.mother_kind, v.mother_par)
            descs[i].ndaughters = nd
            descs[i].daughters = C.cast(sh, C.POINTER(GeoShape))
            descs[i].placements = C.cast(pl, C.POINTER(GeoPlacement))
            self._keep += [sh, pl]
            self.nd.append(nd)
        h = C.c_void_p()
        _check(lib.geo_geometry_create(descs, len(vols), C.byref(h)))
        self._h = h
        self._lib = lib

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.geo_geometry_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def launch_config(self):
        u, w = C.c_int32(), C.c_int32()
        _check(self._lib.geo_get_launch_config(self._h, C.byref(u), C.byref(w)))
        return int(u.value), int(w.value)

    def set_launch_config(self, tracks_per_lane: int, waves_per_simd: int):
        _check(self._lib.geo_set_launch_config(self._h, int(tracks_per_lane), int(waves_per_simd)))

    @property
    def batched_graph(self) -> bool:
        """Whether geo_navigate_batched replays a HIP graph (else two launches)."""
        v = C.c_int32()
        _check(self._lib.geo_get_batched_graph(self._h, C.byref(v)))
        return bool(v.value)

    @batched_graph.setter
    def batched_graph(self, use_graph: bool):
        _check(self._lib.geo_set_batched_graph(self._h, 1 if use_graph else 0))

    @property
    def culling(self) -> bool:
        v = C.c_int32()
        _check(self._lib.geo_get_culling(self._h, C.byref(v)))
        return bool(v.value)

    @culling.setter
    def culling(self, enable: bool):
        _check(self._lib.geo_set_culling(self._h, 1 if enable else 0))

    def set_kernel_timing(self, enable: bool):
        """Record events around the batched navigator kernel (measurement)."""
        _check(self._lib.geo_set_kernel_timing(self._h, 1 if enable else 0))

    def batched_kernel_ms(self) -> float:
        """Duration of the navigator kernel of the latest batched call (waits
        for it); needs set_kernel_timing(True) first."""
        v = C.c_float()
        _check(self._lib.geo_batched_kernel_ms(self._h, C.byref(v)))
        return float(v.value)


def geo_geometry_create(volumes) -> Geometry:
    return Geometry(volumes)


def geo_navigate_basket(g: Geometry, volume: int, o: torch.Tensor, d: torch.Tensor | None = None,
                        offsets: torch.Tensor | None = None, hitpt: bool = False, stream=None):
    """Navigator of Fig. 1b over one basket. Returns (step, hit) or
    (step, hit, hitpt (3, n)) as tensors on the tracks' device."""
    if not _has_dirs(o, d):
        raise ValueError("the navigator needs directions")
    t = tracks_struct(o, d)
    n = t.n
    dev = o.device
    if offsets is not None:
        _need(offsets, "offsets", (g.nd[volume], 3))
    step = torch.empty(n, dtype=torch.float64, device=dev)
    hit = torch.empty(n, dtype=torch.int32, device=dev)
    hp = torch.empty((3, n), dtype=torch.float64, device=dev) if hitpt else None
    _check(g._lib.geo_navigate_basket(g.handle, int(volume), t, _ptr(offsets), _ptr(step), _ptr(hit),
                                      _ptr(hp), _stream(stream)))
    return (step, hit, hp) if hitpt else (step, hit)


def geo_navigate_safety(g: Geometry, volume: int, points: torch.Tensor,
                        offsets: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Isotropic safety of the navigator for (3, n) or (6, n) points."""
    t = tracks_struct(points)
    if offsets is not None:
        _need(offsets, "offsets", (g.nd[volume], 3))
    out = torch.empty(t.n, dtype=torch.float64, device=points.device)
    _check(g._lib.geo_navigate_safety(g.handle, int(volume), t, _ptr(offsets), _ptr(out), _stream(stream)))
    return out


def geo_locate(g: Geometry, volume: int, points: torch.Tensor, offsets: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """Daughter index holding each point, -1 (mother only) or -2 (outside)."""
    t = tracks_struct(points)
    if offsets is not None:
        _need(offsets, "offsets", (g.nd[volume], 3))
    out = torch.empty(t.n, dtype=torch.int32, device=points.device)
    _check(g._lib.geo_locate(g.handle, int(volume), t, _ptr(offsets), _ptr(out), _stream(stream)))
    return out


def _baskets(volume, offset, n):
    volume = np.asarray(volume, np.int64).reshape(-1)
    offset = np.asarray(offset, np.int64).reshape(-1)
    n = np.asarray(n, np.int64).reshape(-1)
    if not (volume.shape == offset.shape == n.shape):
        raise ValueError("basket arrays differ in length")
    arr = (GeoBasket * max(len(n), 1))()
    for i in range(len(n)):
        arr[i] = GeoBasket(int(volume[i]), 0, int(offset[i]), int(n[i]))
    return arr, len(n)


def geo_navigate_batched(g: Geometry, basket_volume, basket_offset, basket_n, tracks: torch.Tensor,
                         step: torch.Tensor | None = None, hit: torch.Tensor | None = None,
                         stream=None):
    """All baskets in one persistent launch. Outputs are indexed like the
    pool; returns (step, hit)."""
    t = tracks_struct(tracks)
    n = t.n
    if step is None:
        step = torch.empty(n, dtype=torch.float64, device=tracks.device)
    if hit is None:
        hit = torch.empty(n, dtype=torch.int32, device=tracks.device)
    _need(step, "step", (n,))
    _need(hit, "hit", (n,), torch.int32)
    arr, nb = _baskets(basket_volume, basket_offset, basket_n)
    _check(g._lib.geo_navigate_batched(g.handle, arr, nb, t, _ptr(step), _ptr(hit), _stream(stream)))
    return step, hit


def geo_navigate_batched_census(g: Geometry, basket_volume, basket_offset, basket_n,
                                tracks: torch.Tensor, stream=None):
    """Instrumented batched run. Returns (step, hit, counts[CENSUS_SLOTS])
    with counts as documented in geonav.h: lane-evaluations per slot
    2 * kind + hole, culling tests at CENSUS_CULL, tracks at CENSUS_TRACKS."""
    t = tracks_struct(tracks)
    n = t.n
    step = torch.empty(n, dtype=torch.float64, device=tracks.device)
    hit = torch.empty(n, dtype=torch.int32, device=tracks.device)
    arr, nb = _baskets(basket_volume, basket_offset, basket_n)
    counts = (C.c_uint64 * CENSUS_SLOTS)()
    _check(g._lib.geo_navigate_batched_census(g.handle, arr, nb, t, _ptr(step), _ptr(hit), counts,
                                              _stream(stream)))
    return step, hit, [int(c) for c in counts]


def geo_autotune(g: Geometry, basket_volume, basket_offset, basket_n, tracks: torch.Tensor, stream=None):
    t = tracks_struct(tracks)
    arr, nb = _baskets(basket_volume, basket_offset, basket_n)
    _check(g._lib.geo_autotune(g.handle, arr, nb, t, _stream(stream)))
    return g.launch_config()


def geo_navigate_backward(g: Geometry, volume: int, o: torch.Tensor, d: torch.Tensor,
                          offsets: torch.Tensor | None = None, gstep: torch.Tensor | None = None,
                          ghit: torch.Tensor | None = None, want_o: bool = True, want_d: bool = True,
                          want_off: bool = True, stream=None):
    """Adjoint of the navigator. Returns (g_o (3, n), g_d (3, n), g_off (nd, 3));
    entries not wanted are None."""
    t = tracks_struct(o, d)
    n = t.n
    dev = o.device
    nd = g.nd[volume]
    if offsets is not None:
        _need(offsets, "offsets", (nd, 3))
    if gstep is not None:
        _need(gstep, "gstep", (n,))
    if ghit is not None:
        _need(ghit, "ghit", (3, n))
    g_o = torch.empty((3, n), dtype=torch.float64, device=dev) if want_o else None
    g_d = torch.empty((3, n), dtype=torch.float64, device=dev) if want_d else None
    g_off = torch.zeros((nd, 3), dtype=torch.float64, device=dev) if (want_off and nd > 0) else None
    _check(g._lib.geo_navigate_backward(g.handle, int(volume), t, _ptr(offsets), _ptr(gstep), _ptr(ghit),
                                        _ptr(g_o), _ptr(g_d), _ptr(g_off), _stream(stream)))
    if want_off and nd == 0:
        g_off = torch.zeros((0, 3), dtype=torch.float64, device=dev)
    return g_o, g_d, g_off


def geo_navigate_backward_noalloc(g: Geometry, volume: int, o: torch.Tensor, d: torch.Tensor,
                                  offsets: torch.Tensor | None, gstep: torch.Tensor | None,
                                  ghit: torch.Tensor | None, g_o: torch.Tensor | None, g_d: torch.Tensor | None,
                                  g_off: torch.Tensor | None, stream=None):
    """geo_navigate_backward into caller-provided outputs (None to skip):
    g_o, g_d (3, n) and g_off (nd, 3) float64 on the tracks' device. Neither
    this wrapper nor the library allocates anything."""
    t = tracks_struct(o, d)
    n = t.n
    nd = g.nd[volume]
    for name, x, shape in (("offsets", offsets, (nd, 3)), ("gstep", gstep, (n,)), ("ghit", ghit, (3, n)),
                           ("g_o", g_o, (3, n)), ("g_d", g_d, (3, n)), ("g_off", g_off, (nd, 3))):
        if x is not None:
            _need(x, name, shape)
    _check(g._lib.geo_navigate_backward_noalloc(g.handle, int(volume), t, _ptr(offsets), _ptr(gstep), _ptr(ghit),
                                                _ptr(g_o), _ptr(g_d), _ptr(g_off), _stream(stream)))


class Navigate(torch.autograd.Function):
    """Differentiable navigator step: (o, d, offsets) -> (step, hit point, hit).

    forward:  geo_navigate_basket (hit is a non-differentiable int32 output)
    backward: geo_navigate_backward with the upstream gradients of step and
              hit point; the active surface is recomputed, not stored.
    """

    @staticmethod
    def forward(ctx, geometry: Geometry, volume: int, o: torch.Tensor, d: torch.Tensor,
                offsets: torch.Tensor | None = None):
        step, hit, hp = geo_navigate_basket(geometry, volume, o, d, offsets, hitpt=True)
        ctx.geometry = geometry
        ctx.volume = volume
        ctx.save_for_backward(o, d, offsets if offsets is not None else torch.empty(0))
        ctx.has_offsets = offsets is not None
        ctx.mark_non_differentiable(hit)
        return step, hp, hit

    @staticmethod
    def backward(ctx, g_step, g_hitpt, _g_hit):
        o, d, offs = ctx.saved_tensors
        offsets = offs if ctx.has_offsets else None
        gs = None if g_step is None else g_step.contiguous()
        gh = None if g_hitpt is None else g_hitpt.contiguous()
        need_o, need_d = ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        need_off = ctx.has_offsets and ctx.needs_input_grad[4]
        g_o, g_d, g_off = geo_navigate_backward(ctx.geometry, ctx.volume, o, d, offsets, gs, gh,
                                                want_o=need_o, want_d=need_d, want_off=need_off)
        return None, None, g_o, g_d, (g_off if need_off else None)


def navigate(geometry: Geometry, volume: int, o, d, offsets=None):
    """(step, hit point (3, n), hit) with autograd through Navigate."""
    return Navigate.apply(geometry, volume, o, d, offsets)
