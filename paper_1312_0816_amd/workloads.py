"""Seeded synthetic workloads: shapes, logical volumes and track baskets.

This module only *draws* inputs. It evaluates none of the shape queries and
none of the navigator: no Contains, Safety or distance is computed here. Both
the CPU oracle and the HIP path read the exact arrays it returns.

Everything is drawn from ``numpy.random.default_rng(seed)`` (PCG64), so a
(workload, seed) pair names one byte-identical input.

Layouts
-------
* Tracks: one C-contiguous float64 array of shape (6, n). Rows are
  x, y, z, ux, uy, uz, i.e. six SoA component arrays. This is the "basket"
  container of the paper (section 2): the particles of one logical volume,
  contiguous in memory.
* Shape: ``(kind, par)`` with ``par`` five float64 values, ROOT-style
  half-lengths centred on the origin with z as the axis:
  BOX (dx, dy, dz), TUBE (rmin, rmax, dz), CONE (dz, rmin1, rmax1, rmin2,
  rmax2), where the "1" radii sit at z = -dz and the "2" radii at z = +dz.
* Volume: a mother shape and daughters placed by a rotation R (row-major 3x3)
  and a translation T, so that a daughter-frame point q sits at R q + T in
  the mother frame (the navigator of section 3, Fig. 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BOX, TUBE, CONE, TUBS, CONS, PCON = 0, 1, 2, 3, 4, 5
KIND_NAMES = {BOX: "box", TUBE: "tube", CONE: "cone", TUBS: "tube segment",
              CONS: "cone segment", PCON: "polycone"}
PCON_MAX = 8   # z planes of a polycone
NPAR = 3 + 3 * PCON_MAX   # parameters per shape (zero-padded)


def pcon_par(phi1, dphi, planes):
    """Polycone parameters {phi1, dphi, nz, z_0, rmin_0, rmax_0, ...} from a
    list of (z, rmin, rmax) planes (z strictly increasing)."""
    out = [float(phi1), float(dphi), float(len(planes))]
    for z, a, b in planes:
        out += [float(z), float(a), float(b)]
    return np.array(out)


def pcon_planes(par):
    """(z, rmin, rmax) arrays of a polycone's parameters."""
    par = np.asarray(par, np.float64).reshape(-1)
    n = int(par[2])
    q = par[3:3 + 3 * n].reshape(n, 3)
    return q[:, 0], q[:, 1], q[:, 2]

# Shape-suite shapes (parameter order as above).
SUITE_SHAPES = {
    BOX: np.array([10.0, 20.0, 30.0, 0.0, 0.0]),
    TUBE: np.array([5.0, 15.0, 20.0, 0.0, 0.0]),
    CONE: np.array([20.0, 0.0, 10.0, 5.0, 20.0]),
    # 240-degree tube segment (a non-convex azimuth range) and a 150-degree
    # cone segment with a hole that closes to 2 at the narrow end
    TUBS: np.array([5.0, 15.0, 20.0, np.pi / 6, 4 * np.pi / 3]),
    CONS: np.array([20.0, 2.0, 10.0, 5.0, 20.0, -np.pi / 4, 5 * np.pi / 6]),
    # polycone of four sections: the hole opens from an apex at z = -20,
    # the outer radius rises to a plateau and falls again
    PCON: pcon_par(0.0, 2 * np.pi, [(-20.0, 0.0, 6.0), (-8.0, 3.0, 12.0), (0.0, 3.0, 15.0),
                                    (12.0, 5.0, 15.0), (20.0, 2.0, 8.0)]),
}

# Polycones for the parity tests: two planes (the cone of the suite), a
# pipe with a flared end, eight planes with a zig-zag outer profile, the
# same cut to a non-convex range, a spindle (apexes at both ends) cut to a
# convex range, and three collinear planes (the suite cone again).
_ZIGZAG = [(-30.0, 2.0, 8.0), (-22.0, 3.0, 12.0), (-15.0, 3.0, 6.0), (-5.0, 1.0, 14.0),
           (0.0, 1.0, 14.0), (6.0, 4.0, 9.0), (18.0, 2.0, 16.0), (30.0, 2.0, 5.0)]
PCON_VARIANTS = [
    pcon_par(0.0, 2 * np.pi, [(-20.0, 0.0, 10.0), (20.0, 5.0, 20.0)]),
    pcon_par(0.0, 2 * np.pi, [(-10.0, 0.0, 5.0), (0.0, 0.0, 5.0), (10.0, 0.0, 10.0)]),
    pcon_par(0.0, 2 * np.pi, _ZIGZAG),
    pcon_par(0.4, 4.0, _ZIGZAG),
    pcon_par(-1.0, 1.5, [(-12.0, 0.0, 0.0), (0.0, 0.0, 10.0), (12.0, 0.0, 0.0)]),
    pcon_par(0.0, 2 * np.pi, [(-20.0, 0.0, 10.0), (0.0, 2.5, 15.0), (20.0, 5.0, 20.0)]),
]

# Further segments for the parity tests: narrow, right-angle, half and wide
# ranges, ranges that wrap through phi = pi, solid (no hole) profiles whose
# faces meet on the axis, and a range just short of a full turn.
SEGMENT_VARIANTS = [
    (TUBS, np.array([0.0, 10.0, 10.0, 0.0, np.pi / 2])),
    (TUBS, np.array([2.0, 10.0, 5.0, np.pi / 2, 3 * np.pi / 2])),
    (TUBS, np.array([4.0, 12.0, 8.0, 2.5, 0.3])),
    (TUBS, np.array([0.0, 12.0, 8.0, -1.0, np.pi])),
    (TUBS, np.array([3.0, 9.0, 6.0, 0.7, 2 * np.pi - 1e-3])),
    (CONS, np.array([10.0, 0.0, 10.0, 0.0, 20.0, 0.0, np.pi])),
    (CONS, np.array([5.0, 2.0, 4.0, 2.0, 4.0, -np.pi / 4, np.pi / 2])),
    (CONS, np.array([12.0, 0.0, 3.0, 6.0, 14.0, 2.0, 4.0])),
    (CONS, np.array([12.0, 1.0, 14.0, 0.0, 3.0, -3.0, 1.2])),
]

MOTHER_HALF = 200.0


def isotropic(rng: np.random.Generator, n: int):
    """Unit directions with cos(theta) ~ U[-1, 1] and phi ~ U[0, 2 pi)."""
    ct = rng.uniform(-1.0, 1.0, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    return st * np.cos(ph), st * np.sin(ph), ct


def pack_tracks(x, y, z, ux, uy, uz) -> np.ndarray:
    return np.ascontiguousarray(np.stack([x, y, z, ux, uy, uz]).astype(np.float64))


@dataclass
class Volume:
    """A logical volume: mother shape plus placed daughters."""

    mother_kind: int
    mother_par: np.ndarray                     # (NPAR,) or shorter, zero-padded
    kinds: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))   # (nd,)
    pars: np.ndarray = field(default_factory=lambda: np.zeros((0, NPAR)))    # (nd, <= NPAR)
    rots: np.ndarray = field(default_factory=lambda: np.zeros((0, 9)))       # (nd, 9) row-major R
    trs: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))        # (nd, 3) T
    bound_r: np.ndarray = field(default_factory=lambda: np.zeros(0))         # (nd,) generator-side bounding radius

    @property
    def nd(self) -> int:
        return int(self.kinds.shape[0])

    def normalized(self) -> "Volume":
        mp = np.zeros(NPAR)
        m = np.asarray(self.mother_par, np.float64).reshape(-1)
        mp[:m.size] = m
        pr = np.asarray(self.pars, np.float64)
        pr = pr.reshape(pr.shape[0] if pr.ndim == 2 else 0, -1) if pr.size else np.zeros((0, NPAR))
        pars = np.zeros((pr.shape[0], NPAR))
        pars[:, :pr.shape[1]] = pr
        return Volume(int(self.mother_kind), mp,
                      np.ascontiguousarray(self.kinds, np.int32).reshape(-1),
                      pars,
                      np.ascontiguousarray(self.rots, np.float64).reshape(-1, 9),
                      np.ascontiguousarray(self.trs, np.float64).reshape(-1, 3),
                      np.ascontiguousarray(self.bound_r, np.float64).reshape(-1))


# ----------------------------------------------------------------------------
# Shape-suite inputs
# ----------------------------------------------------------------------------

def box_c0(seed: int = 1000, n: int = 1024):
    """Box (10, 20, 30): origins uniform in the cube of half-size 60,
    isotropic directions. Returns (kind, par, tracks)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-60.0, 60.0, (3, n))
    u = isotropic(rng, n)
    return BOX, SUITE_SHAPES[BOX].copy(), pack_tracks(p[0], p[1], p[2], *u)


def segment_range(kind, par):
    """(phi1, dphi) of a tube or cone segment's or polycone's parameters
    (padded or not)."""
    par = np.asarray(par, np.float64).reshape(-1)
    if kind == PCON:
        return float(par[0]), float(par[1])
    return (float(par[3]), float(par[4])) if kind == TUBS else (float(par[5]), float(par[6]))


def _sample_profile(rng, z, rin, rout, n):
    """(r, z) uniform in the volume of revolution of a piecewise-linear
    profile: z by acceptance on the cross-section pi (ro^2 - ri^2) against
    the bound max(rout)^2, then r^2 uniform in the annulus."""
    zs = [np.zeros(0)]
    need = n
    bound = float(np.max(rout)) ** 2
    while need > 0:
        m = 2 * need + 64
        zz = rng.uniform(z[0], z[-1], m)
        ri, ro = np.interp(zz, z, rin), np.interp(zz, z, rout)
        acc = rng.uniform(0.0, bound, m) < (ro * ro - ri * ri)
        zs.append(zz[acc][:need])
        need -= zs[-1].size
    zz = np.concatenate(zs)
    ri, ro = np.interp(zz, z, rin), np.interp(zz, z, rout)
    return np.sqrt(rng.uniform(ri * ri, ro * ro)), zz


def _sample_in_shape(rng, kind, par, n):
    """Points uniformly distributed in the shape's volume, by construction
    (not by a membership test). Segments draw the azimuth in their range."""
    par = np.asarray(par, np.float64).reshape(-1)
    if kind == BOX:
        return [rng.uniform(-par[i], par[i], n) for i in range(3)]
    if kind in (TUBE, TUBS):
        rmin, rmax, dz = par[0], par[1], par[2]
        z = rng.uniform(-dz, dz, n)
        r = np.sqrt(rng.uniform(rmin * rmin, rmax * rmax, n))
        ph = rng.uniform(0.0, 2.0 * np.pi, n) if kind == TUBE else par[3] + rng.uniform(0.0, par[4], n)
        return [r * np.cos(ph), r * np.sin(ph), z]
    if kind in (CONE, CONS):
        dz, rmin1, rmax1, rmin2, rmax2 = par[:5]
        # Radii vary linearly between the end faces; the cross-section area
        # pi (ro^2 - ri^2) sets the z density. Sample z by acceptance against
        # the bound max(rmax1, rmax2)^2, then r^2 uniform in the annulus.
        zs = [np.zeros(0)]
        need = n
        bound = max(rmax1, rmax2) ** 2
        while need > 0:
            m = 2 * need + 64
            z = rng.uniform(-dz, dz, m)
            f = (z + dz) / (2.0 * dz)
            ro = rmax1 + (rmax2 - rmax1) * f
            ri = rmin1 + (rmin2 - rmin1) * f
            acc = rng.uniform(0.0, bound, m) < (ro * ro - ri * ri)
            zs.append(z[acc][:need])
            need -= zs[-1].size
        z = np.concatenate(zs)
        f = (z + dz) / (2.0 * dz)
        ro = rmax1 + (rmax2 - rmax1) * f
        ri = rmin1 + (rmin2 - rmin1) * f
        r = np.sqrt(rng.uniform(ri * ri, ro * ro))
        ph = rng.uniform(0.0, 2.0 * np.pi, n) if kind == CONE else par[5] + rng.uniform(0.0, par[6], n)
        return [r * np.cos(ph), r * np.sin(ph), z]
    if kind == PCON:
        r, z = _sample_profile(rng, *pcon_planes(par), n)
        ph = par[0] + rng.uniform(0.0, min(par[1], 2.0 * np.pi), n)
        return [r * np.cos(ph), r * np.sin(ph), z]
    raise ValueError(kind)


def shape_suite_c1(kind: int, n: int = 1 << 20, seed: int | None = None, par=None):
    """Shape-suite workload for one shape (SUITE_SHAPES[kind] unless `par` is
    given): half the origins drawn inside the shape, half uniform in the cube
    of half-size 50 around it (that half is not filtered, so a few percent of
    it also lands inside), randomly interleaved, isotropic directions.
    Returns (kind, par, tracks)."""
    if seed is None:
        seed = 1100 + kind
    rng = np.random.default_rng(seed)
    par = (SUITE_SHAPES[kind] if par is None else np.asarray(par, np.float64)).copy()
    n_in = n // 2
    n_out = n - n_in
    pin = _sample_in_shape(rng, kind, par, n_in)
    pout = rng.uniform(-50.0, 50.0, (3, n_out))
    p = np.concatenate([np.stack(pin), pout], axis=1)
    perm = rng.permutation(n)
    p = p[:, perm]
    u = isotropic(rng, n)
    return kind, par, pack_tracks(p[0], p[1], p[2], *u)


# ----------------------------------------------------------------------------
# Detector volumes
# ----------------------------------------------------------------------------

def euler_zxz(phi, theta, psi) -> np.ndarray:
    """R = Rz(phi) Rx(theta) Rz(psi), row-major 9 values."""
    def rz(a):
        c, s = np.cos(a), np.sin(a)
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])

    def rx(a):
        c, s = np.cos(a), np.sin(a)
        return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])

    return (rz(phi) @ rx(theta) @ rz(psi)).reshape(9)


def _draw_daughter(rng, kind):
    """Sizes uniform in [5, 20]; inner radii U[0, 0.75] * outer, set to 0
    with probability 1/4. Returns (par, bounding radius about the centre)."""
    if kind == BOX:
        d = rng.uniform(5.0, 20.0, 3)
        return np.array([d[0], d[1], d[2], 0.0, 0.0, 0.0, 0.0]), float(np.sqrt((d * d).sum()))

    def inner(rmax):
        r = rng.uniform(0.0, 0.75) * rmax
        return 0.0 if rng.uniform() < 0.25 else r

    if kind == TUBE:
        rmax = rng.uniform(5.0, 20.0)
        dz = rng.uniform(5.0, 20.0)
        rmin = inner(rmax)
        return np.array([rmin, rmax, dz, 0.0, 0.0]), float(np.hypot(rmax, dz))
    if kind == CONE:
        dz = rng.uniform(5.0, 20.0)
        rmax1 = rng.uniform(5.0, 20.0)
        rmax2 = rng.uniform(5.0, 20.0)
        rmin1 = inner(rmax1)
        rmin2 = inner(rmax2)
        return (np.array([dz, rmin1, rmax1, rmin2, rmax2]),
                float(np.hypot(max(rmax1, rmax2), dz)))
    if kind in (TUBS, CONS):
        # the base drawn as above, cut to phi1 ~ U[0, 2 pi), dphi ~ U[0.3, 2 pi - 0.3]
        par, rb = _draw_daughter(rng, TUBE if kind == TUBS else CONE)
        ang = [rng.uniform(0.0, 2 * np.pi), rng.uniform(0.3, 2 * np.pi - 0.3)]
        return np.concatenate([par[:3] if kind == TUBS else par[:5], ang]), rb
    if kind == PCON:
        # 3..6 planes over [-dz, dz] at least 0.5 apart; radii per plane as
        # above; cut to a random range with probability 1/2
        nz = int(rng.integers(3, 7))
        dz = rng.uniform(5.0, 20.0)
        while True:
            z = np.concatenate([[-dz], np.sort(rng.uniform(-dz, dz, nz - 2)), [dz]])
            if np.all(np.diff(z) >= 0.5):
                break
        rout = rng.uniform(5.0, 20.0, nz)
        rin = np.array([inner(r) for r in rout])
        if rng.uniform() < 0.5:
            phi1, dphi = rng.uniform(0.0, 2 * np.pi), rng.uniform(0.3, 2 * np.pi - 0.3)
        else:
            phi1, dphi = 0.0, 2 * np.pi
        return pcon_par(phi1, dphi, list(zip(z, rin, rout))), float(np.hypot(rout.max(), dz))
    raise ValueError(kind)


def _place_daughters(rng, centres, cell_half, kind_cycle=(BOX, TUBE, CONE)):
    nd = len(centres)
    kinds = np.array([kind_cycle[i % len(kind_cycle)] for i in range(nd)], np.int32)
    pars = np.zeros((nd, NPAR))
    rots = np.zeros((nd, 9))
    trs = np.zeros((nd, 3))
    bound = np.zeros(nd)
    for i in range(nd):
        par, rb = _draw_daughter(rng, int(kinds[i]))
        ang = rng.uniform(0.0, 1.0, 3) * np.array([2 * np.pi, np.pi, 2 * np.pi])
        jit = cell_half - rb
        assert jit > 0.0
        pars[i, :par.size] = par
        rots[i] = euler_zxz(*ang)
        trs[i] = np.asarray(centres[i], float) + rng.uniform(-jit, jit, 3)
        bound[i] = rb
    return kinds, pars, rots, trs, bound


def toy_detector_volume(seed: int = 1200) -> Volume:
    """Mother box (200, 200, 200) holding 32 daughters on a 4 x 4 x 2 grid of
    cells (x, y centres at +-50, +-150; z centres at +-100). Daughter i has
    kind i mod 3, a ZXZ rotation with uniformly drawn Euler angles and a
    jittered cell-centre translation. Each daughter's bounding sphere stays
    inside its 100-wide cell, so daughters cannot overlap."""
    rng = np.random.default_rng(seed)
    cs = [-150.0, -50.0, 50.0, 150.0]
    centres = [(x, y, z) for z in (-100.0, 100.0) for y in cs for x in cs]
    kinds, pars, rots, trs, bound = _place_daughters(rng, centres, 50.0)
    return Volume(BOX, np.array([MOTHER_HALF] * 3 + [0.0, 0.0]), kinds, pars, rots, trs, bound)


def mixed_detector_volume(seed: int = 1250) -> Volume:
    """The toy detector's layout (mother box (200)^3, 32 daughters on the
    4 x 4 x 2 grid of cells) with daughter i of kind i mod 6: box, tube,
    cone, tube segment, cone segment, polycone; segments cut to
    phi1 ~ U[0, 2 pi), dphi ~ U[0.3, 2 pi - 0.3] (convex and non-convex
    ranges); polycones of 3..6 planes, half of them cut likewise."""
    rng = np.random.default_rng(seed)
    cs = [-150.0, -50.0, 50.0, 150.0]
    centres = [(x, y, z) for z in (-100.0, 100.0) for y in cs for x in cs]
    kinds, pars, rots, trs, bound = _place_daughters(rng, centres, 50.0,
                                                     (BOX, TUBE, CONE, TUBS, CONS, PCON))
    return Volume(BOX, np.array([MOTHER_HALF] * 3 + [0.0, 0.0]), kinds, pars, rots, trs, bound)


def grid_volume(rng, nd: int) -> Volume:
    """Mother box (200)^3 with nd daughters in distinct, randomly chosen cells
    of a 4 x 4 x 4 grid of 100-wide cells, drawn as in the toy detector."""
    cs = [-150.0, -50.0, 50.0, 150.0]
    cells = [(x, y, z) for z in cs for y in cs for x in cs]
    pick = rng.choice(len(cells), size=nd, replace=False)
    centres = [cells[i] for i in pick]
    kinds, pars, rots, trs, bound = _place_daughters(rng, centres, 50.0)
    return Volume(BOX, np.array([MOTHER_HALF] * 3 + [0.0, 0.0]), kinds, pars, rots, trs, bound)


def tracks_in_mother(rng, vol: Volume, n: int) -> np.ndarray:
    """n tracks uniform in the box mother, outside every daughter: an origin
    is redrawn when it falls in a daughter's bounding sphere (the sphere the
    placement above keeps inside the daughter's cell). Isotropic directions."""
    h = vol.mother_par[:3]
    out = np.empty((3, 0))
    need = n
    while need > 0:
        m = int(need * 1.15) + 1024
        p = rng.uniform(-1.0, 1.0, (3, m)) * h[:, None]
        ok = np.ones(m, bool)
        for k in range(vol.nd):
            d = p - vol.trs[k][:, None]
            ok &= (d * d).sum(axis=0) > vol.bound_r[k] ** 2
        p = p[:, ok][:, :need]
        out = np.concatenate([out, p], axis=1)
        need = n - out.shape[1]
    u = isotropic(rng, n)
    return pack_tracks(out[0], out[1], out[2], *u)


def tracks_uniform_in_mother(rng, vol: Volume, n: int) -> np.ndarray:
    """n tracks uniform in the box mother with no rejection at all (origins
    fill the daughters too, and come arbitrarily close to their surfaces);
    isotropic directions. A track that starts inside a daughter has step 0
    and that daughter as its hit."""
    h = np.asarray(vol.mother_par, np.float64)[:3]
    p = rng.uniform(-1.0, 1.0, (3, n)) * h[:, None]
    u = isotropic(rng, n)
    return pack_tracks(p[0], p[1], p[2], *u)


def toy_detector_c2(seed: int = 1200, n: int = 1 << 22):
    """Toy-detector navigator workload: the 32-daughter volume and n tracks.
    Returns (volume, tracks)."""
    vol = toy_detector_volume(seed)
    rng = np.random.default_rng(seed + 1)
    return vol, tracks_in_mother(rng, vol, n)


@dataclass
class BatchedWorkload:
    volumes: list            # list[Volume]
    basket_volume: np.ndarray  # (nb,) int32
    basket_offset: np.ndarray  # (nb,) int64, into the track pool
    basket_n: np.ndarray       # (nb,) int64
    tracks: np.ndarray         # (6, sum n) pool


def batched_c3(seed: int = 1300, nvol: int = 64, nb: int = 512,
               nmin: int = 32, nmax: int = 65536, scale: float = 1.0,
               reject: bool = True) -> BatchedWorkload:
    """Batched workload: nvol volumes (mother box (200)^3, 1..64 daughters
    each, uniform), nb baskets with volume = b mod nvol and size
    floor(nmin * (nmax / nmin)^u), u ~ U[0, 1) (log-uniform). The track pool
    is the concatenation of the baskets. ``scale`` shrinks every basket
    (at least one track) for small test cases. With ``reject`` False the
    tracks are uniform in the mother with no rejection
    (``tracks_uniform_in_mother``); the geometry and basket sizes are the
    same."""
    rng = np.random.default_rng(seed)
    vols = []
    for _ in range(nvol):
        nd = int(rng.integers(1, 65))
        vols.append(grid_volume(rng, nd))
    u = rng.uniform(0.0, 1.0, nb)
    sizes = np.floor(nmin * (nmax / nmin) ** u).astype(np.int64)
    if scale != 1.0:
        sizes = np.maximum(1, np.floor(sizes * scale).astype(np.int64))
    bvol = (np.arange(nb) % nvol).astype(np.int32)
    offs = np.zeros(nb, np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    parts = []
    for b in range(nb):
        draw = tracks_in_mother if reject else tracks_uniform_in_mother
        parts.append(draw(rng, vols[bvol[b]], int(sizes[b])))
    pool = np.ascontiguousarray(np.concatenate(parts, axis=1))
    return BatchedWorkload(vols, bvol, offs, sizes, pool)


def adjoint_c4(seed: int = 1400, n: int = 1 << 20, detector_seed: int = 1200):
    """Adjoint workload: the toy detector (same geometry as the navigator
    workload), n tracks, and target points uniform in the mother.
    Returns (volume, tracks, targets (3, n))."""
    vol = toy_detector_volume(detector_seed)
    rng = np.random.default_rng(seed)
    tracks = tracks_in_mother(rng, vol, n)
    rng_t = np.random.default_rng(seed + 1)
    targets = np.ascontiguousarray(rng_t.uniform(-MOTHER_HALF, MOTHER_HALF, (3, n)))
    return vol, tracks, targets


# ----------------------------------------------------------------------------
# The paper's toy detector (section 3.2): a tubular mother holding two tubes
# (beampipe, shield), four boxes (detector plates) and two cones (endcaps).
# The paper gives its composition but no dimensions; the ones below are this
# project's choice, non-overlapping by construction.
# ----------------------------------------------------------------------------

PAPER_MOTHER = np.array([0.0, 100.0, 200.0, 0.0, 0.0])      # tube rmin, rmax, dz


def paper_toy_detector() -> Volume:
    """Tube mother (0, 100, 200) with
      beampipe tube (3, 4, 180) and shield tube (40, 45, 150) on the axis,
      four plates: boxes (5, 20, 100) at radius 70 on the x and y axes
        (the y ones turned by 90 degrees about z),
      two endcaps: cones (dz 10; rmin 5 -> 5, rmax 50 -> 90) at z = +170 and,
        turned by 180 degrees about x, at z = -170.
    Radial layout: beampipe r <= 4, shield 40..45, plates 65..77.7,
    endcaps 5..90 for 160 <= |z| <= 180; the shield ends at |z| = 150 and the
    plates at |z| = 100."""
    kinds = np.array([TUBE, TUBE, BOX, BOX, BOX, BOX, CONE, CONE], np.int32)
    pars = np.array([
        [3.0, 4.0, 180.0, 0.0, 0.0],
        [40.0, 45.0, 150.0, 0.0, 0.0],
        [5.0, 20.0, 100.0, 0.0, 0.0],
        [5.0, 20.0, 100.0, 0.0, 0.0],
        [5.0, 20.0, 100.0, 0.0, 0.0],
        [5.0, 20.0, 100.0, 0.0, 0.0],
        [10.0, 5.0, 50.0, 5.0, 90.0],
        [10.0, 5.0, 50.0, 5.0, 90.0],
    ])
    rz90 = euler_zxz(np.pi / 2, 0.0, 0.0)
    rx180 = euler_zxz(0.0, np.pi, 0.0)
    eye = np.eye(3).reshape(9)
    rots = np.stack([eye, eye, eye, eye, rz90, rz90, eye, rx180])
    trs = np.array([
        [0.0, 0.0, 0.0], [0.0, 0.0, 0.0],
        [70.0, 0.0, 0.0], [-70.0, 0.0, 0.0], [0.0, 70.0, 0.0], [0.0, -70.0, 0.0],
        [0.0, 0.0, 170.0], [0.0, 0.0, -170.0],
    ])
    bound = np.array([np.hypot(4.0, 180.0), np.hypot(45.0, 150.0)] +
                     [float(np.sqrt(5.0 ** 2 + 20.0 ** 2 + 100.0 ** 2))] * 4 +
                     [float(np.hypot(90.0, 10.0))] * 2)
    return Volume(TUBE, PAPER_MOTHER.copy(), kinds, pars, rots, trs, bound)


def _cyl_shell(rng, n, r0, r1, z0, z1):
    """n points uniform in {r0 <= r <= r1, z0 <= z <= z1} (cylindrical shell)."""
    r = np.sqrt(rng.uniform(r0 * r0, r1 * r1, n))
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    z = rng.uniform(z0, z1, n)
    return np.stack([r * np.cos(ph), r * np.sin(ph), z])


def paper_toy_tracks(seed: int = 1500, n: int = 1 << 20) -> np.ndarray:
    """Tracks in the mother's exclusive part (outside every daughter), drawn
    from cylindrical regions that are empty by construction of
    paper_toy_detector(), each with probability proportional to its volume:
      5 <= r <= 39,  |z| <= 150      between beampipe and shield
      46 <= r <= 64, |z| <= 150      between shield and plates
      78 <= r <= 99, |z| <= 150      outside the plates
      5 <= r <= 99, 151 <= |z| <= 159 between shield end and endcaps
      5 <= r <= 99, 181 <= |z| <= 199 beyond the endcaps
    Isotropic directions. (The thin regions next to each daughter are left
    out, so origins stay at least 1 unit from every daughter.)"""
    rng = np.random.default_rng(seed)
    regions = [(5.0, 39.0, -150.0, 150.0), (46.0, 64.0, -150.0, 150.0), (78.0, 99.0, -150.0, 150.0),
               (5.0, 99.0, 151.0, 159.0), (5.0, 99.0, -159.0, -151.0),
               (5.0, 99.0, 181.0, 199.0), (5.0, 99.0, -199.0, -181.0)]
    vol = np.array([(r1 * r1 - r0 * r0) * (z1 - z0) for r0, r1, z0, z1 in regions])
    counts = rng.multinomial(n, vol / vol.sum())
    pts = np.concatenate([_cyl_shell(rng, c, *reg) for c, reg in zip(counts, regions)], axis=1)
    pts = pts[:, rng.permutation(n)]
    u = isotropic(rng, n)
    return pack_tracks(pts[0], pts[1], pts[2], *u)
