"""The compacted navigator (culling tests queue (track, daughter) pairs that
are then evaluated one per lane) against the sequential loop it replaces
and against the oracle, on geometries built to stress it: a line of 150
daughters that every track of a wavefront needs (the queue fills and is
flushed many times per round), equal steps to two touching daughters whose
pairs land in different flushes (the lower index must win, as in the
sequential loop), and tracks starting on a daughter's surface (step 0)."""
import numpy as np
import pytest

from paper_1312_0816_amd import workloads as W
from tests.test_gpu_navigator import check_nav

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gv():
    import torch
    from paper_1312_0816_amd import geonav
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    geonav.load_library()
    return geonav


def _bits(a):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    return a.view(np.int64) if a.dtype == np.float64 else a


def _volume(mother_half, centres, halves):
    """Box mother with axis-aligned box daughters."""
    nd = len(centres)
    pars = np.zeros((nd, W.NPAR))
    pars[:, :3] = halves
    rots = np.tile(np.eye(3).reshape(9), (nd, 1))
    return W.Volume(W.BOX, np.array(list(mother_half) + [0.0, 0.0]),
                    np.full(nd, W.BOX, np.int32), pars, rots,
                    np.asarray(centres, np.float64), np.linalg.norm(halves, axis=1))


def _line_volume():
    """150 boxes of half size (1, 5, 5) every 4 units along x."""
    centres = [(-300.0 + 4.0 * i, 0.0, 0.0) for i in range(150)]
    return _volume((400.0, 20.0, 20.0), centres, np.tile([1.0, 5.0, 5.0], (150, 1)))


def _line_tracks(rng, n):
    """Tracks near the line, mostly along +x or -x, some isotropic."""
    o = np.stack([rng.uniform(-390, 390, n), rng.uniform(-3, 3, n), rng.uniform(-3, 3, n)])
    d = np.stack(W.isotropic(rng, n))
    along = rng.uniform(size=n) < 0.8
    a = rng.normal(0, 0.01, (2, n))
    s = np.where(rng.uniform(size=n) < 0.5, 1.0, -1.0)
    d_al = np.stack([s, a[0], a[1]])
    d_al /= np.linalg.norm(d_al, axis=0)
    d = np.where(along[None, :], d_al, d)
    t = np.ascontiguousarray(np.concatenate([o, d]))
    # start outside every daughter: push origins in a daughter's slab to a gap
    x = t[0]
    cell = np.round((x + 300.0) / 4.0)
    inside = (np.abs(x - (-300.0 + 4.0 * cell)) <= 1.0) & (cell >= 0) & (cell < 150)
    t[0, inside] = -300.0 + 4.0 * cell[inside] + 2.0
    return t


EVERY_KIND = (W.BOX, W.TUBE, W.CONE, W.TUBS, W.CONS, W.PCON)


def _mixed_line_volume(seed, nd=24, kinds=EVERY_KIND):
    """nd daughters of the given kinds in turn (by default every kind: box,
    tube, cone, their segments, polycones) in a row of 100-wide cells along
    x, mother box (50 nd + 10, 60, 60)."""
    rng = np.random.default_rng(seed)
    centres = [(-50.0 * (nd - 1) + 100.0 * i, 0.0, 0.0) for i in range(nd)]
    kinds, pars, rots, trs, bound = W._place_daughters(rng, centres, 50.0, kinds)
    return W.Volume(W.BOX, np.array([50.0 * nd + 10.0, 60.0, 60.0, 0.0, 0.0]), kinds, pars, rots, trs,
                    bound)


def _mixed_line_tracks(rng, vol, n, dense_frac=0.4):
    """A fraction of the tracks near the row's axis, along +x or -x (each
    passes the culling spheres of the daughters ahead of it), starting
    outside every bounding sphere; the rest off the row (|y| in [52, 58])
    moving away from it, which queue nothing."""
    hx = vol.mother_par[0] - 1.0
    dense = rng.uniform(size=n) < dense_frac
    m = int(dense.sum())
    x = rng.uniform(-hx, hx, m)
    yz = rng.uniform(-3.0, 3.0, (2, m))
    for _ in range(100):
        p = np.stack([x, yz[0], yz[1]])
        ins = np.zeros(m, bool)
        for k in range(vol.nd):
            ins |= np.linalg.norm(p - vol.trs[k][:, None], axis=0) < vol.bound_r[k]
        if not ins.any():
            break
        x[ins] = rng.uniform(-hx, hx, int(ins.sum()))
    assert not ins.any()
    sgn = np.where(rng.uniform(size=m) < 0.5, 1.0, -1.0)
    dd = np.stack([sgn, rng.normal(0, 0.01, m), rng.normal(0, 0.01, m)])
    tr = np.zeros((6, n))
    tr[:3, dense] = np.stack([x, yz[0], yz[1]])
    tr[3:, dense] = dd / np.linalg.norm(dd, axis=0)
    k = n - m
    sy = np.where(rng.uniform(size=k) < 0.5, 1.0, -1.0)
    tr[:3, ~dense] = np.stack([rng.uniform(-hx, hx, k), sy * rng.uniform(52, 58, k), rng.uniform(-40, 40, k)])
    dd = np.stack([rng.normal(0, 0.3, k), sy, rng.normal(0, 0.3, k)])
    tr[3:, ~dense] = dd / np.linalg.norm(dd, axis=0)
    return np.ascontiguousarray(tr)


def _all_paths(gv, vols, tr, offsets=None):
    """(step, hit) from the basket navigator with culling (compacted) and
    without (sequential), and from the batched navigator at every launch
    shape; all must agree bit for bit. Returns the compacted result."""
    import torch
    g = gv.Geometry(vols)
    t = torch.from_numpy(tr).cuda()
    o = None if offsets is None else torch.from_numpy(np.ascontiguousarray(offsets)).cuda()
    out = {}
    for cull in (True, False):
        g.culling = cull
        s, h, hp = gv.geo_navigate_basket(g, 0, t, offsets=o, hitpt=True)
        out[cull] = (_bits(s), _bits(h), _bits(hp))
    for a, b in zip(out[True], out[False]):
        assert np.array_equal(a, b)
    if offsets is None:
        n = tr.shape[1]
        g.culling = True
        for u, w in ((1, 0), (2, 0), (4, 0), (8, 0), (4, 2)):
            g.set_launch_config(u, w)
            sb, hb = gv.geo_navigate_batched(g, [0, 0], [0, n // 3], [n // 3, n - n // 3], t)
            assert np.array_equal(_bits(sb), out[True][0]), (u, w)
            assert np.array_equal(_bits(hb), out[True][1]), (u, w)
    g.close()
    return out[True][0].view(np.float64), out[True][1]


def test_queue_overflow_line_of_daughters(gv, orc):
    vol = _line_volume()
    tr = _line_tracks(np.random.default_rng(1700), 3000)
    step, hit = _all_paths(gv, [vol], tr)
    # tracks nearly parallel to the boxes' y and z faces meet them at grazing
    # incidence, which the oracle's double/long double comparison flags
    print(check_nav(orc, vol, tr, step, hit, what="line of 150", max_exempt_frac=0.02))
    assert (hit >= 0).mean() > 0.7  # most tracks end on a daughter


def test_queue_overflow_with_offsets(gv, orc):
    vol = _line_volume()
    tr = _line_tracks(np.random.default_rng(1701), 2000)
    offs = np.random.default_rng(3).uniform(-0.4, 0.4, (vol.nd, 3))
    step, hit = _all_paths(gv, [vol], tr, offsets=offs)
    print(check_nav(orc, vol, tr, step, hit, offsets=offs, what="line of 150, offsets",
                    max_exempt_frac=0.02))


@pytest.mark.parametrize("a_first", [True, False])
def test_ties_across_flushes_take_the_lower_index(gv, a_first):
    """Boxes A (x in [-20, 0]) and B (x in [0, 20]) touch along x = 0; tracks
    in that plane moving +y from y = -100 reach both at t = 95 exactly. 100
    small boxes beyond them along the tracks sit between the two in index
    order, so the pairs of A and of B are evaluated in different flushes."""
    fill_c = [(0.0, 10.0 + 3.0 * i, 0.0) for i in range(100)]
    fill_h = np.tile([1.0, 1.0, 1.0], (100, 1))
    ab_c = [(-10.0, 0.0, 0.0), (10.0, 0.0, 0.0)]
    if not a_first:
        ab_c = ab_c[::-1]
    centres = [ab_c[0]] + fill_c + [ab_c[1]]
    halves = np.concatenate([[[10.0, 5.0, 5.0]], fill_h, [[10.0, 5.0, 5.0]]])
    vol = _volume((200.0, 400.0, 200.0), centres, halves)
    rng = np.random.default_rng(1702)
    n = 1000
    z = rng.uniform(-4, 4, n)
    # directions in the plane x = 0, aimed at the shared face's near edge
    aim_z = rng.uniform(-4.5, 4.5, n)
    d = np.stack([np.zeros(n), np.full(n, 95.0), aim_z - z])
    d /= np.linalg.norm(d, axis=0)
    tr = np.ascontiguousarray(np.stack([np.zeros(n), np.full(n, -100.0), z, d[0], d[1], d[2]]))
    step, hit = _all_paths(gv, [vol], tr)
    assert np.all(hit == 0)
    want = 95.0 / d[1]
    assert np.all(np.abs(step - want) <= 1e-12 * want)


def test_tracks_starting_on_a_daughter_surface(gv, orc):
    """Origins on a face of a daughter (closed sets: inside, DistFromOutside
    0): step +0 and that daughter's index, on every path."""
    vol = _line_volume()
    rng = np.random.default_rng(1703)
    n = 500
    k = rng.integers(0, 150, n)
    o = np.stack([-300.0 + 4.0 * k - 1.0, rng.uniform(-5, 5, n), rng.uniform(-5, 5, n)])
    d = np.stack(W.isotropic(rng, n))
    tr = np.ascontiguousarray(np.concatenate([o, d]))
    step, hit = _all_paths(gv, [vol], tr)
    assert np.all(step.view(np.int64) == 0)        # +0, not -0
    assert np.array_equal(hit, k.astype(np.int32))
    ref, rhit, _ = orc.navigate(vol, tr)
    assert np.all(ref == 0) and np.array_equal(rhit, k)


def test_tangent_to_culling_spheres_in_a_large_mother(gv, orc):
    """A mother of half size 10^4 with 40 small, rotated daughters near its
    corners (|T| up to 1.6e4, bounding radii 1-4): tracks from random origins
    along lines tangent to a daughter's bounding sphere, or passing just
    inside or outside it, where the expanded culling test's rounding
    matters most. Culling on (compacted) and off (sequential) must agree bit
    for bit, and with the oracle."""
    rng = np.random.default_rng(1704)
    nd = 40
    sign = rng.choice([-1.0, 1.0], (nd, 3))
    centres = sign * rng.uniform(7000, 9500, (nd, 3))
    halves = rng.uniform(0.5, 2.0, (nd, 3))
    vol = _volume((1.0e4, 1.0e4, 1.0e4), centres, halves)
    ang = rng.uniform(0, 2 * np.pi, (nd, 3))
    vol.rots = np.stack([W.euler_zxz(*a).reshape(9) for a in ang])
    n = 4000
    k = rng.integers(0, nd, n)
    o = rng.uniform(-9000, 9000, (3, n))
    T = centres[k].T
    r = np.linalg.norm(halves[k], axis=1)
    a = T - o
    a /= np.linalg.norm(a, axis=0)
    perp = np.cross(a.T, rng.normal(size=(n, 3))).T
    perp /= np.linalg.norm(perp, axis=0)
    scale = rng.choice([1.0, 1.0 - 1e-7, 1.0 + 1e-7, 0.5], n)
    target = T + perp * (r * scale)
    d = target - o
    d /= np.linalg.norm(d, axis=0)
    tr = np.ascontiguousarray(np.concatenate([o, d]))
    step, hit = _all_paths(gv, [vol], tr)
    print(check_nav(orc, vol, tr, step, hit, what="tangent lines, large mother"))
    assert (hit >= 0).any()


def test_the_largest_volume(gv, orc):
    """A volume with the most daughters the library accepts (1024 boxes on a
    16 x 16 x 4 grid): basket and batched navigation with culling on and
    off, safety and localization on and off, the adjoint on and off with
    daughter offsets up to 1 in each coordinate (its offset-gradient sort
    holds 1024 bins; the culled forward tests 1024 shifted culling
    records), and the oracle on a sample."""
    import torch
    n_d = gv.GEO_MAX_DAUGHTERS
    ii = np.arange(n_d)
    centres = np.stack([-150.0 + 20.0 * (ii % 16), -150.0 + 20.0 * ((ii // 16) % 16),
                        -60.0 + 40.0 * (ii // 256)], axis=1)
    rng = np.random.default_rng(1705)
    halves = rng.uniform(2.0, 8.0, (n_d, 3))
    vol = _volume((200.0, 200.0, 200.0), centres, halves)
    tr = W.tracks_in_mother(rng, vol, 20000)
    step, hit = _all_paths(gv, [vol], tr)
    idx = np.sort(rng.choice(tr.shape[1], 3000, replace=False))
    print(check_nav(orc, vol, np.ascontiguousarray(tr[:, idx]), step[idx], hit[idx], what="1024 daughters"))
    assert len(np.unique(hit)) > 500
    g = gv.Geometry([vol])
    p = torch.from_numpy(np.ascontiguousarray(tr[:3])).cuda()
    d = torch.from_numpy(np.ascontiguousarray(tr[3:])).cuda()
    gh = torch.from_numpy(rng.normal(size=(3, tr.shape[1]))).cuda()
    offs = torch.from_numpy(rng.uniform(-1.0, 1.0, (n_d, 3))).cuda()
    out = {}
    for cull in (True, False):
        g.culling = cull
        s = gv.geo_navigate_safety(g, 0, p).cpu().numpy()
        w = gv.geo_locate(g, 0, p).cpu().numpy()
        go, gd, goff = gv.geo_navigate_backward(g, 0, p, d, offs, None, gh)
        out[cull] = [s.view(np.int64), w, _bits(go), _bits(gd), _bits(goff)]
    g.close()
    for a, b in zip(out[True], out[False]):
        assert np.array_equal(a, b)
    ps = np.ascontiguousarray(tr[:3, idx])
    ref = orc.navigate_safety(vol, ps, None, "d")
    assert np.all(np.abs(out[True][0].view(np.float64)[idx] - ref) <= 1e-12 * np.maximum(ref, 1.0))
    assert np.array_equal(out[True][1][idx], orc.locate(vol, ps, None, "d"))


@pytest.mark.parametrize("seed", range(6))
def test_random_mixed_detectors_bitwise(gv, seed):
    """Mixed detectors (all six kinds) from several seeds, with random
    offsets: every culled (compacted) path equals its sequential
    counterpart bit for bit: basket with hit points, batched at a random
    launch shape, safety, localization and the adjoint."""
    import torch
    rng = np.random.default_rng(1800 + seed)
    vols = [W.mixed_detector_volume(1250 + 10 * seed + i) for i in range(3)]
    sizes = [int(x) for x in rng.integers(1, 3000, 5)]
    parts, bv, bo, off = [], [], [], 0
    for b, m in enumerate(sizes):
        parts.append(W.tracks_in_mother(rng, vols[b % 3], m))
        bv.append(b % 3)
        bo.append(off)
        off += m
    tr = np.ascontiguousarray(np.concatenate(parts, axis=1))
    t = torch.from_numpy(tr).cuda()
    g = gv.Geometry(vols)
    u, w = [(1, 0), (2, 0), (4, 0), (8, 0), (2, 3), (4, 2)][seed]
    g.set_launch_config(u, w)
    v0 = vols[0]
    t0 = t[:, :sizes[0]].contiguous()
    offs = torch.from_numpy(rng.uniform(-1.5, 1.5, (v0.nd, 3))).cuda()
    gh = torch.from_numpy(rng.normal(size=(3, sizes[0]))).cuda()
    out = {}
    for cull in (True, False):
        g.culling = cull
        r = []
        r += [_bits(x) for x in gv.geo_navigate_basket(g, 0, t0, offsets=offs, hitpt=True)]
        r += [_bits(x) for x in gv.geo_navigate_batched(g, bv, bo, sizes, t)]
        r.append(_bits(gv.geo_navigate_safety(g, 0, t0[:3].contiguous(), offs)))
        r.append(_bits(gv.geo_locate(g, 0, t0[:3].contiguous(), offs)))
        o = t0[:3].contiguous()
        d = t0[3:].contiguous()
        r += [_bits(x) for x in gv.geo_navigate_backward(g, 0, o, d, offs, None, gh)]
        out[cull] = r
    g.close()
    for a, b in zip(out[True], out[False]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("mixed", [False, True])
def test_direction_length_over_the_supported_range(gv, orc, mixed):
    """Directions scaled by factors over the supported range, 1e-20 to
    1e100 (the culling test normalises d per track): every path agrees bit
    for bit, and the steps, ray parameters t = length / |d|, times the
    factor match the oracle's steps for the unscaled tracks."""
    vol = W.mixed_detector_volume() if mixed else W.toy_detector_volume()
    rng = np.random.default_rng(1500 + int(mixed))
    n = 3001
    tr = W.tracks_in_mother(rng, vol, n)
    scale = rng.choice([1e-20, 1e-8, 1.0, 1e8, 1e50, 1e100], n)
    ts = tr.copy()
    ts[3:] *= scale
    step, hit = _all_paths(gv, [vol], np.ascontiguousarray(ts))
    # the mixed detector's segments and polycones graze more often: 9 of
    # these 3001 tracks are ill-conditioned at 1e-12 (the oracle's double
    # and long double builds disagree)
    check_nav(orc, vol, tr, step * scale, hit, what=f"scaled directions, mixed={mixed}",
              max_exempt_frac=5e-3)


@pytest.mark.parametrize("n", [(1 << 16) + 37, (1 << 20) + 37])
@pytest.mark.parametrize("polycones", [True, False])
def test_dense_queues_of_every_kind(gv, orc, n, polycones):
    """A row of 24 daughters of every kind (or every kind but the polycone:
    the kernels for segments, five kind classes), 40 % of the tracks along
    it (about 1.9 queued pairs per track): the workgroups' pooled last
    flushes hold more than 64 pairs of one kind, and many wavefronts end
    with more than 128 queued pairs (flushed by the wavefront alone) or
    flush within the loop. One round of 64 tracks per wavefront at 2^16
    tracks, four at 2^20. Culled and sequential paths agree bit for bit, at
    every batched launch shape; a sample matches the oracle."""
    vol = _mixed_line_volume(1900, kinds=EVERY_KIND if polycones else EVERY_KIND[:5])
    rng = np.random.default_rng(1910)
    tr = _mixed_line_tracks(rng, vol, n)
    step, hit = _all_paths(gv, [vol], tr)
    idx = np.sort(rng.choice(n, size=4000, replace=False))
    print(check_nav(orc, vol, np.ascontiguousarray(tr[:, idx]), step[idx], hit[idx],
                    what=f"dense row of every kind, {n} tracks", max_exempt_frac=5e-3))
    assert (hit >= 0).mean() > 0.1  # the tracks along the row end on a daughter


@pytest.mark.parametrize("with_offsets", [False, True])
def test_wide_basket_of_every_kind(gv, orc, with_offsets):
    """A basket of 2^20 + 37 tracks in a volume holding every kind (the wide
    compacted form, 4 rounds of 64 tracks per wavefront): culled and
    sequential paths agree bit for bit, hit points included, with and
    without offsets; a sample matches the oracle."""
    vol = W.mixed_detector_volume()
    rng = np.random.default_rng(1601 + int(with_offsets))
    n = (1 << 20) + 37
    tr = W.tracks_in_mother(rng, vol, n)
    offs = rng.uniform(-0.5, 0.5, (vol.nd, 3)) if with_offsets else None
    step, hit = _all_paths(gv, [vol], tr, offs)
    idx = np.sort(rng.choice(n, size=4000, replace=False))
    print(check_nav(orc, vol, np.ascontiguousarray(tr[:, idx]), step[idx], hit[idx], offsets=offs,
                    what=f"wide basket, offsets={with_offsets}", max_exempt_frac=5e-3))
