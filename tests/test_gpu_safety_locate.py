"""Parity of the navigator's isotropic safety (geo_navigate_safety) and of
localization (geo_locate) with the oracle."""
import numpy as np
import pytest

from paper_1312_0816_amd import workloads as W
from tests.parity import check_values, rel_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gv():
    import torch
    from paper_1312_0816_amd import geonav
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    geonav.load_library()
    return geonav


def _points(vol, n, seed):
    """Points of three kinds: the mother's own part, inside daughters (by
    construction) and outside the mother."""
    rng = np.random.default_rng(seed)
    own = W.tracks_in_mother(rng, vol, n)[:3] if vol.mother_kind == W.BOX else rng.uniform(-150, 150, (3, n))
    ins = []
    for k in range(vol.nd):
        q = np.stack(W._sample_in_shape(rng, int(vol.kinds[k]), vol.pars[k], 40))
        ins.append(vol.rots[k].reshape(3, 3) @ q + vol.trs[k][:, None])
    far = rng.uniform(-450, 450, (3, 300))
    return np.ascontiguousarray(np.concatenate([own] + ins + [far], axis=1))


@pytest.mark.parametrize("offsets", [False, True])
def test_safety_and_locate_toy_detector(gv, orc, offsets):
    import torch
    vol = W.toy_detector_volume()
    p = _points(vol, 20000, 31)
    offs = np.random.default_rng(1).uniform(-2, 2, (vol.nd, 3)) if offsets else None
    g = gv.Geometry([vol])
    tp = torch.from_numpy(p).cuda()
    to = None if offs is None else torch.from_numpy(offs).cuda()
    s = gv.geo_navigate_safety(g, 0, tp, to).cpu().numpy()
    w = gv.geo_locate(g, 0, tp, to).cpu().numpy()
    ref = orc.navigate_safety(vol, p, offs, "ld")
    ill = rel_diff(orc.navigate_safety(vol, p, offs, "d"), ref) > 1e-13
    print(check_values(s, ref, ill, "navigator safety"))
    rw = orc.locate(vol, p, offs, "ld")
    near = ref < 1e-9
    assert np.array_equal(w[~near], rw[~near])
    assert {-2, -1} <= set(np.unique(w)) and len(np.unique(w)) == vol.nd + 2
    # culling on and off give identical bits
    g.culling = False
    s2 = gv.geo_navigate_safety(g, 0, tp, to).cpu().numpy()
    w2 = gv.geo_locate(g, 0, tp, to).cpu().numpy()
    assert np.array_equal(s.view(np.int64), s2.view(np.int64)) and np.array_equal(w, w2)
    g.close()


def test_safety_and_locate_other_volumes(gv, orc):
    import torch
    for vol in (W.paper_toy_detector(), W.Volume(W.CONE, np.array([250.0, 10.0, 200.0, 30.0, 350.0]))):
        p = _points(vol, 5000, 3)
        g = gv.Geometry([vol])
        tp = torch.from_numpy(p).cuda()
        s = gv.geo_navigate_safety(g, 0, tp).cpu().numpy()
        w = gv.geo_locate(g, 0, tp).cpu().numpy()
        ref = orc.navigate_safety(vol, p, None, "ld")
        ill = rel_diff(orc.navigate_safety(vol, p, None, "d"), ref) > 1e-13
        check_values(s, ref, ill, "safety other volume")
        near = ref < 1e-9
        assert np.array_equal(w[~near], orc.locate(vol, p, None, "ld")[~near])
        g.close()


def test_empty_and_errors(gv):
    import torch
    g = gv.Geometry([W.toy_detector_volume()])
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    assert gv.geo_navigate_safety(g, 0, e).numel() == 0
    assert gv.geo_locate(g, 0, e).numel() == 0
    with pytest.raises(gv.GeoError):
        gv.geo_locate(g, 5, torch.zeros((3, 4), dtype=torch.float64, device="cuda"))
    g.close()


@pytest.mark.parametrize("offsets", [False, True])
def test_large_point_sets(gv, orc, offsets):
    """2^20 + 37 points: culling on and off give identical bits, and 6000
    sampled points match the oracle."""
    import torch
    vol = W.toy_detector_volume()
    rng = np.random.default_rng(33)
    n = (1 << 20) + 37
    extra = _points(vol, 12000, 34)  # inside daughters and outside the mother too
    p = np.ascontiguousarray(np.concatenate([W.tracks_in_mother(rng, vol, n - extra.shape[1])[:3],
                                             extra], axis=1))
    p = np.ascontiguousarray(p[:, rng.permutation(p.shape[1])])
    offs = rng.uniform(-2, 2, (vol.nd, 3)) if offsets else None
    g = gv.Geometry([vol])
    tp = torch.from_numpy(p).cuda()
    to = None if offs is None else torch.from_numpy(offs).cuda()
    s = gv.geo_navigate_safety(g, 0, tp, to).cpu().numpy()
    w = gv.geo_locate(g, 0, tp, to).cpu().numpy()
    g.culling = False
    s2 = gv.geo_navigate_safety(g, 0, tp, to).cpu().numpy()
    w2 = gv.geo_locate(g, 0, tp, to).cpu().numpy()
    g.close()
    assert np.array_equal(s.view(np.int64), s2.view(np.int64)) and np.array_equal(w, w2)
    idx = np.sort(rng.choice(p.shape[1], 6000, replace=False))
    ps = np.ascontiguousarray(p[:, idx])
    ref = orc.navigate_safety(vol, ps, offs, "ld")
    ill = rel_diff(orc.navigate_safety(vol, ps, offs, "d"), ref) > 1e-13
    print(check_values(s[idx], ref, ill, "large safety"))
    near = ref < 1e-9
    assert np.array_equal(w[idx][~near], orc.locate(vol, ps, offs, "ld")[~near])
