"""Culling changes the work done, never the results: the navigators give
bit-identical outputs with culling on (compacted evaluation of the pairs
that pass) and off (every daughter evaluated in lockstep)."""
import numpy as np
import pytest

from paper_1312_0816_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gv():
    import torch
    from paper_1312_0816_amd import geonav
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    geonav.load_library()
    return geonav


def _bits(a):
    return a.cpu().numpy().view(np.uint64) if a.dtype.is_floating_point else a.cpu().numpy()


def test_basket_culling_bit_identical(gv):
    import torch
    vol, tr = W.toy_detector_c2()
    g = gv.Geometry([vol])
    assert g.culling
    t = torch.from_numpy(tr).cuda()
    offs = torch.from_numpy(np.random.default_rng(5).uniform(-2, 2, (vol.nd, 3))).cuda()
    res = {}
    for cull in (True, False):
        g.culling = cull
        res[cull] = [gv.geo_navigate_basket(g, 0, t), gv.geo_navigate_basket(g, 0, t, offsets=offs,
                                                                              hitpt=True)]
    torch.cuda.synchronize()
    for a, b in zip(res[True], res[False]):
        for x, y in zip(a, b):
            assert np.array_equal(_bits(x), _bits(y))
    g.close()


def test_batched_culling_bit_identical(gv):
    import torch
    wl = W.batched_c3()
    g = gv.Geometry(wl.volumes)
    t = torch.from_numpy(wl.tracks).cuda()
    out = {}
    for cull in (True, False):
        g.culling = cull
        s, h = gv.geo_navigate_batched(g, wl.basket_volume, wl.basket_offset, wl.basket_n, t)
        torch.cuda.synchronize()
        out[cull] = (_bits(s), _bits(h))
    assert np.array_equal(out[True][0], out[False][0])
    assert np.array_equal(out[True][1], out[False][1])
    g.close()


@pytest.mark.parametrize("shift", [0.0, 5.0])
def test_backward_culling_bit_identical(gv, shift):
    """The adjoint with culling on and off, with zero offsets and with
    offsets of up to 5 in each coordinate (the culled forward then tests
    the culling records moved by the offsets)."""
    import torch
    vol, tr, tgt = W.adjoint_c4(n=200000)
    g = gv.Geometry([vol])
    o = torch.from_numpy(np.ascontiguousarray(tr[:3])).cuda()
    d = torch.from_numpy(np.ascontiguousarray(tr[3:])).cuda()
    gh = torch.from_numpy(np.ascontiguousarray(tgt)).cuda()
    rng = np.random.default_rng(11)
    offs = torch.from_numpy(rng.uniform(-shift, shift, (vol.nd, 3))).cuda()
    out = {}
    for cull in (True, False):
        g.culling = cull
        out[cull] = [_bits(x) for x in gv.geo_navigate_backward(g, 0, o, d, offs, None, gh)]
    for a, b in zip(out[True], out[False]):
        assert np.array_equal(a, b)
    g.close()


def test_census_counts(gv):
    """The census variant returns the same outputs and consistent counts:
    every track counted once; without culling every (track, daughter) pair
    is one lane-evaluation; with culling fewer."""
    import torch
    wl = W.batched_c3(scale=0.05)
    g = gv.Geometry(wl.volumes)
    t = torch.from_numpy(wl.tracks).cuda()
    s0, h0 = gv.geo_navigate_batched(g, wl.basket_volume, wl.basket_offset, wl.basket_n, t)
    s1, h1, c_on = gv.geo_navigate_batched_census(g, wl.basket_volume, wl.basket_offset, wl.basket_n, t)
    g.culling = False
    s2, h2, c_off = gv.geo_navigate_batched_census(g, wl.basket_volume, wl.basket_offset, wl.basket_n, t)
    assert np.array_equal(_bits(s0), _bits(s1)) and np.array_equal(_bits(s0), _bits(s2))
    assert np.array_equal(_bits(h0), _bits(h1)) and np.array_equal(_bits(h0), _bits(h2))
    n = int(wl.basket_n.sum())
    pairs = int(sum(int(wl.basket_n[b]) * wl.volumes[int(wl.basket_volume[b])].nd
                    for b in range(len(wl.basket_n))))
    T, Q = gv.CENSUS_TRACKS, gv.CENSUS_CULL
    assert len(c_on) == gv.CENSUS_SLOTS
    assert c_on[T] == n and c_off[T] == n
    assert sum(c_off[:14]) == pairs and c_off[Q] == 0
    assert c_on[Q] == pairs and 0 < sum(c_on[:14]) < pairs
    g.close()
