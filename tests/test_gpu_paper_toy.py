"""The paper's own toy detector (section 3.2): tubular mother, two tubes, four
boxes, two cones. Navigator parity, and the basket-size scan of the paper's
benchmark protocol (N consecutive particles from a pool, N x P constant) in
the batched form."""
import numpy as np
import pytest

from paper_1312_0816_amd import workloads as W
from tests.parity import check_ties, check_values, ill_conditioned

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gv():
    import torch
    from paper_1312_0816_amd import geonav
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    geonav.load_library()
    return geonav


def test_paper_toy_navigator_parity(gv, orc):
    import torch
    vol = W.paper_toy_detector()
    tr = W.paper_toy_tracks(n=30000)
    g = gv.Geometry([vol])
    s, h = gv.geo_navigate_basket(g, 0, torch.from_numpy(tr).cuda())
    s, h = s.cpu().numpy(), h.cpu().numpy()
    ref, ill = ill_conditioned(lambda x: orc.navigate(vol, x, None, "d")[0],
                               lambda x: orc.navigate(vol, x, None, "ld")[0], tr)
    print(check_values(s, ref, ill, "paper toy"))
    _, rh, gap = orc.navigate(vol, tr, None, "ld")
    assert np.array_equal(h[gap >= 1e-9], rh[gap >= 1e-9])
    print("ties", check_ties(orc, vol, tr, s, h, gap, what="paper toy"))
    assert len(np.unique(h)) == vol.nd + 1
    g.close()


@pytest.mark.parametrize("N", [16, 1024, 65536])
def test_paper_toy_basket_scan(gv, orc, N):
    """P = 2^18 / N baskets of N consecutive tracks from a random start in a
    2^20-track pool, in one batched launch: bit-identical to one launch per
    basket, and equal to the oracle on sampled baskets."""
    import torch
    vol = W.paper_toy_detector()
    pool = W.paper_toy_tracks()
    total = 1 << 18
    start = int(np.random.default_rng(N).integers(0, pool.shape[1] - total))
    P = total // N
    offs = start + N * np.arange(P)
    g = gv.Geometry([vol])
    t = torch.from_numpy(pool).cuda()
    s, h = gv.geo_navigate_batched(g, np.zeros(P, np.int32), offs, np.full(P, N), t)
    torch.cuda.synchronize()
    s, h = s.cpu().numpy(), h.cpu().numpy()
    rng = np.random.default_rng(7)
    for b in rng.choice(P, size=min(P, 4), replace=False):
        o = int(offs[b])
        sub = t[:, o:o + N].contiguous()
        s1, h1 = gv.geo_navigate_basket(g, 0, sub)
        assert np.array_equal(s1.cpu().numpy().view(np.int64), s[o:o + N].view(np.int64))
        assert np.array_equal(h1.cpu().numpy(), h[o:o + N])
        tr = np.ascontiguousarray(pool[:, o:o + min(N, 2000)])
        ref, ill = ill_conditioned(lambda x: orc.navigate(vol, x, None, "d")[0],
                                   lambda x: orc.navigate(vol, x, None, "ld")[0], tr)
        check_values(s[o:o + tr.shape[1]], ref, ill, f"N={N} basket {b}")
        _, rh, gap = orc.navigate(vol, tr, None, "ld")
        m = tr.shape[1]
        assert np.array_equal(h[o:o + m][gap >= 1e-9], rh[gap >= 1e-9])
        check_ties(orc, vol, tr, s[o:o + m], h[o:o + m], gap, what=f"N={N} basket {b}")
    g.close()
