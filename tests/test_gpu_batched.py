"""The batched persistent navigator (geo_navigate_batched): bit-identical to
per-basket launches, oracle parity on samples, every launch shape, graph
replays, and the autotuner."""
import json
import os

import numpy as np
import pytest

from paper_1312_0816_amd import workloads as W
from tests.parity import batched_parity, check_ties, check_values, ill_conditioned

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gv():
    import torch
    from paper_1312_0816_amd import geonav
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    geonav.load_library()
    return geonav


@pytest.fixture(scope="module")
def small():
    return W.batched_c3(scale=0.03)


def per_basket(gv, g, wl, t):
    import torch
    n = t.shape[1]
    step = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    hit = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    for b in range(len(wl.basket_n)):
        o, m = int(wl.basket_offset[b]), int(wl.basket_n[b])
        if m == 0:
            continue
        sub = t[:, o:o + m].contiguous()
        s, h = gv.geo_navigate_basket(g, int(wl.basket_volume[b]), sub)
        step[o:o + m] = s
        hit[o:o + m] = h
    torch.cuda.synchronize()
    return step.cpu().numpy(), hit.cpu().numpy()


def batched(gv, g, wl, t):
    import torch
    s, h = gv.geo_navigate_batched(g, wl.basket_volume, wl.basket_offset, wl.basket_n, t)
    torch.cuda.synchronize()
    return s.cpu().numpy(), h.cpu().numpy()


def test_batched_bit_identical_to_per_basket(gv, small):
    """Every launch shape, with the two kernels as two launches and as a
    graph replay, equals the per-basket navigator bit for bit."""
    import torch
    g = gv.Geometry(small.volumes)
    t = torch.from_numpy(small.tracks).cuda()
    s0, h0 = per_basket(gv, g, small, t)
    assert not g.batched_graph  # the default: two launches
    for graph in (False, True):
        g.batched_graph = graph
        assert g.batched_graph == graph
        for U in (1, 2, 4, 8):
            for Wv in (0, 2, 4, 8):
                g.set_launch_config(U, Wv)
                s1, h1 = batched(gv, g, small, t)
                assert np.array_equal(s1.view(np.int64), s0.view(np.int64)), (graph, U, Wv)
                assert np.array_equal(h1, h0), (graph, U, Wv)
    with pytest.raises(gv.GeoError):
        gv._check(g._lib.geo_set_batched_graph(g.handle, 2))
    g.close()


def test_batched_matches_oracle(gv, orc, small):
    import torch
    g = gv.Geometry(small.volumes)
    t = torch.from_numpy(small.tracks).cuda()
    s, h = batched(gv, g, small, t)
    rng = np.random.default_rng(4)
    for b in rng.choice(len(small.basket_n), size=40, replace=False):
        o, m = int(small.basket_offset[b]), int(small.basket_n[b])
        vol = small.volumes[int(small.basket_volume[b])]
        tr = np.ascontiguousarray(small.tracks[:, o:o + m])
        ref, ill = ill_conditioned(lambda x: orc.navigate(vol, x, None, "d")[0],
                                   lambda x: orc.navigate(vol, x, None, "ld")[0], tr)
        check_values(s[o:o + m], ref, ill, f"basket {b}")
        _, rh, gap = orc.navigate(vol, tr, None, "ld")
        assert np.array_equal(h[o:o + m][gap >= 1e-9], rh[gap >= 1e-9])
        check_ties(orc, vol, tr, s[o:o + m], h[o:o + m], gap, what=f"basket {b}")
    g.close()


@pytest.mark.parametrize("graph", [True, False])
def test_graph_replays_interleaved(gv, small, graph):
    """Replay the cached graph (or the two launches) several times with other
    device work and host synchronisation in between; every replay equals
    the first."""
    import torch
    g = gv.Geometry(small.volumes)
    g.batched_graph = graph
    t = torch.from_numpy(small.tracks).cuda()
    s0, h0 = batched(gv, g, small, t)
    for rep in range(5):
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
        step = torch.zeros(t.shape[1], dtype=torch.float64, device="cuda")
        hit = torch.zeros(t.shape[1], dtype=torch.int32, device="cuda")
        gv.geo_navigate_batched(g, small.basket_volume, small.basket_offset, small.basket_n, t, step, hit)
        junk.item()
        torch.cuda.synchronize()
        assert np.array_equal(step.cpu().numpy(), s0)
        assert np.array_equal(hit.cpu().numpy(), h0)
    # a different basket list (a subset, reversed) on the same handle
    sel = np.arange(len(small.basket_n))[::-3]
    step = torch.full((t.shape[1],), -5.0, dtype=torch.float64, device="cuda")
    hit = torch.full((t.shape[1],), -5, dtype=torch.int32, device="cuda")
    gv.geo_navigate_batched(g, small.basket_volume[sel], small.basket_offset[sel], small.basket_n[sel], t,
                            step, hit)
    torch.cuda.synchronize()
    s2, h2 = step.cpu().numpy(), hit.cpu().numpy()
    covered = np.zeros(t.shape[1], bool)
    for b in sel:
        covered[small.basket_offset[b]:small.basket_offset[b] + small.basket_n[b]] = True
    assert np.array_equal(s2[covered], s0[covered]) and np.array_equal(h2[covered], h0[covered])
    assert np.all(s2[~covered] == -5.0) and np.all(h2[~covered] == -5)
    g.close()


@pytest.mark.parametrize("shape", [(4, 0), (2, 2)])
def test_back_to_back_calls_with_different_baskets(gv, small, shape):
    """Eight calls queued without synchronisation, each on its own basket
    list (subsets in different orders) and its own outputs, the submission
    switching between two launches and the graph replay: each call's tile
    expansion rewrites the handle's tile buffer and (persistent shape) queue
    cursors, so every call must see its own tiles."""
    import torch
    g = gv.Geometry(small.volumes)
    g.set_launch_config(*shape)
    t = torch.from_numpy(small.tracks).cuda()
    s0, h0 = per_basket(gv, g, small, t)
    nb = len(small.basket_n)
    idx = np.arange(nb)
    sels = [idx, idx[::-1], idx[::2], idx[1::3], idx[::-5], np.roll(idx, nb // 3), idx[nb // 2:], idx[:nb // 2][::-1]]
    graphs = [False, False, True, False, True, True, False, False]
    n = t.shape[1]
    outs = []
    for c, sel in enumerate(sels):
        g.batched_graph = graphs[c]
        step = torch.full((n,), -5.0 - c, dtype=torch.float64, device="cuda")
        hit = torch.full((n,), -5 - c, dtype=torch.int32, device="cuda")
        gv.geo_navigate_batched(g, small.basket_volume[sel], small.basket_offset[sel], small.basket_n[sel], t,
                                step, hit)
        outs.append((sel, step, hit))
    torch.cuda.synchronize()
    for c, (sel, step, hit) in enumerate(outs):
        s, h = step.cpu().numpy(), hit.cpu().numpy()
        covered = np.zeros(n, bool)
        for b in sel:
            covered[small.basket_offset[b]:small.basket_offset[b] + small.basket_n[b]] = True
        assert np.array_equal(s[covered].view(np.int64), s0[covered].view(np.int64)), c
        assert np.array_equal(h[covered], h0[covered]), c
        assert np.all(s[~covered] == -5.0 - c) and np.all(h[~covered] == -5 - c), c
    g.close()


def test_contiguous_baskets_joined(gv, small):
    """Each basket cut into contiguous pieces of random sizes: given in
    order, the pieces of a basket are joined back before tiling; shuffled,
    only pieces that happen to meet again after the sort are. Both equal
    the per-basket navigator bit for bit, as does a single-volume pool cut
    into 16-track baskets (the paper's scan at its smallest basket size)."""
    import torch
    g = gv.Geometry(small.volumes)
    t = torch.from_numpy(small.tracks).cuda()
    s0, h0 = per_basket(gv, g, small, t)
    rng = np.random.default_rng(17)
    vol, off, cnt = [], [], []
    for b in range(len(small.basket_n)):
        o, m = int(small.basket_offset[b]), int(small.basket_n[b])
        cuts = np.sort(rng.choice(np.arange(1, m), size=min(m - 1, 3), replace=False)) if m > 1 else []
        edges = [0, *[int(c) for c in cuts], m]
        for a, e in zip(edges[:-1], edges[1:]):
            vol.append(int(small.basket_volume[b]))
            off.append(o + a)
            cnt.append(e - a)
    vol, off, cnt = np.array(vol, np.int32), np.array(off, np.int64), np.array(cnt, np.int64)
    for order in (np.arange(len(vol)), rng.permutation(len(vol))):
        s, h = gv.geo_navigate_batched(g, vol[order], off[order], cnt[order], t)
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy().view(np.int64), s0.view(np.int64))
        assert np.array_equal(h.cpu().numpy(), h0)
    g.close()
    # one volume, 16-track baskets back to back
    vol1 = small.volumes[int(np.argmax([v.nd for v in small.volumes]))]
    g1 = gv.Geometry([vol1])
    n = 16 * 1000 + 7
    tr = torch.from_numpy(W.tracks_in_mother(np.random.default_rng(18), vol1, n)).cuda()
    offs = np.arange(0, n, 16, dtype=np.int64)
    cnts = np.minimum(16, n - offs)
    s1, h1 = gv.geo_navigate_batched(g1, np.zeros(len(offs), np.int32), offs, cnts, tr)
    s2, h2 = gv.geo_navigate_basket(g1, 0, tr)
    torch.cuda.synchronize()
    assert np.array_equal(s1.cpu().numpy().view(np.int64), s2.cpu().numpy().view(np.int64))
    assert np.array_equal(h1.cpu().numpy(), h2.cpu().numpy())
    g1.close()


def test_basket_calls_in_a_captured_graph(gv, small):
    """geo_navigate_basket calls captured in one HIP graph (torch.cuda.graph)
    and replayed three times, with output clearing, other device work and
    host synchronisation between the replays: every replay equals the eager
    per-basket result bit for bit."""
    import torch
    g = gv.Geometry(small.volumes)
    t = torch.from_numpy(small.tracks).cuda()
    s0, h0 = per_basket(gv, g, small, t)
    subs = []
    for b in range(len(small.basket_n)):
        o, m = int(small.basket_offset[b]), int(small.basket_n[b])
        if m > 0:
            subs.append((o, m, int(small.basket_volume[b]), t[:, o:o + m].contiguous()))
    torch.cuda.synchronize()
    cg = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    outs = []
    with torch.cuda.graph(cg, stream=cs):
        for o, m, v, sub in subs:
            outs.append((o, m) + tuple(gv.geo_navigate_basket(g, v, sub, stream=cs)))
    torch.cuda.current_stream().wait_stream(cs)
    for rep in range(3):
        for _, _, st, ht in outs:
            st.fill_(-1.0)
            ht.fill_(-7)
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
        cg.replay()
        junk.item()
        torch.cuda.synchronize()
        for o, m, st, ht in outs:
            assert np.array_equal(st.cpu().numpy().view(np.int64), s0[o:o + m].view(np.int64)), (rep, o)
            assert np.array_equal(ht.cpu().numpy(), h0[o:o + m]), (rep, o)
    del cg
    g.close()


def test_full_workload_bit_identical(gv):
    """The full 512-basket, 64-volume workload (about 4.4M tracks)."""
    import torch
    wl = W.batched_c3()
    assert len(wl.volumes) == 64 and len(wl.basket_n) == 512
    g = gv.Geometry(wl.volumes)
    t = torch.from_numpy(wl.tracks).cuda()
    s0, h0 = per_basket(gv, g, wl, t)
    s1, h1 = batched(gv, g, wl, t)
    assert np.array_equal(s1.view(np.int64), s0.view(np.int64))
    assert np.array_equal(h1, h0)
    g.close()


THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.mark.parametrize("reject", [True, False])
def test_full_workload_every_track_matches_oracle(gv, orc, reject):
    """The full batched workload (512 baskets, 64 volumes), every track
    against the oracle's long-double build; with reject=False the tracks are
    uniform in each mother with no rejection (some start inside daughters,
    many near their surfaces)."""
    import torch
    wl = W.batched_c3(reject=reject)
    g = gv.Geometry(wl.volumes)
    t = torch.from_numpy(wl.tracks).cuda()
    s, h = batched(gv, g, wl, t)
    g.close()
    rep = batched_parity(orc, wl, s, h, threads=THREADS)
    print(f"batched workload, reject={reject}, every track:", rep)
    assert rep["ok"], rep
    assert rep["exempt"] <= max(8, 2e-3 * rep["tracks"])
    assert rep["hit_ties"] <= max(8, 1e-3 * rep["tracks"])


def test_empty_baskets_and_errors(gv, small):
    import torch
    g = gv.Geometry(small.volumes)
    t = torch.from_numpy(small.tracks).cuda()
    s, h = gv.geo_navigate_batched(g, [0, 1], [0, 5], [0, 0], t)   # all empty: no-op
    with pytest.raises(gv.GeoError):
        gv.geo_navigate_batched(g, [0], [t.shape[1] - 2], [5], t)  # past the pool
    with pytest.raises(gv.GeoError):
        gv.geo_navigate_batched(g, [99], [0], [5], t)             # bad volume
    g.close()


def test_autotune_and_cache(gv, small, tmp_path, monkeypatch):
    import torch
    path = tmp_path / "tune.json"
    monkeypatch.setenv("GEONAV_AUTOTUNE_CACHE", str(path))
    g = gv.Geometry(small.volumes)
    t = torch.from_numpy(small.tracks).cuda()
    u, w = gv.geo_autotune(g, small.basket_volume, small.basket_offset, small.basket_n, t)
    assert u in (1, 2, 4, 8) and 0 <= w <= 8
    graph = g.batched_graph
    data = json.loads(path.read_text())
    assert len(data) == 1 and list(data.values())[0] == [u, w, int(graph)]
    g2 = gv.Geometry(small.volumes)
    g2.set_launch_config(1, 1)
    g2.batched_graph = not graph
    assert gv.geo_autotune(g2, small.basket_volume, small.basket_offset, small.basket_n, t) == (u, w)
    assert g2.batched_graph == graph
    # an entry of two numbers (written before the launch mode was tuned)
    # reads as two launches
    key = list(data.keys())[0]
    path.write_text(json.dumps({key: [u, w]}))
    g2.batched_graph = True
    assert gv.geo_autotune(g2, small.basket_volume, small.basket_offset, small.basket_n, t) == (u, w)
    assert not g2.batched_graph
    g.close()
    g2.close()
    assert os.path.exists(path)


@pytest.mark.parametrize("graph", [False, True])
def test_kernel_timing_events(gv, small, graph):
    """The timing events around the navigator kernel (on the stream, or
    nodes of the graph): a positive duration below the whole call's, the
    same outputs with them, and a clear error before any timed call."""
    import time
    import torch
    g = gv.Geometry(small.volumes)
    g.batched_graph = graph
    t = torch.from_numpy(small.tracks).cuda()
    args = (small.basket_volume, small.basket_offset, small.basket_n, t)
    s0, h0 = gv.geo_navigate_batched(g, *args)
    with pytest.raises(gv.GeoError):
        g.batched_kernel_ms()
    g.set_kernel_timing(True)
    with pytest.raises(gv.GeoError):
        g.batched_kernel_ms()
    for _ in range(3):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        s1, h1 = gv.geo_navigate_batched(g, *args)
        ms = g.batched_kernel_ms()
        wall = 1e3 * (time.perf_counter() - w0)
        assert 0.0 < ms < wall
        assert torch.equal(s0.view(torch.int64), s1.view(torch.int64)) and torch.equal(h0, h1)
    g.set_kernel_timing(False)
    s2, h2 = gv.geo_navigate_batched(g, *args)
    assert torch.equal(s0.view(torch.int64), s2.view(torch.int64)) and torch.equal(h0, h2)
    with pytest.raises(gv.GeoError):
        g.batched_kernel_ms()
    g.close()
