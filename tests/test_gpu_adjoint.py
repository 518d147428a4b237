"""The adjoint navigator (geo_navigate_backward / Navigate autograd) against
central finite differences of the oracle, on the toy detector."""
import numpy as np
import pytest

from paper_1312_0816_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-6


@pytest.fixture(scope="module")
def gv():
    import torch
    from paper_1312_0816_amd import geonav
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    geonav.load_library()
    return geonav


def _close(ad, fd, what):
    """Per component |ad - fd| <= 1e-6 max(|fd|, 1e-3 rms(fd))."""
    floor = 1e-3 * np.sqrt(np.mean(fd * fd)) + 1e-300
    err = np.abs(ad - fd) / np.maximum(np.abs(fd), floor)
    bad = err > RTOL
    assert not bad.any(), f"{what}: {int(bad.sum())} components beyond {RTOL}, worst {err.max():.3g}"
    return float(err.max())


def _oracle_upstream(orc, vol, tracks, targets, offs):
    s, _, _ = orc.navigate(vol, tracks, offs, "ld")
    h = tracks[:3] + s[None, :] * tracks[3:]
    return 2.0 * (h - targets)          # dL/dh for L = sum |h - g|^2


def test_full_size_loss_gradients_match_fd(gv, orc):
    """1M tracks through Navigate (forward + autograd backward) with
    L = sum |hit point - target|^2; 3000 sampled tracks compared with the
    oracle's central differences (h = 1e-6) wherever the oracle finds the
    track smooth within the stencil."""
    import torch
    vol, tracks, targets = W.adjoint_c4()
    n = tracks.shape[1]
    g = gv.Geometry([vol])
    o = torch.from_numpy(np.ascontiguousarray(tracks[:3])).cuda().requires_grad_()
    d = torch.from_numpy(np.ascontiguousarray(tracks[3:])).cuda().requires_grad_()
    offs = torch.zeros((vol.nd, 3), dtype=torch.float64, device="cuda", requires_grad=True)
    tg = torch.from_numpy(targets).cuda()
    step, hp, hit = gv.navigate(g, 0, o, d, offs)
    loss = ((hp - tg) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g_o, g_d = o.grad.cpu().numpy(), d.grad.cpu().numpy()
    assert np.isfinite(g_o).all() and np.isfinite(g_d).all() and np.isfinite(offs.grad.cpu().numpy()).all()

    rng = np.random.default_rng(21)
    idx = np.sort(rng.choice(n, size=3000, replace=False))
    sub = np.ascontiguousarray(tracks[:, idx])
    zero = np.zeros((vol.nd, 3))
    gh = _oracle_upstream(orc, vol, sub, targets[:, idx], zero)
    fd = orc.navigate_fd(vol, sub, zero, None, gh)
    m = fd["mask"]
    assert m.mean() > 0.9, f"only {m.mean():.3f} of sampled tracks are smooth"
    e1 = _close(g_o[:, idx][:, m], fd["g_o"][:, m], "g_o")
    e2 = _close(g_d[:, idx][:, m], fd["g_d"][:, m], "g_d")
    print({"sampled": int(idx.size), "smooth": int(m.sum()), "max_err_g_o": e1, "max_err_g_d": e2})
    g.close()


def test_offset_gradient_matches_fd_sum(gv, orc):
    """g_off = sum over tracks of dL/d delta_k, compared with the sum of the
    oracle's per-track central differences over tracks smooth in the
    stencil (the GPU runs on exactly those tracks)."""
    import torch
    vol, tracks, targets = W.adjoint_c4(n=20000, seed=1477)
    offs = np.random.default_rng(2).uniform(-1.0, 1.0, (vol.nd, 3))
    gh = _oracle_upstream(orc, vol, tracks, targets, offs)
    fd = orc.navigate_fd(vol, tracks, offs, None, gh)
    m = fd["mask"]
    assert m.mean() > 0.9
    sub = np.ascontiguousarray(tracks[:, m])
    ghs = np.ascontiguousarray(gh[:, m])
    want = np.zeros((vol.nd, 3))
    for k in range(vol.nd):
        sel = fd["hit"][m] == k
        want[k] = fd["g_off_hit"][:, m][:, sel].sum(axis=1)
    g = gv.Geometry([vol])
    o = torch.from_numpy(np.ascontiguousarray(sub[:3])).cuda()
    d = torch.from_numpy(np.ascontiguousarray(sub[3:])).cuda()
    go, gd, goff = gv.geo_navigate_backward(g, 0, o, d, torch.from_numpy(offs).cuda(), None,
                                            torch.from_numpy(ghs).cuda())
    got = goff.cpu().numpy()
    _close(got, want, "g_off")
    _close(go.cpu().numpy(), fd["g_o"][:, m], "g_o (explicit upstream)")
    _close(gd.cpu().numpy(), fd["g_d"][:, m], "g_d (explicit upstream)")
    # deterministic: a second call gives the same bits
    _, _, goff2 = gv.geo_navigate_backward(g, 0, o, d, torch.from_numpy(offs).cuda(), None,
                                           torch.from_numpy(ghs).cuda(), want_o=False, want_d=False)
    assert np.array_equal(goff2.cpu().numpy(), got)
    g.close()


def test_step_gradient_only(gv, orc):
    """Upstream gradient on the step alone: g_o = ds/do = -n/(n.d)."""
    import torch
    vol, tracks, _ = W.adjoint_c4(n=4000, seed=1499)
    n = tracks.shape[1]
    gs = np.ones(n)
    fd = orc.navigate_fd(vol, tracks, None, gs, None)
    m = fd["mask"]
    g = gv.Geometry([vol])
    o = torch.from_numpy(np.ascontiguousarray(tracks[:3])).cuda()
    d = torch.from_numpy(np.ascontiguousarray(tracks[3:])).cuda()
    go, gd, goff = gv.geo_navigate_backward(g, 0, o, d, None, torch.from_numpy(gs).cuda(), None)
    _close(go.cpu().numpy()[:, m], fd["g_o"][:, m], "ds/do")
    _close(gd.cpu().numpy()[:, m], fd["g_d"][:, m], "ds/dd")
    g.close()


def test_gradcheck_small(gv, orc):
    """torch.autograd.gradcheck on 48 smooth tracks (the finite differences
    here run the GPU forward)."""
    import torch
    vol, tracks, targets = W.adjoint_c4(n=400, seed=1511)
    zero = np.zeros((vol.nd, 3))
    fd = orc.navigate_fd(vol, tracks, zero, None, _oracle_upstream(orc, vol, tracks, targets, zero))
    sel = np.nonzero(fd["mask"] & (fd["hit"] >= 0))[0][:48]
    sub = np.ascontiguousarray(tracks[:, sel])
    g = gv.Geometry([vol])
    o = torch.from_numpy(np.ascontiguousarray(sub[:3])).cuda().requires_grad_()
    d = torch.from_numpy(np.ascontiguousarray(sub[3:])).cuda().requires_grad_()
    offs = torch.zeros((vol.nd, 3), dtype=torch.float64, device="cuda", requires_grad=True)

    def f(o_, d_, off_):
        s, hp, _ = gv.navigate(g, 0, o_.contiguous(), d_.contiguous(), off_.contiguous())
        return s, hp

    assert torch.autograd.gradcheck(f, (o, d, offs), eps=1e-7, atol=1e-5, rtol=1e-5)
    g.close()


def test_backward_edge_cases(gv):
    """Empty basket; a volume whose tracks start outside the mother (step 0:
    gradient of the hit point only)."""
    import torch
    vol = W.toy_detector_volume()
    g = gv.Geometry([vol])
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    go, gd, goff = gv.geo_navigate_backward(g, 0, e, e, None, None, None)
    assert go.numel() == 0 and torch.all(goff == 0)
    o = torch.tensor([[500.0], [0.0], [0.0]], dtype=torch.float64, device="cuda")
    d = torch.tensor([[1.0], [0.0], [0.0]], dtype=torch.float64, device="cuda")
    gh = torch.tensor([[1.0], [2.0], [3.0]], dtype=torch.float64, device="cuda")
    go, gd, goff = gv.geo_navigate_backward(g, 0, o, d, None, torch.ones(1, dtype=torch.float64,
                                                                          device="cuda"), gh)
    assert torch.equal(go[:, 0].cpu(), torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64))
    assert torch.all(gd == 0) and torch.all(goff == 0)
    g.close()
