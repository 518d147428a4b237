"""The full-size parity checks (tests/parity.py) on the CPU: outputs taken
from the oracle itself pass, and a planted error of each kind — a step off
by more than 1e-12, a wrong hit outside a tie, a hit on a tie that names a
volume not reached at the step — is caught and not exempted."""
import numpy as np
import pytest

from paper_1312_0816_amd import workloads as W
from tests.parity import batched_parity, check_ties, nav_parity, shape_parity


@pytest.fixture(scope="module")
def toy(orc):
    vol, t = W.toy_detector_c2(n=4000, seed=1200)
    s, h, _ = orc.navigate(vol, t, None, "ld")
    return vol, t, s, h


def test_oracle_outputs_pass(orc, toy):
    vol, t, s, h = toy
    rep = nav_parity(orc, vol, t, s, h, threads=4)
    assert rep["ok"] and rep["beyond_1e-12"] == 0 and rep["not_exempt"] == 0


def test_planted_step_error_is_caught(orc, toy):
    vol, t, s, h = toy
    s2 = s.copy()
    i = int(np.nonzero((s2 > 1) & (s2 < 1e30))[0][7])
    s2[i] *= 1 + 5e-12
    rep = nav_parity(orc, vol, t, s2, h, threads=4)
    assert not rep["ok"] and rep["not_exempt"] == 1 and rep["not_exempt_examples"][0]["track"] == i


def test_planted_hit_error_is_caught(orc, toy):
    vol, t, s, h = toy
    h2 = h.copy()
    i = int(np.nonzero(h2 >= 0)[0][3])
    h2[i] = (h2[i] + 1) % vol.nd
    rep = nav_parity(orc, vol, t, s, h2, threads=4)
    assert not rep["ok"] and rep["hit_mismatch_outside_ties"] == 1


def test_tie_validity(orc):
    """Two touching boxes reached at the same step: either index is a valid
    winner; the mother (-1) is not."""
    pars = np.zeros((2, W.NPAR))
    pars[:, :3] = [10.0, 5.0, 5.0]
    vol = W.Volume(W.BOX, np.array([200.0, 200.0, 200.0, 0, 0]), np.zeros(2, np.int32), pars,
                   np.tile(np.eye(3).reshape(9), (2, 1)), np.array([[-10.0, 0, 0], [10.0, 0, 0]]),
                   np.full(2, 12.3))
    n = 16
    z = np.linspace(-3, 3, n)
    t = np.ascontiguousarray(np.stack([np.zeros(n), np.full(n, -100.0), z, np.zeros(n), np.ones(n),
                                       np.zeros(n)]))
    s, h, gap = orc.navigate(vol, t, None, "ld")
    assert np.all(gap < 1e-9) and np.all(np.abs(s - 95.0) < 1e-12)
    assert check_ties(orc, vol, t, s, np.ones(n, np.int32), gap, max_tie_frac=1.0) == n
    assert check_ties(orc, vol, t, s, np.zeros(n, np.int32), gap, max_tie_frac=1.0) == n
    with pytest.raises(AssertionError):
        check_ties(orc, vol, t, s, np.full(n, -1, np.int32), gap, max_tie_frac=1.0)
    with pytest.raises(AssertionError):
        check_ties(orc, vol, t, s, np.ones(n, np.int32), gap, max_tie_frac=0.0)


def test_batched_and_shape_forms(orc):
    wl = W.batched_c3(scale=0.003, nvol=4, nb=8)
    s = np.zeros(wl.tracks.shape[1])
    h = np.zeros(wl.tracks.shape[1], np.int32)
    for b in range(len(wl.basket_n)):
        o, m = int(wl.basket_offset[b]), int(wl.basket_n[b])
        s[o:o + m], h[o:o + m], _ = orc.navigate(wl.volumes[int(wl.basket_volume[b])],
                                                 np.ascontiguousarray(wl.tracks[:, o:o + m]), None, "ld")
    assert batched_parity(orc, wl, s, h, threads=2)["ok"]
    s[3] += 1e-6
    rep = batched_parity(orc, wl, s, h, threads=2)
    assert not rep["ok"] and rep["not_exempt"] == 1
    kind, par, t = W.box_c0(n=2000)
    for q in (0, 1, 2, 3):
        ref = orc.shape_query(kind, par, q, t, "ld")
        assert shape_parity(orc, kind, par, q, t, ref, threads=2)["ok"]
        bad = ref.copy()
        j = int(np.nonzero(bad == 0)[0][0]) if q == 0 else int(np.nonzero((bad > 1) & (bad < 1e30))[0][0])
        bad[j] = 1 if q == 0 else bad[j] * (1 + 1e-10)
        assert shape_parity(orc, kind, par, q, t, bad, threads=2)["not_exempt"] == 1
