"""Parity of the polycone (kind 5) on the GPU with the oracle: the suite
polycone at ragged and full sizes, six variants (two planes, a flared pipe,
eight planes with a zig-zag profile uncut and cut, a spindle cut to a
convex range, collinear planes), tracks along the section planes and in the
cut faces, and the errors the library rejects."""
import numpy as np
import pytest

from paper_1312_0816_amd import workloads as W
from tests.test_gpu_shapes import compare, gpu_query

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gv():
    import torch
    from paper_1312_0816_amd import geonav
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    geonav.load_library()
    return geonav


@pytest.mark.parametrize("v", range(len(W.PCON_VARIANTS)))
def test_polycone_variants(gv, orc, v):
    par = W.PCON_VARIANTS[v]
    _, _, t = W.shape_suite_c1(W.PCON, n=20000, seed=3300 + v, par=par)
    print(compare(gv, orc, W.PCON, par, t, f"polycone variant {v}"))


def test_tracks_along_section_planes(gv, orc):
    """Origins on the planes between sections (where the profile kinks),
    isotropic and in-plane directions, and tracks aimed at points of the
    kinks' circles."""
    rng = np.random.default_rng(51)
    for v in (1, 2, 3):
        par = W.PCON_VARIANTS[v]
        z, rin, rout = W.pcon_planes(par)
        parts = []
        for j in range(1, len(z) - 1):
            m = 1500
            r = rng.uniform(0, 1.3 * rout[j], m)
            ph = rng.uniform(0, 2 * np.pi, m)
            p = np.stack([r * np.cos(ph), r * np.sin(ph), np.full(m, z[j])])
            u = np.stack(W.isotropic(rng, m))
            flat = rng.uniform(size=m) < 0.3
            u[2, flat] = 0.0
            u[:, flat] /= np.linalg.norm(u[:, flat], axis=0)
            parts.append(np.concatenate([p, u]))
            # aimed at the outer kink circle
            o = rng.uniform(-40, 40, (3, m))
            aim = np.stack([rout[j] * np.cos(ph), rout[j] * np.sin(ph), np.full(m, z[j])])
            d = aim - o
            d /= np.linalg.norm(d, axis=0)
            parts.append(np.concatenate([o, d]))
        t = np.ascontiguousarray(np.concatenate(parts, axis=1))
        # at most 0.0746 of one variant's tracks exempt for one query (the
        # oracle's classification of these seeded inputs), plus 0.01
        print(compare(gv, orc, W.PCON, par, t, f"section planes variant {v}", max_exempt_frac=0.0846))


def test_two_plane_polycone_matches_cone_on_gpu(gv):
    """The two-plane polycone and the cone go through different kernels;
    they agree to 1e-12 except on a tiny fraction of grazing tracks."""
    from tests.parity import rel_diff
    _, par, t = W.shape_suite_c1(W.CONE, n=50000, seed=9)
    for q in (0, 1, 2, 3):
        a = gpu_query(gv, W.CONE, par, q, t)
        b = gpu_query(gv, W.PCON, W.PCON_VARIANTS[0], q, t)
        if q == 0:
            assert np.mean(a != b) < 1e-4
        else:
            assert np.mean(rel_diff(b, a) > 1e-12) < 1e-4


def test_polycone_errors(gv):
    import torch
    t = torch.zeros((6, 8), dtype=torch.float64, device="cuda")
    bad = [W.pcon_par(0, 2 * np.pi, [(0, 0, 5)]),                                 # one plane
           W.pcon_par(0, 2 * np.pi, [(0, 0, 5), (0, 0, 6)]),                      # z not increasing
           W.pcon_par(0, 2 * np.pi, [(0, 3, 2), (1, 0, 6)]),                      # rmin > rmax
           W.pcon_par(0, 0.0, [(0, 0, 5), (1, 0, 6)]),                            # dphi = 0
           W.pcon_par(0, 2 * np.pi, [(0, 0, 0), (1, 0, 0), (2, 0, 3)])]           # empty section
    for par in bad:
        with pytest.raises(gv.GeoError):
            gv.geo_shape_query(W.PCON, par, 0, t)
    nine = W.pcon_par(0, 2 * np.pi, [(i, 0, 5) for i in range(9)])
    with pytest.raises((gv.GeoError, ValueError)):
        gv.geo_shape_query(W.PCON, nine, 0, t)
