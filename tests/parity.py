"""Parity rules between the HIP path and the oracle.

Reference values come from the oracle's long-double build. A floating-point
result must satisfy |gpu - ref| <= 1e-12 * max(|ref|, 1) (GEO_BIG compared
exactly) unless the track is ill-conditioned, i.e. one of:
  * the oracle's double and long-double builds differ by more than
    1e-13 * max(|ref|, 1) (or one of them misses while the other hits);
  * moving the origin by 1e-9 along any axis (both signs) changes the result
    by more than an FP64 evaluation can resolve at 1e-12: the difference
    quotient kappa satisfies kappa * (|p| + |ref| + 1) * 8 eps > 1e-12 * max(|ref|, 1),
    or flips hit/miss, in either the double or the long-double build (a line
    that only touches the closed solid at one point is a hit or a miss by
    rounding, and one build may see the flip where the other does not);
  * for Contains: the point lies within 1e-9 of the surface;
  * for the navigator's hit index: the two smallest candidate distances are
    within 1e-9 of each other.
Exempt tracks are counted and reported, never silently dropped, and their
number is bounded by the tests.
"""
from __future__ import annotations

import numpy as np

BIG = 1e30
TOL = 1e-12
EPS = 2.220446049250313e-16
DELTA = 1e-9


def rel_diff(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    bigmis = (a >= BIG) != (b >= BIG)
    d = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    d = np.where((a >= BIG) & (b >= BIG), 0.0, d)
    return np.where(bigmis, np.inf, d)


def _kappa(f, tracks, ref):
    """Largest difference quotient of f under +-DELTA moves of the origin."""
    kap = np.zeros(tracks.shape[1])
    for axis in range(3):
        for sgn in (1.0, -1.0):
            t2 = tracks.copy()
            t2[axis] += sgn * DELTA
            r = f(t2)
            flip = (r >= BIG) != (ref >= BIG)
            dq = np.where((r >= BIG) & (ref >= BIG), 0.0, np.abs(r - ref) / DELTA)
            kap = np.maximum(kap, np.where(flip, np.inf, dq))
    return kap


def ill_conditioned(f_d, f_ld, tracks):
    """Flags for tracks whose result FP64 cannot be trusted to 1e-12.
    f_d / f_ld: callables tracks -> values (oracle double / long double)."""
    ref = f_ld(tracks)
    rd = f_d(tracks)
    flag = rel_diff(rd, ref) > 1e-13
    kap = np.maximum(_kappa(f_d, tracks, rd), _kappa(f_ld, tracks, ref))
    scale = np.linalg.norm(tracks[:3], axis=0) + np.where(ref < BIG, np.abs(ref), 0.0) + 1.0
    flag |= kap * scale * 8 * EPS > TOL * np.maximum(np.where(ref < BIG, np.abs(ref), 1.0), 1.0)
    return ref, flag


def check_values(gpu, ref, exempt, what, max_exempt_frac=2e-3):
    """Assert the rule above and return a small report dict."""
    gpu = np.asarray(gpu, np.float64)
    e = rel_diff(gpu, ref)
    bad = (e > TOL) & ~exempt
    rep = {"what": what, "n": int(gpu.size), "exempt": int(exempt.sum()),
           "exempt_fail": int(((e > TOL) & exempt).sum()),
           "max_rel_err": float(np.max(np.where(exempt, 0.0, e))) if gpu.size else 0.0}
    assert not np.any(np.isnan(gpu)), f"{what}: NaN in GPU output"
    if bad.any():
        idx = np.nonzero(bad)[0][:8]
        raise AssertionError(f"{what}: {int(bad.sum())} tracks beyond 1e-12: "
                             + ", ".join(f"#{i}: gpu={gpu[i]!r} ref={ref[i]!r}" for i in idx))
    assert rep["exempt"] <= max(8, max_exempt_frac * gpu.size), f"{what}: too many exempt {rep}"
    return rep
