"""Parity rules between the HIP path and the oracle.

Reference values come from the oracle's long-double build. A floating-point
result must satisfy |gpu - ref| <= 1e-12 * max(|ref|, 1) (GEO_BIG compared
exactly) unless the track is ill-conditioned, i.e. one of:
  * (the double / long-double rule) the oracle's double and long-double
    builds differ by more than 1e-13 * max(|ref|, 1) (or one of them misses
    while the other hits);
  * (the sensitivity rule) moving the origin by 1e-9 along any axis (both
    signs) changes the result by more than an FP64 evaluation can resolve at
    1e-12: the difference quotient kappa satisfies
    kappa * (|p| + |ref| + 1) * 8 eps > 1e-12 * max(|ref|, 1), or flips
    hit/miss, in either the double or the long-double build (a line that
    only touches the closed solid at one point is a hit or a miss by
    rounding, and one build may see the flip where the other does not);
  * for Contains: the point lies within 1e-9 of the surface;
  * for the navigator's hit index: the two smallest candidate distances are
    within 1e-9 of each other. On such a tie the GPU's hit must still be a
    valid winner: the oracle's distance to the volume it names (the
    daughter's DistFromOutside in its frame, or the mother's DistFromInside
    for -1) equals the GPU's step within 1e-9.
Exempt tracks are counted and reported (split into those the double /
long-double rule flags and those only the sensitivity rule adds), never
silently dropped, and their number is bounded by the tests.

Two forms: the sampled checks (``ill_conditioned`` + ``check_values``)
classify every track of a sample; the full-size checks (``nav_parity``,
``shape_parity``) take the long-double reference of every track, on a
thread pool, and classify only the tracks beyond the tolerance.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

BIG = 1e30
TOL = 1e-12
EPS = 2.220446049250313e-16
DELTA = 1e-9
TIE_GAP = 1e-9


class Exemptions(np.ndarray):
    """Boolean flags of the ill-conditioned tracks; ``c15`` holds the part
    that the double / long-double rule alone flags."""

    def __new__(cls, flag, c15):
        obj = np.asarray(flag, bool).view(cls)
        obj.c15 = np.asarray(c15, bool)
        return obj

    def __array_finalize__(self, obj):
        self.c15 = getattr(obj, "c15", None)


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
    f_d / f_ld: callables tracks -> values (oracle double / long double).
    Returns (long-double reference, Exemptions)."""
    tracks = np.ascontiguousarray(tracks)
    ref = f_ld(tracks)
    rd = f_d(tracks)
    c15 = rel_diff(rd, ref) > 1e-13
    kap = np.maximum(_kappa(f_d, tracks, rd), _kappa(f_ld, tracks, ref))
    scale = np.linalg.norm(tracks[:3], axis=0) + np.where(ref < BIG, np.abs(ref), 0.0) + 1.0
    sens = kap * scale * 8 * EPS > TOL * np.maximum(np.where(ref < BIG, np.abs(ref), 1.0), 1.0)
    return ref, Exemptions(c15 | sens, c15)


def check_values(gpu, ref, exempt, what, max_exempt_frac=2e-3):
    """Assert the rule above and return a small report dict."""
    gpu = np.asarray(gpu, np.float64)
    e = rel_diff(gpu, ref)
    bad = (e > TOL) & ~exempt
    c15 = getattr(exempt, "c15", None)
    rep = {"what": what, "n": int(gpu.size), "exempt": int(np.sum(exempt)),
           "exempt_fail": int(((e > TOL) & exempt).sum()),
           "max_rel_err": float(np.max(np.where(exempt, 0.0, e))) if gpu.size else 0.0}
    if c15 is not None:
        rep["exempt_double_vs_long_double"] = int(c15.sum())
        rep["exempt_sensitivity_only"] = int((np.asarray(exempt, bool) & ~c15).sum())
    assert not np.any(np.isnan(gpu)), f"{what}: NaN in GPU output"
    if bad.any():
        idx = np.nonzero(bad)[0][:8]
        raise AssertionError(f"{what}: {int(bad.sum())} tracks beyond 1e-12: "
                             + ", ".join(f"#{i}: gpu={gpu[i]!r} ref={ref[i]!r}" for i in idx))
    assert rep["exempt"] <= max(8, max_exempt_frac * gpu.size), f"{what}: too many exempt {rep}"
    return rep


# ---------------------------------------------------------------- navigator

def _local_tracks(vol, k, tracks, offsets=None):
    """Tracks (6, m) of the mother frame in daughter k's frame:
    R^T (p - T - delta), R^T d."""
    R = np.asarray(vol.rots[k], np.float64).reshape(3, 3)
    t = np.asarray(vol.trs[k], np.float64).copy()
    if offsets is not None:
        t = t + np.asarray(offsets, np.float64).reshape(-1, 3)[k]
    p = R.T @ (tracks[:3] - t[:, None])
    d = R.T @ tracks[3:6]
    return np.ascontiguousarray(np.concatenate([p, d]))


def candidate_step(orc, vol, tracks, hit, offsets=None):
    """The oracle's (long double) distance from each track to the volume its
    `hit` names: the mother's DistFromInside for -1, else that daughter's
    DistFromOutside in its own frame."""
    tracks = np.ascontiguousarray(tracks, np.float64)
    hit = np.asarray(hit)
    out = np.full(hit.shape[0], np.nan)
    for k in np.unique(hit):
        sel = hit == k
        sub = np.ascontiguousarray(tracks[:, sel])
        if k < 0:
            out[sel] = orc.dist_in(int(vol.mother_kind), vol.mother_par, sub, "ld")
        elif k < vol.nd:
            out[sel] = orc.dist_out(int(vol.kinds[k]), vol.pars[k], _local_tracks(vol, int(k), sub, offsets),
                                    "ld")
    return out


def check_ties(orc, vol, tracks, step, hit, gap, offsets=None, what="nav", max_tie_frac=1e-3):
    """On every tie track (gap < TIE_GAP) the GPU's hit must name a volume
    whose oracle distance equals the GPU's step within 1e-9; the number of
    ties is bounded. Returns the tie count."""
    tie = np.asarray(gap) < TIE_GAP
    idx = np.nonzero(tie)[0]
    if idx.size:
        s = np.asarray(step, np.float64)[idx]
        cand = candidate_step(orc, vol, np.ascontiguousarray(np.asarray(tracks)[:, idx]),
                              np.asarray(hit)[idx], offsets)
        ok = np.abs(cand - s) <= TIE_GAP * np.maximum(np.abs(s), 1.0)
        ok &= np.asarray(hit)[idx] >= -1
        assert ok.all(), (f"{what}: {int((~ok).sum())} tie tracks whose GPU hit is not a valid winner, "
                          f"e.g. #{idx[~ok][:4]} step {s[~ok][:4]} candidate {cand[~ok][:4]}")
    assert idx.size <= max(8, max_tie_frac * tie.size), f"{what}: {idx.size} ties"
    return int(idx.size)


def parallel_chunks(fn, n, threads, chunk=16384):
    """Calls fn(lo, hi) over [0, n) in chunks on a thread pool (the oracle's
    ctypes calls release the GIL)."""
    spans = [(lo, min(n, lo + chunk)) for lo in range(0, n, chunk)]
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(lambda s: fn(*s), spans))


def nav_parity(orc, vol, tracks, step, hit, offsets=None, threads=16):
    """Every track of a basket against the oracle's long-double build: steps
    beyond 1e-12 and hit mismatches outside ties are classified by the
    ill-conditioning rules (on those tracks only), and ties are checked for
    a valid winner. Returns a report; ``not_exempt`` must be 0."""
    tracks = np.ascontiguousarray(tracks, np.float64)
    step = np.asarray(step, np.float64)
    hit = np.asarray(hit)
    n = tracks.shape[1]
    ref = np.empty(n)
    rhit = np.empty(n, np.int32)
    gap = np.empty(n)

    def run(lo, hi):
        s, h, g = orc.navigate(vol, np.ascontiguousarray(tracks[:, lo:hi]), offsets, "ld")
        ref[lo:hi], rhit[lo:hi], gap[lo:hi] = s, h, g

    parallel_chunks(run, n, threads)
    e = rel_diff(step, ref)
    tie = gap < TIE_GAP
    beyond = e > TOL
    hit_mis = (hit != rhit) & ~tie
    sus = np.nonzero(beyond | hit_mis)[0]
    rep = {"tracks": int(n), "reference": "oracle long-double build, every track",
           "max_rel_err": float(np.max(e[np.isfinite(e)])) if n else 0.0,
           "beyond_1e-12": int(beyond.sum()), "hit_mismatch_outside_ties": int(hit_mis.sum()),
           "exempt": 0, "exempt_double_vs_long_double": 0, "exempt_sensitivity_only": 0,
           "not_exempt": 0, "nan": int(np.isnan(step).sum())}
    exempt = np.zeros(n, bool)
    if sus.size:
        sub = np.ascontiguousarray(tracks[:, sus])
        _, ill = ill_conditioned(lambda t: orc.navigate(vol, t, offsets, "d")[0],
                                 lambda t: orc.navigate(vol, t, offsets, "ld")[0], sub)
        flag = np.asarray(ill, bool)
        exempt[sus[flag]] = True
        rep["exempt"] = int(flag.sum())
        rep["exempt_double_vs_long_double"] = int(ill.c15.sum())
        rep["exempt_sensitivity_only"] = int((flag & ~ill.c15).sum())
        rep["not_exempt"] = int((~flag).sum())
        rep["not_exempt_examples"] = [
            {"track": int(i), "gpu": float(step[i]), "ref": float(ref[i]), "hit": int(hit[i]),
             "ref_hit": int(rhit[i])} for i in sus[~flag][:4]]
    fin = np.isfinite(e) & ~exempt
    rep["max_rel_err_not_exempt"] = float(np.max(e[fin])) if fin.any() else 0.0
    rep["hit_ties"] = int(tie.sum())
    try:
        check_ties(orc, vol, tracks, step, hit, gap, offsets, max_tie_frac=1.0)
        rep["ties_invalid"] = 0
    except AssertionError as err:
        rep["ties_invalid"] = str(err)[:200]
    rep["ok"] = rep["not_exempt"] == 0 and rep["ties_invalid"] == 0 and rep["nan"] == 0
    return rep


def shape_parity(orc, kind, par, query, tracks, got, threads=16):
    """Every output of one shape query against the oracle's long-double
    build; Contains bit-exact except within 1e-9 of the surface, distances
    and Safety within 1e-12 except ill-conditioned tracks (classified on the
    tracks beyond the tolerance only). Returns a report; ``not_exempt`` must
    be 0."""
    tracks = np.ascontiguousarray(tracks, np.float64)
    n = tracks.shape[1]
    ref = np.empty(n, np.uint8 if query == 0 else np.float64)

    def run(lo, hi):
        ref[lo:hi] = orc.shape_query(kind, par, query, np.ascontiguousarray(tracks[:, lo:hi]), "ld")

    parallel_chunks(run, n, threads, chunk=65536)
    rep = {"tracks": int(n), "reference": "oracle long-double build, every output"}
    if query == 0:
        mis = np.nonzero(np.asarray(got) != ref)[0]
        near = (orc.safety(kind, par, np.ascontiguousarray(tracks[:, mis]), "ld") < 1e-9
                if mis.size else np.zeros(0, bool))
        rep.update({"mismatch": int(mis.size), "exempt": int(near.sum()), "not_exempt": int((~near).sum())})
    else:
        got = np.asarray(got, np.float64)
        e = rel_diff(got, ref)
        sus = np.nonzero(e > TOL)[0]
        rep.update({"max_rel_err": float(np.max(e[np.isfinite(e)])) if n else 0.0,
                    "beyond_1e-12": int(sus.size), "exempt": 0, "not_exempt": 0,
                    "nan": int(np.isnan(got).sum())})
        if sus.size:
            _, ill = ill_conditioned(lambda t: orc.shape_query(kind, par, query, t, "d"),
                                     lambda t: orc.shape_query(kind, par, query, t, "ld"),
                                     np.ascontiguousarray(tracks[:, sus]))
            rep["exempt"] = int(ill.sum())
            rep["exempt_double_vs_long_double"] = int(ill.c15.sum())
            rep["exempt_sensitivity_only"] = int((np.asarray(ill, bool) & ~ill.c15).sum())
            rep["not_exempt"] = int((~np.asarray(ill, bool)).sum())
    rep["ok"] = rep["not_exempt"] == 0 and rep.get("nan", 0) == 0
    return rep


def batched_parity(orc, wl, step, hit, threads=16):
    """nav_parity over a batched workload (every track of every basket),
    grouped by volume; returns the summed report."""
    step = np.asarray(step, np.float64)
    hit = np.asarray(hit)
    keys = ("tracks", "beyond_1e-12", "hit_mismatch_outside_ties", "exempt", "exempt_double_vs_long_double",
            "exempt_sensitivity_only", "not_exempt", "nan", "hit_ties")
    tot = {k: 0 for k in keys}
    tot.update({"reference": "oracle long-double build, every track", "max_rel_err": 0.0,
                "max_rel_err_not_exempt": 0.0, "ties_invalid": 0, "not_exempt_examples": []})
    bv = np.asarray(wl.basket_volume)
    for v in np.unique(bv):
        idx = np.concatenate([np.arange(int(wl.basket_offset[b]), int(wl.basket_offset[b] + wl.basket_n[b]))
                              for b in np.nonzero(bv == v)[0]])
        if idx.size == 0:
            continue
        rep = nav_parity(orc, wl.volumes[int(v)], np.ascontiguousarray(wl.tracks[:, idx]), step[idx], hit[idx],
                         threads=threads)
        for k in keys:
            tot[k] += rep[k]
        tot["max_rel_err"] = max(tot["max_rel_err"], rep["max_rel_err"])
        tot["max_rel_err_not_exempt"] = max(tot["max_rel_err_not_exempt"], rep["max_rel_err_not_exempt"])
        if rep["ties_invalid"]:
            tot["ties_invalid"] = rep["ties_invalid"]
        for ex in rep.get("not_exempt_examples", []):
            tot["not_exempt_examples"].append(dict(ex, track=int(idx[ex["track"]]), volume=int(v)))
    tot["ok"] = tot["not_exempt"] == 0 and tot["ties_invalid"] == 0 and tot["nan"] == 0
    return tot
