"""Benchmark: batched navigator throughput on one MI355X.

One step = one geo_navigate_batched call over the batched workload: 512
baskets (sizes log-uniform in 32..65536 tracks) over 64 logical volumes,
each a box mother (200)^3 with 1..64 daughters (box/tube/cone) on a 4x4x4
grid (about 4.26M tracks, FP64). The step runs the whole navigator path:
basket load, geometry access, master-to-local transforms, every daughter's
DistFromOutside, the mother's DistFromInside, min/argmin and the outputs,
in one navigator launch after the kernel that expands the baskets into
tiles (the persistent kernel, or one wavefront per tile; the two kernels
launched one after the other or replayed from a cached HIP graph; whichever
the autotuner finds faster, the other submission timed beside it).

Clock ramp: the GPU reaches its full clock only after some tens of
milliseconds of sustained load, so before the W warmup steps and the K
timed steps the step runs back to back for a fixed wall time (RAMP_MS,
reported as ``clock_ramp_ms``); the timed steps follow at once.

Printed: one JSON line with tracks/s, the plain per-basket comparison (512
separate geo_navigate_basket launches doing the same work, issued one by one
and, beside that, captured in one HIP graph), the roofline of the dominant
kernel (the batched navigator: its algorithmic HBM bytes, 60 per track,
over its duration from HIP events recorded around the kernel; beside it the same with every cache flushed before each launch, the
counter traffic, the VALU issue and FP64 rates from the committed counter
summary, and the flops the kernel issues), the rows of the other hot-path
kernels, the CPU oracle timed on this host, and the parity of every output
of the headline step (and of the rows' workloads) against the oracle's
long-double build. The headline value is null unless that parity passes.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--copy-probe]
                       [--launch U,W[,graph|direct] | --no-autotune] [--no-rows] [--no-scan] [--no-plain]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "navigator tracks/sec at 1e-12 rel err (batched vs plain) + % HBM roofline"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6          # 256 CU x 64 FP64 FMA lanes x 2 flop x 2.4 GHz
FP64_LANE_PEAK = 256 * 64 * 2.4e9          # FP64 lane-instructions per second (39.3 T)
WAVE_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4      # wave64 VALU instructions per second (614 G):
                                           # one per SIMD every 4 cycles
BYTES_PER_TRACK = 60             # 6 x 8 B in (x, y, z, ux, uy, uz) + 8 B step + 4 B hit
# Estimated FP64 instructions per track of the dense navigator (every
# daughter evaluated): about 60 for the mother and the track, about 130 per
# daughter (transform, DistFromOutside with its divisions and square roots).
DENSE_FP64_BASE, DENSE_FP64_PER_DAUGHTER = 60, 130
RAMP_MS = 200.0                  # back-to-back steps before the timed region
FLUSH_BYTES = 1 << 30            # read between launches for the cold-cache timing
CPU_PASSES = 3                   # whole-workload passes of the oracle on all threads
PROFILE = "k_nav_tiles_batched512.md"

# Algorithmic FP64 operations of the navigator formulas (add, sub, mul, div,
# sqrt = 1 flop; fma = 2), counted from the per-lane algorithm. The work a
# launch does comes from the library's census (geo_navigate_batched_census):
# lane-evaluations per daughter kind, culling tests and tracks.
FLOPS_MOTHER_BOX = 6             # box DistFromInside: 3 x (sub, div)
FLOPS_TRACK_CULL = 24            # once per track: |d|^2 (5), 1 / |d| (sqrt, div), |p|^2 (5),
                                 # p.e with e = d / |d| (6), -2 p (3), -e (3)
FLOPS_CULL_TEST = 14             # (p - T).e (3 fma), |p|^2 - 2 p.T (3 fma), the half-line's
                                 # distance term (fma)
FLOPS_ROTATION = 30              # R^T w and R^T d (2 x 3 x (mul + 2 fma))
FLOPS_DIST_OUT = [               # census slot 2 * kind + hole
    21, 21,                      # box: 3 slab excesses + 3 faces x (div, mul, 2 fma)
    28, 37,                      # tube: r^2, z planes (10), A, B, outer (9) [, inner (9)]
    40, 55,                      # cone: r^2, radii, squares, z planes, outer (15) [, inner (15)]
    88, 107,                     # tube segment: tube + range tests of the start point and
                                 # of each base hit (6 each, 4 more for a nappe hit point)
                                 # + two face entries (19 each)
    112, 137,                    # cone segment: likewise, face entries 25 each
]
# polycone with ns sections (census slots 10..13: uncut, uncut with a hole,
# cut, cut with a hole): r^2 and the two end planes (22), per section the
# outer nappe entry (18) and, with a hole, the inner one (18); cut: range
# tests (6 + 6 per section) and the face entries (15 + 8 per section)
FLOPS_PCON_BASE, FLOPS_PCON_NAPPE = 22, 18
FLOPS_PCON_CUT_BASE, FLOPS_PCON_CUT_SECTION = 21, 14


def pcon_flops(ns: float, hole: bool, cut: bool) -> float:
    f = FLOPS_PCON_BASE + FLOPS_PCON_NAPPE * ns * (2 if hole else 1)
    return f + ((FLOPS_PCON_CUT_BASE + FLOPS_PCON_CUT_SECTION * ns) if cut else 0)


def census_flops(counts, cull: bool, pcon_sections: float = 0.0) -> float:
    """FP64 flops of one launch from its census counts; pcon_sections is the
    mean number of sections of the polycones evaluated."""
    from paper_1312_0816_amd import geonav as gv
    f = counts[gv.CENSUS_TRACKS] * (FLOPS_MOTHER_BOX + (FLOPS_TRACK_CULL if cull else 0))
    f += counts[gv.CENSUS_CULL] * FLOPS_CULL_TEST
    per_eval_extra = FLOPS_ROTATION + 3                    # w = p - T, then R^T w and R^T d
    for slot in range(len(FLOPS_DIST_OUT)):
        f += counts[slot] * (per_eval_extra + FLOPS_DIST_OUT[slot])
    for slot in range(10, 14):
        f += counts[slot] * (per_eval_extra + pcon_flops(pcon_sections, slot % 2 == 1, slot >= 12))
    return float(f)


def dense_fp64_instructions(wl) -> float:
    """Estimated FP64 lane-instructions of one dense (every daughter
    evaluated) pass over the batched workload."""
    nd = np.array([wl.volumes[int(v)].nd for v in wl.basket_volume], np.float64)
    return float(np.sum(np.asarray(wl.basket_n, np.float64) * (DENSE_FP64_BASE + DENSE_FP64_PER_DAUGHTER * nd)))


def _time_ms(fn, reps=10, warm=3):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def clock_ramp(fn, ms: float) -> float:
    """Runs fn back to back for about ms of wall time (checked every 8 calls
    against the device's progress); returns the wall time spent."""
    import torch
    t0 = time.perf_counter()
    while True:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()
        if (time.perf_counter() - t0) * 1e3 >= ms:
            return (time.perf_counter() - t0) * 1e3


def host_info() -> dict:
    """CPUs of this host as this process sees them."""
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cgroup_cpus": None,
            "model": None}
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            info["cgroup_cpus"] = int(q) / int(per)
    except (OSError, ValueError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def cpu_threads(info: dict) -> int:
    """Oracle threads: the CPUs this process may use, at most 16 (the host's
    share for one GPU)."""
    n = info["affinity"] or 1
    if info["cgroup_cpus"]:
        n = min(n, max(1, int(info["cgroup_cpus"])))
    return max(1, min(16, n))


def measure_rows(gv, W, dev, steps, scan=True):
    """The other rows of the hot path, each on its own workload (not part of
    the step above): the shape queries on the shape-suite distribution tiled
    to 2^26 tracks (3.2 GB, far above the 256 MB last-level cache), the plain
    navigator on the toy detector (2^22 tracks, 32 daughters), on the same
    tracks tiled to 2^26, on 2^22 tracks uniform in its mother with no
    rejection, and on the variant with every kind among the daughters, the
    navigator's safety and localization, and the adjoint on the toy detector
    (2^20 tracks). Returns (rows, outputs kept for the parity check)."""
    import torch
    rows, keep = {}, {}
    qbytes = {0: 25, 1: 32, 2: 56, 3: 56}
    qname = {0: "contains", 1: "safety", 2: "dist_in", 3: "dist_out"}
    shapes = {}
    for kind in (W.BOX, W.TUBE, W.CONE, W.TUBS, W.CONS, W.PCON):
        _, par, tr = W.shape_suite_c1(kind)
        m = tr.shape[1]
        big = torch.from_numpy(tr).to(dev).repeat(1, 64).contiguous()   # 2^26 tracks
        n = big.shape[1]
        outs = {0: torch.empty(n, dtype=torch.uint8, device=dev),
                1: torch.empty(n, dtype=torch.float64, device=dev)}
        res, got = {}, {}
        for q in (0, 1, 2, 3):
            out = outs[0] if q == 0 else outs[1]
            ms = _time_ms(lambda: gv.geo_shape_query(kind, par, q, big, out))
            gbs = qbytes[q] * n / (ms * 1e-3) / 1e9
            res[qname[q]] = {"ms": ms, "tracks_per_s": n / (ms * 1e-3), "GBps": gbs,
                             "hbm_frac": gbs / HBM_PEAK_GBS}
            got[q] = out[:m].cpu().numpy()          # the first copy: the 2^20-track suite
        shapes[W.KIND_NAMES[kind]] = res
        keep[("shape", kind)] = (par, tr, got)
        del big, outs
        torch.cuda.empty_cache()
    rows["shape_queries_2^26"] = shapes

    def basket_row(vol, tr, name, tile=1):
        g = gv.Geometry([vol])
        t = torch.from_numpy(tr).to(dev)
        if tile > 1:
            t = t.repeat(1, tile).contiguous()
        n = t.shape[1]
        step = torch.empty(n, dtype=torch.float64, device=dev)
        hit = torch.empty(n, dtype=torch.int32, device=dev)
        trs, sp, hp = gv.tracks_struct(t), gv._ptr(step), gv._ptr(hit)
        lib, hs = g._lib, gv._stream()
        run = lambda: gv._check(lib.geo_navigate_basket(g.handle, 0, trs, None, sp, hp, None, hs))  # noqa: E731
        clock_ramp(run, 50.0)
        ms = _time_ms(run)
        gbs = BYTES_PER_TRACK * n / (ms * 1e-3) / 1e9
        row = {"ms": ms, "tracks_per_s": n / (ms * 1e-3), "GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
               "tracks": n}
        m = tr.shape[1]
        out = (step[:m].cpu().numpy(), hit[:m].cpu().numpy())
        if tile == 1:
            _, _, counts = gv.geo_navigate_batched_census(g, [0], [0], [n], t)
            row["evaluated_fraction"] = sum(counts[:14]) / max(1, counts[gv.CENSUS_CULL])
            row["evaluated_pairs_per_track"] = sum(counts[:14]) / n
        rows[name] = row
        return g, t, out

    vol, tr = W.toy_detector_c2()
    g, t, out = basket_row(vol, tr, "navigator_toy_detector_2^22")
    keep["toy"] = (vol, tr) + out
    n = t.shape[1]
    trs, lib, hs = gv.tracks_struct(t), g._lib, gv._stream()
    saf = torch.empty(n, dtype=torch.float64, device=dev)
    loc = torch.empty(n, dtype=torch.int32, device=dev)
    ms_s = _time_ms(lambda: gv._check(lib.geo_navigate_safety(g.handle, 0, trs, None, gv._ptr(saf), hs)))
    ms_l = _time_ms(lambda: gv._check(lib.geo_locate(g.handle, 0, trs, None, gv._ptr(loc), hs)))
    rows["navigator_safety_toy_detector_2^22"] = {"ms": ms_s, "points_per_s": n / (ms_s * 1e-3),
                                                  "GBps": 32 * n / (ms_s * 1e-3) / 1e9}
    rows["locate_toy_detector_2^22"] = {"ms": ms_l, "points_per_s": n / (ms_l * 1e-3),
                                        "GBps": 28 * n / (ms_l * 1e-3) / 1e9}
    g.close()
    del t, saf, loc
    g, t, _ = basket_row(vol, tr, "navigator_toy_detector_2^26_oversized", tile=16)
    rows["navigator_toy_detector_2^26_oversized"]["note"] = (
        "the 2^22 toy-detector tracks tiled 16 times: 2^26 tracks, 4.0 GB moved per launch, "
        "16x the 256 MB last-level cache")
    g.close()
    del t
    torch.cuda.empty_cache()
    tru = W.tracks_uniform_in_mother(np.random.default_rng(1280), vol, 1 << 22)
    g, t, out = basket_row(vol, tru, "navigator_toy_detector_uniform_in_mother_2^22")
    keep["toy_uniform"] = (vol, tru) + out
    g.close()
    del t

    mix = W.mixed_detector_volume()
    trm = W.tracks_in_mother(np.random.default_rng(1270), mix, 1 << 22)
    g, t, out = basket_row(mix, trm, "navigator_mixed_detector_2^22")
    keep["mixed"] = (mix, trm) + out
    rows["navigator_mixed_detector_2^22"]["daughters"] = ("32: box, tube, cone, tube segment, cone segment, "
                                                          "polycone in turn")
    g.close()
    del t

    vola, tra, tgt = W.adjoint_c4()
    g = gv.Geometry([vola])
    n = tra.shape[1]
    o = torch.from_numpy(np.ascontiguousarray(tra[:3])).to(dev)
    d = torch.from_numpy(np.ascontiguousarray(tra[3:])).to(dev)
    gh = torch.from_numpy(np.ascontiguousarray(tgt)).to(dev)
    offs = torch.zeros((vola.nd, 3), dtype=torch.float64, device=dev)
    ms = _time_ms(lambda: gv.geo_navigate_backward(g, 0, o, d, offs, None, gh))
    rows["adjoint_toy_detector_2^20"] = {"ms": ms, "tracks_per_s": n / (ms * 1e-3),
                                        "GBps": 128 * n / (ms * 1e-3) / 1e9,
                                        "outputs": "g_o, g_d (3 x n) and g_off (32 x 3)"}
    g.close()
    del o, d, gh
    if scan:
        rows["paper_toy_detector_basket_scan"] = basket_scan(gv, W, dev)
    return rows, keep


SCAN_TOTAL = 1 << 20


def basket_scan(gv, W, dev):
    """The paper's benchmark protocol on its toy detector: P baskets of N
    consecutive particles from a random start in a 2^20-track pool, N x P =
    2^20 fixed; runtime per particle for one launch per basket and for all
    baskets in one batched launch (N x P = 2^20), in pool order (neighbouring
    baskets are joined into full wavefronts) and in a random order (each
    basket tiled on its own)."""
    import torch
    vol = W.paper_toy_detector()
    pool = W.paper_toy_tracks(n=1 << 21)
    g = gv.Geometry([vol])
    t = torch.from_numpy(pool).to(dev)
    n = t.shape[1]
    step = torch.empty(n, dtype=torch.float64, device=dev)
    hit = torch.empty(n, dtype=torch.int32, device=dev)
    lib, hs = g._lib, gv._stream()
    tr = gv.tracks_struct(t)
    start = 0 if n == SCAN_TOTAL else int(np.random.default_rng(1501).integers(0, n - SCAN_TOTAL))
    out = {}
    for N in (16, 64, 256, 1024, 4096, 16384, 65536):
        P = SCAN_TOTAL // N
        offs = start + N * np.arange(P)
        barr, nb = gv._baskets(np.zeros(P, np.int32), offs, np.full(P, N))
        sp, hp = gv._ptr(step), gv._ptr(hit)
        # 20 warmup calls: the first call of each of the library's 16 staging
        # buffers grows it to this basket count
        ms_b = _time_ms(lambda: gv._check(lib.geo_navigate_batched(g.handle, barr, nb, tr, sp, hp, hs)),
                        reps=10, warm=20)
        # the same baskets in a random order: no two neighbours in the list
        # follow one another in the pool, so none is joined to the next and
        # every basket's last wavefront runs part empty
        perm = np.random.default_rng(1502 + N).permutation(P)
        barr_s, nb_s = gv._baskets(np.zeros(P, np.int32), offs[perm], np.full(P, N))
        ms_s = _time_ms(lambda: gv._check(lib.geo_navigate_batched(g.handle, barr_s, nb_s, tr, sp, hp, hs)),
                        reps=10, warm=20)
        plain = [(gv.GeoTracks(tr.x + 8 * o, tr.y + 8 * o, tr.z + 8 * o, tr.ux + 8 * o, tr.uy + 8 * o,
                               tr.uz + 8 * o, N),
                  gv.C.c_void_p(step.data_ptr() + 8 * o), gv.C.c_void_p(hit.data_ptr() + 4 * o))
                 for o in (int(v) for v in offs)]

        def run_plain():
            for tb, s_, h_ in plain:
                gv._check(lib.geo_navigate_basket(g.handle, 0, tb, None, s_, h_, None, hs))

        ms_p = _time_ms(run_plain, reps=1 if P > 1024 else 3, warm=1 if P <= 4096 else 0)
        out[str(N)] = {"baskets": P,
                       "batched_ns_per_particle": ms_b * 1e6 / SCAN_TOTAL,
                       "batched_shuffled_ns_per_particle": ms_s * 1e6 / SCAN_TOTAL,
                       "per_basket_launches_ns_per_particle": ms_p * 1e6 / SCAN_TOTAL}
    g.close()
    return out


def kernel_source_digest() -> str:
    """Digest of the device code (comments and layout stripped), naming the
    kernel source a committed counter summary was taken on."""
    import re
    h = hashlib.sha256()
    for f in ("geonav_device.hpp", "geonav_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1312_0816_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def read_profile(tag: str, digest: str, launch: str, field: str, name: str = PROFILE):
    """A figure from the committed rocprofv3 summary profiles/<name>: the
    `field` of the line `<tag>: kernel_source=<digest> launch=<launch> ...`,
    if one was taken on this kernel source and launch shape, else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if not line.startswith(tag + ":"):
                continue
            vals = dict(kv.split("=", 1) for kv in line.split()[1:] if "=" in kv)
            if vals.get("kernel_source") == digest and vals.get("launch") == launch:
                try:
                    return float(vals[field])
                except (KeyError, ValueError):
                    return None
    return None


def read_traffic(digest: str, launch: str):
    """HBM bytes per launch of the batched kernel (FETCH_SIZE + WRITE_SIZE,
    calibrated on a device copy) from the committed counter summary."""
    return read_profile("traffic", digest, launch, "bytes_per_launch")


def oracle_leg(wl, gpu_step, gpu_hit, info, keep, unrejected):
    """The CPU side: the oracle (double build, as it stands) timed over the
    whole batched workload on all of this host's threads and on one thread,
    and the parity of every GPU output against the oracle's long-double
    build (the headline step; the rows' workloads when measured)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from tests.parity import batched_parity, nav_parity, shape_parity

    oracle._load()
    threads = cpu_threads(info)
    jobs = []
    for b in range(len(wl.basket_n)):
        o, m = int(wl.basket_offset[b]), int(wl.basket_n[b])
        for s in range(0, m, 16384):
            jobs.append((int(wl.basket_volume[b]), o + s, min(16384, m - s)))
    n = int(wl.tracks.shape[1])

    def run(job):
        v, o, m = job
        oracle.navigate(wl.volumes[v], np.ascontiguousarray(wl.tracks[:, o:o + m]), None, "d")

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for _ in range(CPU_PASSES):
            list(ex.map(run, jobs))
    dt = (time.perf_counter() - t0) / CPU_PASSES
    t0 = time.perf_counter()
    for job in jobs:
        run(job)
    dt1 = time.perf_counter() - t0
    base = {"value": n / dt, "unit": "tracks/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole batched workload ({n} tracks, {len(wl.basket_n)} baskets), oracle double "
                      f"build: {CPU_PASSES} passes on {threads} threads ({dt:.2f} s per pass) and one pass "
                      f"on one thread ({dt1:.2f} s)",
            "one_thread_value": n / dt1, "host": info}
    # the sequential (one particle at a time) navigator of Fig. 1a on the
    # paper's toy detector, one thread: the analogue of the paper's scalar
    # baseline in its basket-size scan
    from paper_1312_0816_amd import workloads as W
    vol = W.paper_toy_detector()
    sub = np.ascontiguousarray(W.paper_toy_tracks()[:, :SCAN_TOTAL])
    t0 = time.perf_counter()
    oracle.navigate(vol, sub, None, "d")
    base["paper_toy_detector_1thread_ns_per_particle"] = (time.perf_counter() - t0) * 1e9 / SCAN_TOTAL

    parity = batched_parity(oracle, wl, gpu_step, gpu_hit, threads=threads)
    rows = {}
    if unrejected is not None:
        wlu, su, hu = unrejected
        rows["batched_uniform_in_mother"] = batched_parity(oracle, wlu, su, hu, threads=threads)
    for key, val in keep.items():
        if isinstance(key, tuple) and key[0] == "shape":
            par, tr, got = val
            name = W.KIND_NAMES[key[1]]
            for q, out in got.items():
                rows[f"shape_suite_{name}_q{q}"] = shape_parity(oracle, key[1], par, q, tr, out, threads)
        elif key in ("toy", "toy_uniform", "mixed"):
            v, tr, s, h = val
            name = {"toy": "navigator_toy_detector_2^22",
                    "toy_uniform": "navigator_toy_detector_uniform_in_mother_2^22",
                    "mixed": "navigator_mixed_detector_2^22"}[key]
            rows[name] = nav_parity(oracle, v, tr, s, h, threads=threads)
    for r in list(rows.values()) + [parity]:
        if not r.get("not_exempt"):
            r.pop("not_exempt_examples", None)
    return base, parity, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and the parity check")
    ap.add_argument("--no-rows", action="store_true", help="skip the per-row measurements")
    ap.add_argument("--no-scan", action="store_true",
                    help="skip the basket-size scan among the rows (tens of thousands of launches)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip timing the plain per-basket form (for profiling the batched kernel)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch", default=None,
                    help="force the batched launch shape 'tracks_per_lane,waves_per_simd' (no autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the navigator has no multi-GPU path (tracks "
              "are independent, so each GPU would take its own share of the baskets); run "
              "with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1312_0816_amd import geonav as gv
    from paper_1312_0816_amd import workloads as W

    gv.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    info = host_info()

    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    wl = W.batched_c3()
    n = int(wl.tracks.shape[1])
    g = gv.Geometry(wl.volumes)
    t = torch.from_numpy(wl.tracks).to(dev)
    step = torch.empty(n, dtype=torch.float64, device=dev)
    hit = torch.empty(n, dtype=torch.int32, device=dev)
    bv, bo, bn = wl.basket_volume, wl.basket_offset, wl.basket_n

    if args.launch:
        parts = args.launch.split(",")
        g.set_launch_config(int(parts[0]), int(parts[1]))
        if len(parts) > 2:
            g.batched_graph = parts[2] == "graph"
    elif not args.no_autotune:
        gv.geo_autotune(g, bv, bo, bn, t)
    U, Wv = g.launch_config()
    use_graph = g.batched_graph

    # Host-side call arguments are marshalled once; each step is then one C
    # call (batched) or one C call per basket (plain), on torch's stream.
    lib = g._lib
    hs = gv._stream()
    barr, nb = gv._baskets(bv, bo, bn)
    tr_all = gv.tracks_struct(t)
    sp, hp = gv._ptr(step), gv._ptr(hit)

    def batched_step():
        gv._check(lib.geo_navigate_batched(g.handle, barr, nb, tr_all, sp, hp, hs))

    # plain form: one launch per basket on the same pool, outputs at the same
    # positions
    pstep = torch.empty(n, dtype=torch.float64, device=dev)
    phit = torch.empty(n, dtype=torch.int32, device=dev)
    plain = []
    for b in range(len(bn)):
        o, m = int(bo[b]), int(bn[b])
        if m == 0:
            continue
        tb = gv.GeoTracks(*[tr_all.x + 8 * o, tr_all.y + 8 * o, tr_all.z + 8 * o,
                            tr_all.ux + 8 * o, tr_all.uy + 8 * o, tr_all.uz + 8 * o], m)
        plain.append((int(bv[b]), tb, gv.C.c_void_p(pstep.data_ptr() + 8 * o),
                      gv.C.c_void_p(phit.data_ptr() + 4 * o)))

    def plain_step():
        for v, tb, s_, h_ in plain:
            gv._check(lib.geo_navigate_basket(g.handle, v, tb, None, s_, h_, None, hs))

    # one step of each form: the batched result must equal the plain one bit
    # for bit
    batched_step()
    plain_step()
    torch.cuda.synchronize()
    same = bool(torch.equal(step.view(torch.int64), pstep.view(torch.int64)) and torch.equal(hit, phit))

    # work census of one launch (instrumented variant, outside the timed region)
    _, _, counts = gv.geo_navigate_batched_census(g, bv, bo, bn, t)

    # clock ramp, then W warmup steps, then the K timed steps at once. HIP
    # events on the launch stream bracket the timed region (one pair, so that
    # no per-step event packets sit between the launches).
    ramp_ms = clock_ramp(batched_step, RAMP_MS)
    for _ in range(args.warmup):
        batched_step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        batched_step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1) / args.steps
    ms_per_step = 1e3 * wall / args.steps
    out_step, out_hit = step.cpu().numpy(), hit.cpu().numpy()

    # the navigator kernel alone: events recorded right before and after it
    # (on the stream, or as nodes of the graph; the tile expansion and the
    # gaps between calls fall outside), read after each launch
    k_launches = max(args.steps, 100)
    g.set_kernel_timing(True)
    clock_ramp(batched_step, 50.0)
    kms = []
    for _ in range(k_launches):
        batched_step()
        kms.append(g.batched_kernel_ms())
    kernel_ms = float(np.mean(kms))
    # the same with every cache flushed first: a 1 GiB read between launches
    # evicts the workload (255 MB) from L2 and the 256 MB last-level cache,
    # so the kernel reads its tracks from HBM (a read leaves clean lines: a
    # write would charge the kernel for writing the flush buffer back)
    flush = torch.ones(FLUSH_BYTES // 8, dtype=torch.float64, device=dev)
    kms_cold = []
    for _ in range(min(k_launches, 50)):
        flush.sum()
        batched_step()
        kms_cold.append(g.batched_kernel_ms())
    del flush
    kernel_ms_cold = float(np.mean(kms_cold))

    # the same batched launch without culling (every daughter of every track
    # evaluated), for the record: its kernel time from the same events
    g.culling = False
    _, _, counts_nocull = gv.geo_navigate_batched_census(g, bv, bo, bn, t)
    batched_step()
    kms_nc = []
    for _ in range(20):
        batched_step()
        kms_nc.append(g.batched_kernel_ms())
    nocull_kernel_ms = float(np.mean(kms_nc))
    g.set_kernel_timing(False)
    clock_ramp(batched_step, 20.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched_step()
    torch.cuda.synchronize()
    nocull_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    g.culling = True
    batched_step()

    # the other submission of the two kernels (a graph replay instead of two
    # launches, or the reverse), for the record
    g.batched_graph = not use_graph
    clock_ramp(batched_step, 20.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched_step()
    torch.cuda.synchronize()
    other_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    g.batched_graph = use_graph
    batched_step()

    # timed: plain per-basket launches (after W warmup steps of their own)
    plain_ms = None
    if not args.no_plain:
        for _ in range(max(args.warmup, 5)):
            plain_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plain_step()
        torch.cuda.synchronize()
        plain_ms = 1e3 * (time.perf_counter() - t0) / args.steps

    # the plain form with its launches captured in one HIP graph and the
    # graph replayed once per step: the per-basket kernels without the
    # host's cost of 512 launches
    plain_graph_ms, plain_graph_same = None, None
    if not args.no_plain:
        cg = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(stream)
        with torch.cuda.graph(cg, stream=cs):
            hcap = gv._stream(cs)
            for v, tb, s_, h_ in plain:
                gv._check(lib.geo_navigate_basket(g.handle, v, tb, None, s_, h_, None, hcap))
        stream.wait_stream(cs)
        pstep.fill_(-1.0)
        phit.fill_(-2)
        cg.replay()
        torch.cuda.synchronize()
        plain_graph_same = bool(torch.equal(step.view(torch.int64), pstep.view(torch.int64))
                                and torch.equal(hit, phit))
        for _ in range(max(args.warmup, 5)):
            cg.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            cg.replay()
        torch.cuda.synchronize()
        plain_graph_ms = 1e3 * (time.perf_counter() - t0) / args.steps
        plain_graph_same = plain_graph_same and bool(
            torch.equal(step.view(torch.int64), pstep.view(torch.int64)) and torch.equal(hit, phit))
        del cg

    # culling where it is weakest: the same geometry and basket sizes with
    # tracks uniform in each mother (no rejection: some start inside a
    # daughter, many close to one)
    unrejected, unrej_row = None, None
    if not args.no_rows:
        wlu = W.batched_c3(reject=False)
        tu = torch.from_numpy(wlu.tracks).to(dev)
        su = torch.empty(n, dtype=torch.float64, device=dev)
        hu = torch.empty(n, dtype=torch.int32, device=dev)
        tru, spu, hpu = gv.tracks_struct(tu), gv._ptr(su), gv._ptr(hu)
        ustep = lambda: gv._check(lib.geo_navigate_batched(g.handle, barr, nb, tru, spu, hpu, hs))  # noqa: E731
        clock_ramp(ustep, 50.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ustep()
        torch.cuda.synchronize()
        ums = 1e3 * (time.perf_counter() - t0) / args.steps
        _, _, ucounts = gv.geo_navigate_batched_census(g, bv, bo, bn, tu)
        unrej_row = {"value": n / (ums * 1e-3), "unit": "tracks/s", "ms_per_step": ums,
                     "evaluated_pairs_per_track": sum(ucounts[:14]) / n,
                     "headline_evaluated_pairs_per_track": sum(counts[:14]) / n}
        unrejected = (wlu, su.cpu().numpy(), hu.cpu().numpy())
        del tu, su, hu

    value = n / (ms_per_step * 1e-3)
    digest = kernel_source_digest()
    launch = f"{U},{Wv}"
    traffic = read_traffic(digest, launch)
    hbm_gbs = BYTES_PER_TRACK * n / (kernel_ms * 1e-3) / 1e9
    hbm_cold = BYTES_PER_TRACK * n / (kernel_ms_cold * 1e-3) / 1e9
    flops = census_flops(counts, True)
    flops_nocull = census_flops(counts_nocull, False)
    valu = read_profile("valu", digest, launch, "valu_per_launch")
    f64 = read_profile("valu", digest, launch, "f64_per_launch")
    f64_nc = read_profile("valu", digest, launch + ",nocull", "f64_per_launch")
    dense = dense_fp64_instructions(wl)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "tracks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "clock_ramp_ms": ramp_ms,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"batched navigation: {len(bn)} baskets (32-65536 tracks, log-uniform) over "
                        f"{len(wl.volumes)} volumes (box mother (200)^3, 1-64 box/tube/cone daughters), "
                        f"{n} tracks, FP64, one navigator launch",
            "baskets": int(len(bn)), "volumes": int(len(wl.volumes)), "tracks": n,
            "launch": {"tracks_per_lane": U, "waves_per_simd": Wv, "graph": bool(use_graph),
                       "autotuned": not (args.no_autotune or args.launch)},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_nav_persistent" if Wv > 0 else "k_nav_tiles") + f"<{U}, cull>",
            "achieved": hbm_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hbm_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_track": BYTES_PER_TRACK,
            "tracks_per_launch": n,
            "kernel_ms_per_launch": kernel_ms,
            "timing": f"HIP events recorded around the navigator kernel, mean over {k_launches} launches",
            "cold_caches": {"kernel_ms_per_launch": kernel_ms_cold, "achieved": hbm_cold,
                            "frac": hbm_cold / HBM_PEAK_GBS,
                            "timing": f"the same events, a 1 GiB read before each of {len(kms_cold)} launches"},
            "graph_launch_ms": float(ev_ms),
            "achieved_over_graph_launch": BYTES_PER_TRACK * n / (ev_ms * 1e-3) / 1e9,
            "valu_issue": None if valu is None else {
                "wave_instructions_per_launch": valu, "issue_frac": valu / (kernel_ms * 1e-3) / WAVE_ISSUE_PEAK,
                "fp64_lane_instructions_per_launch": f64 * 64,
                "fp64_frac": f64 * 64 / (kernel_ms * 1e-3) / FP64_LANE_PEAK,
                "source": f"profiles/{PROFILE} (rocprofv3 SQ counters on this kernel source)"},
            "issued_flops": {"flops_per_launch": flops, "TFLOPs": flops / (kernel_ms * 1e-3) / 1e12,
                             "issued_flops_frac": flops / (kernel_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                             "note": "FP64 flops the culled kernel issues, counted from its census"},
            "dense_fp64": {
                "estimated_lane_instructions_per_launch": dense,
                "note": "the dense navigator's estimated FP64 instructions (60 + 130 per daughter per "
                        "track) over each kernel's time; the culled kernel evaluates a fraction of the pairs",
                "frac_at_culled_kernel_time": dense / (kernel_ms * 1e-3) / FP64_LANE_PEAK,
                "unculled_kernel_ms": nocull_kernel_ms,
                "frac_at_unculled_kernel_time": dense / (nocull_kernel_ms * 1e-3) / FP64_LANE_PEAK,
                "unculled_measured_fp64_lane_instructions_per_launch": None if f64_nc is None else f64_nc * 64,
                "unculled_measured_fp64_frac": None if f64_nc is None else
                f64_nc * 64 / (nocull_kernel_ms * 1e-3) / FP64_LANE_PEAK},
        },
        "plain_per_basket": None if plain_ms is None else {
            "value": n / (plain_ms * 1e-3), "unit": "tracks/s", "ms_per_step": plain_ms,
            "launches": len(plain)},
        "batched_over_plain": None if plain_ms is None else plain_ms / ms_per_step,
        "plain_per_basket_graph": None if plain_graph_ms is None else {
            "value": n / (plain_graph_ms * 1e-3), "unit": "tracks/s", "ms_per_step": plain_graph_ms,
            "launches": len(plain), "equals_batched_bitwise": plain_graph_same},
        "batched_over_plain_graph": None if plain_graph_ms is None else plain_graph_ms / ms_per_step,
        "batched_without_culling": {"value": n / (nocull_ms * 1e-3), "unit": "tracks/s",
                                    "ms_per_step": nocull_ms, "kernel_ms": nocull_kernel_ms,
                                    "flops_per_launch": flops_nocull},
        "batched_other_submission": {"graph": not use_graph, "value": n / (other_ms * 1e-3), "unit": "tracks/s",
                                     "ms_per_step": other_ms},
        "batched_uniform_in_mother": unrej_row,
        "census": {"evaluations_by_kind_hole": counts[:14], "cull_tests": counts[gv.CENSUS_CULL],
                   "tracks": counts[gv.CENSUS_TRACKS],
                   "evaluations_without_culling": int(sum(counts_nocull[:14]))},
        "batched_equals_plain_bitwise": same,
        "kernel_source": digest,
    }
    g.close()
    del t, step, hit, pstep, phit
    torch.cuda.empty_cache()
    keep = {}
    if not args.no_rows:
        out["rows"], keep = measure_rows(gv, W, dev, args.steps, scan=not args.no_scan)
    if not args.no_cpu:
        base, parity, parity_rows = oracle_leg(wl, out_step, out_hit, info, keep, unrejected)
        out["cpu_baseline"] = base
        out["parity"] = parity
        out["parity_rows"] = parity_rows
        out["parity_ok"] = bool(parity["ok"] and all(r["ok"] for r in parity_rows.values()))
        if not parity["ok"]:
            out["value_unchecked"] = out["value"]
            out["value"] = None      # throughput counts only when the step's parity passes
    else:
        out["cpu_baseline"] = None
        out["parity"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
