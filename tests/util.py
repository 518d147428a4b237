"""Shared helpers for the test-suite (brute-force checks, fixtures)."""
from __future__ import annotations

import math
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BIG = 1e30


def load_closed_forms():
    """Rows of tests/golden/closed_forms.txt as
    (kind, par, query, p[3], d[3], expected, text). The cone segment (kind 4)
    has 7 parameters, the polycone (kind 5) 3 + 3 nz (phi1, dphi, nz, then
    z, rmin, rmax per plane), every other kind 5."""
    env = {"sqrt": math.sqrt, "min": min, "pi": math.pi}

    def num(tok):
        return float(eval(tok, {"__builtins__": {}}, env))

    out = []
    with open(os.path.join(GOLDEN_DIR, "closed_forms.txt")) as f:
        for raw in f:
            line = raw.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            kind = int(tok[0])
            npar = 7 if kind == 4 else (3 + 3 * int(tok[3]) if kind == 5 else 5)
            par = [num(v) for v in tok[1:1 + npar]]
            tok = tok[1 + npar:]
            q = int(tok[0])
            p = [num(v) for v in tok[1:4]]
            d = [num(v) for v in tok[4:7]]
            expr = "".join(tok[7:])
            val = BIG if expr == "BIG" else num(expr)
            out.append((kind, par, q, p, d, val, raw.strip()))
    return out


def fib_dirs(n: int) -> np.ndarray:
    """n quasi-uniform unit vectors (Fibonacci sphere), shape (3, n)."""
    i = np.arange(n) + 0.5
    ct = 1.0 - 2.0 * i / n
    st = np.sqrt(1.0 - ct * ct)
    ph = np.pi * (1.0 + 5 ** 0.5) * i
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct])


def rel_err(a, b, floor=1.0):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def to_local(vol, k, pts, offsets=None):
    """Mother-frame points (3, m) into daughter k's frame: R^T (p - T - delta)."""
    R = np.asarray(vol.rots[k], np.float64).reshape(3, 3)
    t = np.asarray(vol.trs[k], np.float64)
    if offsets is not None:
        t = t + np.asarray(offsets, np.float64).reshape(-1, 3)[k]
    return R.T @ (pts - t[:, None])


def first_transition(pred, p, d, tmax, step, want):
    """March t = 0, step, 2 step, ... along p + t d (p, d: (3,) arrays) and
    return the first sample t where pred(points (3, m)) == want, refined by
    bisection to ~1e-13, or None. pred returns a bool array."""
    ts = np.arange(0.0, tmax + step, step)
    pts = p[:, None] + ts[None, :] * d[:, None]
    v = pred(pts)
    idx = np.nonzero(v == want)[0]
    if idx.size == 0:
        return None
    j = int(idx[0])
    if j == 0:
        return 0.0
    lo, hi = ts[j - 1], ts[j]
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if bool(pred((p + mid * d)[:, None])[0]) == want:
            hi = mid
        else:
            lo = mid
    return hi
