"""Closed forms used to pin the oracle (test helpers; no oracle or HIP code here)."""
import math

import numpy as np

from paper_1512_06637_amd import workloads as W

TWO_PI = 2.0 * math.pi


def analytic_volume(s) -> float:
    """Closed-form volumes (prismatoid / frustum formulas) used as Monte Carlo pins."""
    p = s.params
    if s.type == W.BOX:
        return 8.0 * p[0] * p[1] * p[2]
    if s.type == W.TUBS:
        return min(p[4], TWO_PI) * 0.5 * (p[1] ** 2 - p[0] ** 2) * 2 * p[2]
    if s.type == W.CONS:
        rmin1, rmax1, rmin2, rmax2, dz, _, dphi = p
        h = 2 * dz
        fr = lambda a, b: h / 3.0 * (a * a + a * b + b * b)
        return min(dphi, TWO_PI) / 2.0 * (fr(rmax1, rmax2) - fr(rmin1, rmin2))
    if s.type == W.SPHERE:
        return 4.0 / 3.0 * math.pi * (p[1] ** 3 - p[0] ** 3)
    if s.type == W.TRD:
        dx1, dx2, dy1, dy2, dz = p
        h = 2 * dz
        # prismatoid: V = h/6 (A1 + 4 Am + A2)
        A1 = 4 * dx1 * dy1
        A2 = 4 * dx2 * dy2
        Am = 4 * (0.5 * (dx1 + dx2)) * (0.5 * (dy1 + dy2))
        return h / 6.0 * (A1 + 4 * Am + A2)
    if s.type == W.PCON:
        zs, rmin, rmax = W.pcon_arrays(s)
        h = np.diff(zs)
        f = lambda r: np.pi * h / 3.0 * (r[:-1] ** 2 + r[:-1] * r[1:] + r[1:] ** 2)
        return float(np.sum(f(rmax) - f(rmin)))
    raise ValueError(s.type)


def slab_box(h, p, d, want_in):
    """Ray/box by the slab method (numpy, vectorised).  want_in: entry distance of
    outside points (+inf on a miss); else exit distance of inside points."""
    h = np.asarray(h, dtype=np.float64)[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (-h - p) / d
        t2 = (h - p) / d
    lo = np.where(d == 0, -np.inf, np.minimum(t1, t2))
    hi = np.where(d == 0, np.inf, np.maximum(t1, t2))
    # a zero direction component keeps the ray in the slab only if it already is
    lo = np.where((d == 0) & (np.abs(p) > h), np.inf, lo)
    tin = lo.max(axis=0)
    tout = hi.min(axis=0)
    if want_in:
        return np.where((tout > tin) & (tout > 0), np.maximum(tin, 0.0), np.inf)
    return np.maximum(tout, 0.0)


def fibonacci_dirs(n):
    i = np.arange(n) + 0.5
    ct = 1.0 - 2.0 * i / n
    st = np.sqrt(1.0 - ct * ct)
    ph = math.pi * (1.0 + 5 ** 0.5) * i
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct])
