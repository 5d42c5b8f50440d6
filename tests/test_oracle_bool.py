"""Pins of the oracle's composite (Boolean) solids against things other than the
oracle: closed forms of composites that reduce to textbook shapes (two boxes
sharing a face = one box, a box with a cylindrical hole, a sphere clipped by a
cube, a cube clipped by a rotated cube = an octagonal prism), Monte Carlo volume
against analytic volume, ray marching with a plain numpy membership test of the
composition, hand-placed asymmetric placements (a transposed rotation or a sign
error in the placement fails them), surface landing, and the safety bound.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1512_06637_amd import workloads as W
from tests import pins

U, S, I = W.UNION, W.SUBTRACTION, W.INTERSECTION


def rot_axis(axis, ang):
    a = np.asarray(axis, dtype=float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


COMPOSITES = W.composite_solids()
NAMES = list(COMPOSITES)


def box_tracks(s, n, seed):
    rng = np.random.default_rng(seed)
    c, h = W.solid_extent(s)
    P = W.uniform_box_points(rng, n, c, 1.6 * h)
    return W.Tracks(*P, *W.isotropic(rng, n))


def clean(diag):
    return (diag & O.D_DECIDE) == 0


# ------------------------------------------------------------------ parameters
def test_rejects_invalid_composites():
    a, c = W.box(1, 2, 3), W.tubs(0, 1, 2)
    assert O.solid_ok(W.boolean(U, a, c))
    bad_op = W.boolean(U, a, c)
    bad_op.params[0] = 3.0
    assert not O.solid_ok(bad_op)
    nested = W.Solid(W.BOOL, [0.0, float(W.BOOL), 3.0, 1.0, 1.0, 1.0] + [0.0, 3.0, 1, 1, 1] + list(np.eye(3).ravel())
                     + [0.0, 0.0, 0.0])
    assert not O.solid_ok(nested)
    shear = W.boolean(U, a, c, R=np.array([[1, 0.1, 0], [0, 1, 0], [0, 0, 1]]))
    assert not O.solid_ok(shear)
    short = W.boolean(U, a, c)
    short.params = short.params[:-1]
    assert not O.solid_ok(short)
    bad_part = W.boolean(U, a, W.box(1, -1, 1))
    assert not O.solid_ok(bad_part)


# ----------------------------------------------------------------- closed forms
def test_union_of_touching_boxes_is_one_box():
    """Two 20 mm cubes sharing the face x = 10 form the box 40 x 20 x 20 centred
    at x = 10: the shared face is no exit and no entry; distances equal the
    slab method's.  Points within 1e-6 of the shared face are left out of the
    code check (there the composite reports a surface point)."""
    s = COMPOSITES["box_u_box"]
    t = box_tracks(s, 20000, 1)
    P = np.stack([t.x, t.y, t.z])
    D = np.stack([t.dx, t.dy, t.dz])
    big = (20.0, 10.0, 10.0)
    Pc = P - np.array([[10.0], [0.0], [0.0]])
    code = O.inside(s, *P)
    ref = np.where(np.max(np.abs(Pc) - np.array(big)[:, None], axis=0) < 0, O.INSIDE, O.OUTSIDE)
    away = np.abs(np.abs(Pc) - np.array(big)[:, None]).min(axis=0) > 1e-6
    away &= np.abs(P[0] - 10.0) > 1e-6
    assert np.array_equal(code[away], ref[away])
    din, gi = O.distance(s, 0, t)
    dout, go = O.distance(s, 1, t)
    out, ins = (code == O.OUTSIDE) & clean(gi), (code == O.INSIDE) & clean(go)
    ri = pins.slab_box(big, Pc[:, out], D[:, out], True)
    ro = pins.slab_box(big, Pc[:, ins], D[:, ins], False)
    assert np.array_equal(np.isinf(din[out]), np.isinf(ri))
    f = np.isfinite(ri)
    assert np.all(np.abs(din[out][f] - ri[f]) <= 1e-12 * np.maximum(1.0, ri[f]))
    assert np.all(np.abs(dout[ins] - ro) <= 1e-12 * np.maximum(1.0, ro))
    # a ray along the axis through the shared face: one exit at the far end
    t1 = W.Tracks(*[np.array([v]) for v in (-5.0, 1.0, 2.0, 1.0, 0.0, 0.0)])
    assert O.distance(s, 1, t1)[0][0] == 35.0


def _cyl_roots(P, D, r):
    """Ray / infinite cylinder x^2 + y^2 = r^2 roots (t1 <= t2), NaN on a miss."""
    a = D[0] ** 2 + D[1] ** 2
    b = P[0] * D[0] + P[1] * D[1]
    c = P[0] ** 2 + P[1] ** 2 - r * r
    disc = b * b - a * c
    sq = np.sqrt(np.where(disc >= 0, disc, np.nan))
    with np.errstate(divide="ignore", invalid="ignore"):
        return (-b - sq) / a, (-b + sq) / a


def test_box_with_through_hole_closed_form():
    """20 mm cube minus a radius-5 cylinder through it along z.  From the wall,
    DistanceToOut = min(box slab exit, entry into the cylinder ahead).  From
    inside the hole, DistanceToIn = the cylinder exit if the ray is still
    within the cube's z range there, else the ray leaves through the open end
    and never enters."""
    s = COMPOSITES["box_minus_hole"]
    rng = np.random.default_rng(2)
    n = 20000
    P = rng.uniform(-19.9, 19.9, (3, n))
    D = np.stack(W.isotropic(rng, n))
    t = W.Tracks(*P, *D)
    r = np.hypot(P[0], P[1])
    code = O.inside(s, *P)
    wall, hole = r > 5.0 + 1e-6, r < 5.0 - 1e-6
    assert np.all(code[wall] == O.INSIDE) and np.all(code[hole] == O.OUTSIDE)
    dout, go = O.distance(s, 1, t)
    din, gi = O.distance(s, 0, t)
    t1, t2 = _cyl_roots(P, D, 5.0)
    box_exit = pins.slab_box((20.0, 20.0, 20.0), P, D, False)
    ahead = np.where((t1 > 0) & np.isfinite(t1), t1, np.inf)
    ref_out = np.minimum(box_exit, ahead)
    m = wall & clean(go)
    assert m.sum() > 10000
    assert np.all(np.abs(dout[m] - ref_out[m]) <= 1e-11 * np.maximum(1.0, ref_out[m]))
    zx = P[2] + t2 * D[2]
    ref_in = np.where(np.abs(zx) <= 20.0, t2, np.inf)
    m = hole & clean(gi) & (np.abs(np.abs(zx) - 20.0) > 1e-6)
    assert m.sum() > 500
    assert np.array_equal(np.isinf(din[m]), np.isinf(ref_in[m]))
    f = m & np.isfinite(ref_in)
    assert np.all(np.abs(din[f] - ref_in[f]) <= 1e-11 * np.maximum(1.0, ref_in[f]))


def _sphere_roots(P, D, R):
    b = np.sum(P * D, axis=0)
    c = np.sum(P * P, axis=0) - R * R
    disc = b * b - c
    sq = np.sqrt(np.where(disc >= 0, disc, np.nan))
    return -b - sq, -b + sq


def test_sphere_clipped_by_cube_closed_form():
    """Sphere r = 12 intersected with the 20 mm cube: both convex, so along a
    ray the composite is [max(entries), min(exits)]."""
    s = COMPOSITES["sphere_n_cube"]
    t = box_tracks(s, 20000, 3)
    P = np.stack([t.x, t.y, t.z])
    D = np.stack([t.dx, t.dy, t.dz])
    rho = np.sqrt(np.sum(P * P, axis=0))
    m_in = np.max(np.abs(P), axis=0)
    code = O.inside(s, *P)
    away = (np.abs(rho - 12.0) > 1e-6) & (np.abs(m_in - 10.0) > 1e-6)
    ref = np.where((rho < 12.0) & (m_in < 10.0), O.INSIDE, O.OUTSIDE)
    assert np.array_equal(code[away], ref[away])
    s1, s2 = _sphere_roots(P, D, 12.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        a1 = (-10.0 - P) / D
        a2 = (10.0 - P) / D
    b1 = np.max(np.minimum(a1, a2), axis=0)
    b2 = np.min(np.maximum(a1, a2), axis=0)
    lo = np.maximum(np.maximum(s1, b1), 0.0)
    hi = np.minimum(s2, b2)
    din, gi = O.distance(s, 0, t)
    dout, go = O.distance(s, 1, t)
    out = (code == O.OUTSIDE) & clean(gi) & away
    ref_in = np.where(hi - lo > 1e-9, lo, np.inf)
    assert np.array_equal(np.isinf(din[out]), np.isinf(ref_in[out]))
    f = out & np.isfinite(ref_in)
    assert f.sum() > 1000
    assert np.all(np.abs(din[f] - ref_in[f]) <= 1e-11 * np.maximum(1.0, ref_in[f]))
    ins = (code == O.INSIDE) & clean(go)
    assert ins.sum() > 3000
    assert np.all(np.abs(dout[ins] - hi[ins]) <= 1e-11 * np.maximum(1.0, hi[ins]))


# ----------------------------------------------------------------------- volume
def _volume(name):
    if name == "box_u_box":
        return 2 * 8000.0
    if name == "box_minus_hole":
        return 64000.0 - math.pi * 25.0 * 40.0
    if name == "sphere_n_cube":
        cap = math.pi * 4.0 * (36.0 - 2.0) / 3.0  # caps of height 2 beyond |x_i| = 10 are disjoint
        return 4.0 / 3.0 * math.pi * 12.0 ** 3 - 6 * cap
    if name == "cube_n_rot_cube":
        return 8 * 100.0 * math.tan(math.pi / 8) * 20.0  # regular octagon, inradius 10, height 20
    raise KeyError(name)


@pytest.mark.parametrize("name", ["box_u_box", "box_minus_hole", "sphere_n_cube", "cube_n_rot_cube"])
def test_monte_carlo_volume(name):
    s = COMPOSITES[name]
    rng = np.random.default_rng(7)
    c, h = W.solid_extent(s)
    n = 2_000_000
    P = W.uniform_box_points(rng, n, c, 1.25 * h)
    f = np.mean(O.inside(s, *P) != O.OUTSIDE)
    vbox = 8.0 * np.prod(1.25 * h)
    sigma = math.sqrt(f * (1 - f) / n) * vbox
    assert abs(f * vbox - _volume(name)) < 4.0 * sigma, (name, f * vbox, _volume(name), sigma)


# ------------------------------------------------------- placement and membership
@pytest.mark.parametrize("name", NAMES)
def test_codes_match_plain_membership(name):
    """Inside codes against the numpy membership of the composition (C's points
    mapped by R^T (x - t)), for points farther than 1e-5 mm from every
    component surface (checked by membership 1e-5 to either side along all
    three axes)."""
    s = COMPOSITES[name]
    t = box_tracks(s, 40000, 11)
    P = np.stack([t.x, t.y, t.z])
    code = O.inside(s, *P)
    m = W._member(s, P)
    far = np.ones(t.n, bool)
    _, a, c, R, tt = W.bool_parts(s)
    for part, Q in ((a, P), (c, R.T @ (P - tt[:, None]))):
        base = W._member(part, Q)
        for ax in range(3):
            for sg in (-1e-5, 1e-5):
                Q2 = Q.copy()
                Q2[ax] += sg
                far &= W._member(part, Q2) == base
    assert far.sum() > 30000
    ref = np.where(m, O.INSIDE, O.OUTSIDE)
    assert np.array_equal(code[far], ref[far]), name


def _first_change(s, p, d, start_in, h=2e-3, T=None):
    """First parameter where the plain membership of the composite differs from
    start_in, by stepping h then bisecting; +inf when it never does."""
    c, ext = W.solid_extent(s)
    T = T or (np.linalg.norm(p - c) + 2.5 * np.linalg.norm(ext))
    ts = np.arange(1, int(T / h) + 2) * h
    M = W._member(s, p[:, None] + ts[None, :] * d[:, None])
    k = np.nonzero(M != start_in)[0]
    if k.size == 0:
        return math.inf
    lo = ts[k[0] - 1] if k[0] > 0 else 0.0
    hi = ts[k[0]]
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        if W._member(s, (p + mid * d)[:, None])[0] != start_in:
            hi = mid
        else:
            lo = mid
    return hi


@pytest.mark.parametrize("name", NAMES)
def test_distances_match_membership_march(name):
    s = COMPOSITES[name]
    t = box_tracks(s, 150, 13)
    code = O.inside(s, t.x, t.y, t.z)
    din, gi = O.distance(s, 0, t)
    dout, go = O.distance(s, 1, t)
    checked = 0
    for i in range(t.n):
        p = np.array([t.x[i], t.y[i], t.z[i]])
        d = np.array([t.dx[i], t.dy[i], t.dz[i]])
        if code[i] == O.OUTSIDE and clean(gi[i]):
            ref = _first_change(s, p, d, False)
            if math.isinf(ref):
                assert math.isinf(din[i]), (name, i, din[i])
            else:
                assert abs(din[i] - ref) < 2e-6, (name, i, din[i], ref)
            checked += 1
        if code[i] == O.INSIDE and clean(go[i]):
            ref = _first_change(s, p, d, True)
            assert abs(dout[i] - ref) < 2e-6, (name, i, dout[i], ref)
            checked += 1
    assert checked > 100


@pytest.mark.parametrize("name", NAMES)
def test_surface_landing(name):
    s = COMPOSITES[name]
    t = box_tracks(s, 20000, 17)
    code = O.inside(s, t.x, t.y, t.z)
    for direction, side in ((0, O.OUTSIDE), (1, O.INSIDE)):
        dist, dg = O.distance(s, direction, t)
        m = (code == side) & np.isfinite(dist) & clean(dg)
        assert m.sum() > 200
        q = [a[m] + dist[m] * b[m] for a, b in ((t.x, t.dx), (t.y, t.dy), (t.z, t.dz))]
        assert np.all(O.inside(s, *q) == O.SURFACE), (name, direction)


# ----------------------------------------------------------------------- safety
@pytest.mark.parametrize("name", NAMES)
def test_safety_is_a_lower_bound(name):
    """Safety never exceeds the distance to the boundary along any of 256
    directions, and is positive off the surface."""
    s = COMPOSITES[name]
    t = box_tracks(s, 120, 19)
    code = O.inside(s, t.x, t.y, t.z)
    saf = O.safety(s, 0, t.x, t.y, t.z)
    dirs = pins.fibonacci_dirs(256)
    for i in range(t.n):
        if code[i] == O.SURFACE:
            assert saf[i] == 0.0
            continue
        assert saf[i] > 0.0
        P = np.repeat([[t.x[i]], [t.y[i]], [t.z[i]]], 256, axis=1)
        tr = W.Tracks(*P, *dirs)
        dist, _ = O.distance(s, 0 if code[i] == O.OUTSIDE else 1, tr)
        assert saf[i] <= dist.min() + 1e-9, (name, i, saf[i], dist.min())


def test_safety_exact_for_disjoint_sphere_union():
    """Outside two disjoint full spheres the distance to the union is the
    smaller of the two centre distances minus the radius; inside one of them
    it is that sphere's radius minus the centre distance."""
    s = W.boolean(U, W.sphere(0, 10), W.sphere(0, 6), R=rot_axis((1, 1, 0), 0.5), t=(30, 4, -2))
    rng = np.random.default_rng(23)
    P = rng.uniform(-15, 40, (3, 20000))
    d1 = np.sqrt(np.sum(P ** 2, axis=0))
    d2 = np.sqrt(np.sum((P - np.array([[30.0], [4.0], [-2.0]])) ** 2, axis=0))
    saf = O.safety(s, 0, *P)
    code = O.inside(s, *P)
    out = code == O.OUTSIDE
    ref = np.minimum(d1 - 10.0, d2 - 6.0)
    assert np.allclose(saf[out], ref[out], rtol=1e-13, atol=1e-12)
    in1 = (code == O.INSIDE) & (d1 < 10.0)
    assert in1.sum() > 100
    assert np.allclose(saf[in1], 10.0 - d1[in1], rtol=1e-13, atol=1e-12)
