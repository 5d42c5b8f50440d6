"""GPU parity of the solid-level queries (basket_inside / basket_safety /
basket_distance / basket_solid_all) against the CPU oracle, element by element.

Bar: Inside codes bit-exact; FP64 distances and safeties within 1e-12 relative
(1 mm floor) with exact sentinels; tracks the oracle marks ill-conditioned
(including hits whose FP64 conditioning exceeds the bar) are listed in the
session summary and not counted."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1512_06637_amd import workloads as W
from tests.gpu_util import compare_values, cuda, host, say

pytestmark = pytest.mark.gpu

EXTRA = {
    "pcon_hollow": W.config_solids(hollow_pcon=True)["pcon"],
    "cons_seg": W.cons(2.0, 8.0, 4.0, 12.0, 25.0, 0.3, 1.5 * math.pi),
    "tubs_narrow": W.tubs(0.0, 15.0, 20.0, -0.4, 0.7 * math.pi),
    "sphere_full": W.sphere(0.0, 30.0),
    "tubs_half": W.tubs(2.0, 15.0, 20.0, 0.25, math.pi),
    "tubs_hollow_full": W.tubs(3.0, 12.0, 10.0),
}
SOLIDS = dict(W.config_solids(), **EXTRA)
NAMES = list(SOLIDS)
N_SMALL = (1 << 16) + 37  # several tiles of 256 lanes plus a ragged tail


@pytest.fixture(scope="module")
def geo():
    import paper_1512_06637_amd as G
    g = G.Geometry(W.multi_solid_blob([SOLIDS[k] for k in NAMES]))
    yield g
    g.close()


def mixed_tracks(name, n):
    """Thirds inside / outside / within 1e-6 mm of the surface, isotropic."""
    s = SOLIDS[name]
    rng = np.random.default_rng(77 + NAMES.index(name))
    k = n // 3
    pin = W.sample_volume(s, rng, k)
    pout = W.sample_outside(s, rng, k)
    ps, nrm = W.sample_surface(s, rng, n - 2 * k)
    ps = ps + nrm * rng.uniform(-1e-6, 1e-6, n - 2 * k)[None, :]
    P = np.concatenate([pin, pout, ps], axis=1)[:, rng.permutation(n)]
    return W.Tracks(*P, *W.isotropic(rng, n))


def run_all(g, lv, t):
    import torch
    a = [cuda(v) for v in t.arrays()]
    res = {
        "inside": host(g.inside(lv, *a[:3])),
        "safety": host(g.safety(lv, *a[:3])),
        "s_in": host(g.safety(lv, *a[:3], side=1)),
        "s_out": host(g.safety(lv, *a[:3], side=2)),
        "din": host(g.distance(lv, 0, *a)),
        "dout": host(g.distance(lv, 1, *a)),
    }
    torch.cuda.synchronize()
    return res


def check(name, s, t, res, idx=None):
    tt = t if idx is None else t.take(idx)
    sel = (lambda v: v) if idx is None else (lambda v: v[idx])
    ref_in = O.inside(s, tt.x, tt.y, tt.z)
    assert np.array_equal(sel(res["inside"]), ref_in), name
    nbad = 0
    for key, mode in (("safety", 0), ("s_in", 1), ("s_out", 2)):
        ref = O.safety(s, mode, tt.x, tt.y, tt.z)
        _, _, bad = compare_values(sel(res[key]), ref, what=f"{name} {key}")
        nbad += bad.size
    nflag = 0
    for key, d in (("din", 0), ("dout", 1)):
        ref, diag = O.distance(s, d, tt)
        _, flagged, bad = compare_values(sel(res[key]), ref, diag, what=f"{name} {key}")
        nbad += bad.size
        nflag += flagged.size
        if flagged.size:
            say(f"  {name} {key}: {flagged.size} flagged tracks differ (listed): {flagged[:8].tolist()}")
    assert nbad == 0, name
    return nflag


@pytest.mark.parametrize("name", NAMES)
def test_solid_parity_mixed(geo, name):
    say(f"[solid parity] {name} n={N_SMALL}")
    t = mixed_tracks(name, N_SMALL)
    res = run_all(geo, NAMES.index(name), t)
    check(name, SOLIDS[name], t, res)


@pytest.mark.parametrize("name", ["box", "tubs"])
def test_solid_parity_paper_workload(geo, name):
    """Points uniform in a box twice the body's extent, 65,536 tracks."""
    say(f"[solid parity, 2x extent workload] {name}")
    t = W.config1_tracks(name)
    res = run_all(geo, NAMES.index(name), t)
    check(name, SOLIDS[name], t, res)


@pytest.mark.parametrize("name", list(W.CONFIG2_SOLIDS))
def test_solid_parity_full_size(geo, name):
    """All 2^20 tracks of the full-solid-set workload, in the launch shape the
    benchmark times, against the oracle element by element (every query)."""
    say(f"[solid parity, 2^20 full] {name}")
    t = W.config2_tracks(name)
    res = run_all(geo, NAMES.index(name), t)
    nflag = check(name, SOLIDS[name], t, res)
    say(f"  {name}: {t.n} tracks compared, {nflag} flagged values differ (listed)")


@pytest.mark.parametrize("name", NAMES)
def test_fused_all_matches_separate(geo, name):
    import torch
    t = mixed_tracks(name, 4099)
    lv = NAMES.index(name)
    res = run_all(geo, lv, t)
    a = [cuda(v) for v in t.arrays()]
    n = t.n
    o = [torch.empty(n, dtype=torch.int8, device="cuda")] + [torch.empty(n, dtype=torch.float64, device="cuda")
                                                             for _ in range(3)]
    geo.solid_all(lv, *a, *o)
    torch.cuda.synchronize()
    # the fused kernel is held to the same bar against the oracle
    fused = {"inside": host(o[0]), "safety": host(o[1]), "din": host(o[2]), "dout": host(o[3]),
             "s_in": res["s_in"], "s_out": res["s_out"]}
    check(name, SOLIDS[name], t, fused)


@pytest.mark.parametrize("name", NAMES)
def test_fused_distances_bitwise_equal_separate(geo, name):
    """The fused query's distances are the separate queries' bit for bit (the
    same per-ray steps, whatever kernel schedules them: the polycone's
    DistanceToIn and fused queries compact their walking rays per wavefront,
    its DistanceToOut runs one lane per track)."""
    import torch
    t = mixed_tracks(name, N_SMALL)
    lv = NAMES.index(name)
    a = [cuda(v) for v in t.arrays()]
    n = t.n
    o = [torch.empty(n, dtype=torch.int8, device="cuda")] + [torch.empty(n, dtype=torch.float64, device="cuda")
                                                             for _ in range(3)]
    geo.solid_all(lv, *a, *o)
    din = geo.distance(lv, 0, *a)
    dout = geo.distance(lv, 1, *a)
    torch.cuda.synchronize()
    assert np.array_equal(host(o[2]).view(np.int64), host(din).view(np.int64))
    assert np.array_equal(host(o[3]).view(np.int64), host(dout).view(np.int64))


@pytest.mark.parametrize("name", ["pcon", "pcon_hollow"])
def test_pcon_compacted_edge_sizes(geo, name):
    """Ragged sizes around the compacting kernel's tiles (64 tracks per
    wavefront step, 1,024 per workgroup), against the oracle."""
    import torch
    lv = NAMES.index(name)
    base = mixed_tracks(name, 2100)
    for n in (1, 2, 63, 64, 65, 255, 1023, 1024, 1025, 2100):
        t = base.take(np.arange(n))
        a = [cuda(v) for v in t.arrays()]
        din = host(geo.distance(lv, 0, *a))
        o = [torch.empty(n, dtype=torch.int8, device="cuda")] + [torch.empty(n, dtype=torch.float64, device="cuda")
                                                                 for _ in range(3)]
        geo.solid_all(lv, *a, *o)
        torch.cuda.synchronize()
        ref, diag = O.distance(SOLIDS[name], 0, t)
        _, _, bad = compare_values(din, ref, diag, what=f"{name} din n={n}")
        assert bad.size == 0, n
        assert np.array_equal(host(o[2]).view(np.int64), din.view(np.int64)), n


def test_edge_sizes(geo):
    import torch
    lv = NAMES.index("box")
    for n in (0, 1, 63, 64, 65, 257):
        t = mixed_tracks("box", max(n, 3)).take(np.arange(n))
        a = [cuda(v) for v in t.arrays()]
        got = host(geo.distance(lv, 1, *a))
        ref, _ = O.distance(SOLIDS["box"], 1, t)
        assert got.shape == (n,)
        assert np.array_equal(np.isinf(got), np.isinf(ref))
        assert np.all(np.abs(got - ref)[np.isfinite(ref)] <= 1e-12 * np.maximum(1, np.abs(ref[np.isfinite(ref)])))
    torch.cuda.synchronize()


def test_hand_points(geo):
    """Points on faces, edges, corners and the axis, with axis-aligned directions."""
    pts, dirs = [], []
    for name in NAMES:
        c, h = W.solid_extent(SOLIDS[name])
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                for sz in (-1, 0, 1):
                    pts.append(c + h * np.array([sx, sy, sz], dtype=float) * 0.5)
                    pts.append(c + h * np.array([sx, sy, sz], dtype=float))
        pts.append(np.zeros(3))
    P = np.array(pts).T
    rng = np.random.default_rng(3)
    for name in NAMES:
        for D in (np.array([[1.0], [0.0], [0.0]]), np.array([[0.0], [0.0], [-1.0]]),
                  np.stack(W.isotropic(rng, P.shape[1]))):
            D = np.broadcast_to(D, P.shape)
            t = W.Tracks(*[np.ascontiguousarray(v) for v in (*P, *D)])
            res = run_all(geo, NAMES.index(name), t)
            check(name, SOLIDS[name], t, res)


def test_tube_inner_cylinder_cases(geo):
    """Points on and near a hollow tube's inner cylinder (exactly on it on the
    axes, within rounding of it elsewhere, and 1e-12 relative to 0.5 mm off
    it on both sides) moving out from the axis, along the cylinder, towards
    the axis and along z, with signed zeros: the cases where the inner
    cylinder's two roots lie behind the point, at it, or do not exist, which
    decide whether the inner surface is solved at all."""
    offs = [0.0] + [sg * e for e in (1e-10, 4e-10, 1e-9, 1e-6, 0.5) for sg in (-1.0, 1.0)]
    for name in ("tubs", "tubs_half", "tubs_hollow_full"):
        rmin, _, dz = SOLIDS[name].params[:3]
        offs_n = offs + [-1e-12 * rmin, 1e-12 * rmin]
        P, D = [], []
        axes = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]
        angles = axes + [(math.cos(a), math.sin(a)) for a in (0.3, 2.0, 4.4)]
        for c, s in angles:
            u, v = np.array([c, s, 0.0]), np.array([-s, c, 0.0])
            dirs = [u, -u, v, -v, (u + v) / math.sqrt(2), (v - u) / math.sqrt(2),
                    np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, -1.0]),
                    (u + np.array([0.0, 0.0, 1.0])) / math.sqrt(2), (1e-3 * u + v) / math.sqrt(1 + 1e-6)]
            for off in offs_n:
                r = rmin + off
                for z in (0.0, 0.5 * dz, dz):
                    for d in dirs:
                        P.append((r * c, r * s, z))
                        D.append(d)
        # signed zeros: on the cylinder at phi = 0 moving along it with
        # p.y = -0 and d.x = -0 (the radial product is -0)
        for d in ((-0.0, 1.0, 0.0), (-0.0, -1.0, 0.0), (-0.0, 0.0, 1.0)):
            P.append((rmin, -0.0, 0.0))
            D.append(d)
        P, D = np.array(P, dtype=float).T, np.array(D, dtype=float).T
        t = W.Tracks(*[np.ascontiguousarray(a) for a in (*P, *D)])
        say(f"[tube inner cylinder] {name} n={t.n}")
        res = run_all(geo, NAMES.index(name), t)
        check(name, SOLIDS[name], t, res)


@pytest.mark.parametrize("name", ["cons", "cons_seg", "sphere"])
def test_cone_sphere_inner_surface_cases(geo, name):
    """Points on and near the inner surface of a hollow cone (full and a
    three-quarter segment whose planes lie off the axes) and of a spherical
    shell, 1e-10 mm to 0.5 mm off it on both sides, moving out from the axis
    or centre, towards it, along the surface's generator, tangentially and
    along z."""
    s = SOLIDS[name]
    P, D = [], []
    offs = [0.0] + [sg * e for e in (1e-10, 4e-10, 1e-9, 1e-6, 0.5) for sg in (-1.0, 1.0)]
    angles = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)] + [(math.cos(a), math.sin(a)) for a in (0.3, 2.0, 4.4)]
    ez = np.array([0.0, 0.0, 1.0])
    if s.type == W.CONS:
        rmin1, _, rmin2, _, dz = s.params[:5]
        for zf in (-1.0, 0.0, 0.5, 1.0):
            z = zf * dz
            rin = rmin1 + (rmin2 - rmin1) * (z + dz) / (2 * dz)
            for c, sn in angles:
                u, v = np.array([c, sn, 0.0]), np.array([-sn, c, 0.0])
                g = (rmin2 - rmin1) * u + 2 * dz * ez
                g = g / np.linalg.norm(g)  # along the inner cone's generator
                for off in offs:
                    r = rin + off
                    for d in (u, -u, v, ez, -ez, g, -g, (u + ez) / math.sqrt(2)):
                        P.append((r * c, r * sn, z))
                        D.append(d)
    else:
        rmin = s.params[0]
        for c, sn in angles:
            for cz in (0.0, 0.6, -1.0):
                w = np.array([c * math.sqrt(1 - cz * cz), sn * math.sqrt(1 - cz * cz), cz])
                t1 = np.cross(w, ez if abs(cz) < 0.9 else np.array([1.0, 0.0, 0.0]))
                t1 = t1 / np.linalg.norm(t1)
                for off in offs:
                    for d in (w, -w, t1, ez, -ez, (w + t1) / math.sqrt(2)):
                        P.append(tuple((rmin + off) * w))
                        D.append(d)
    P, D = np.array(P, dtype=float).T, np.array(D, dtype=float).T
    t = W.Tracks(*[np.ascontiguousarray(a) for a in (*P, *D)])
    say(f"[inner surface] {name} n={t.n}")
    res = run_all(geo, NAMES.index(name), t)
    check(name, s, t, res)


@pytest.mark.parametrize("name", ["pcon", "pcon_hollow"])
def test_polycone_walk_counters(geo, name):
    """The polycone's work counters (profiling only) add up: every point not
    inside is either rejected by the bounding cylinder or walked by
    DistanceToIn, every point not outside is walked by DistanceToOut (the fused
    query does both, surface points taking both walks), no walk computes more
    than the 9 sections, and profiling leaves the outputs unchanged."""
    import torch
    import paper_1512_06637_amd as G
    lv = NAMES.index(name)
    t = mixed_tracks(name, N_SMALL)
    a = [cuda(v) for v in t.arrays()]
    code = host(geo.inside(lv, *a[:3]))
    not_in, not_out = int((code != G.INSIDE).sum()), int((code != G.OUTSIDE).sum())
    ref_in = host(geo.distance(lv, G.TO_IN, *a))
    geo.profile(work=True)
    try:
        got_in = host(geo.distance(lv, G.TO_IN, *a))
        w_in = geo.profile_read()[2][28:33]
        geo.distance(lv, G.TO_OUT, *a)
        w_out = geo.profile_read()[2][28:33]
        f64 = torch.float64
        geo.solid_all(lv, *a, torch.empty(t.n, dtype=torch.int8, device="cuda"),
                      *[torch.empty(t.n, dtype=f64, device="cuda") for _ in range(3)])
        w_all = geo.profile_read()[2][28:33]
    finally:
        geo.profile()
    say(f"[pcon work] {name}: in {w_in}, out {w_out}, fused {w_all}")
    assert np.array_equal(got_in.view(np.int64), ref_in.view(np.int64))
    assert w_in[2] + w_in[3] == not_in and w_in[1] == w_in[4] == 0
    assert w_out[4] == not_out and w_out[0] == w_out[2] == w_out[3] == 0
    assert w_all[2] + w_all[3] == not_in and w_all[4] == not_out
    assert w_in[0] <= 9 * w_in[3] and w_out[1] <= 9 * w_out[4] and w_in[3] > 0 and w_out[4] > 0
