"""GPU parity of composite (Boolean) solids against the oracle: the solid-level
queries for eight composites covering the three operations, every elementary
part type and rotated placements; then navigation (locate, ComputeStep,
NavSafety, volume Inside, transport on both the per-lane and the basket path)
in a geometry whose volumes are composites, one of them with daughters.

Bar: as for elementary solids (codes bit-exact, FP64 values within 1e-12
relative, oracle-flagged tracks listed) and as for the detector's navigation
(volume sequences bit-exact, steps within the navigation bar)."""
import numpy as np
import pytest

import oracle as O
from paper_1512_06637_amd import workloads as W
from tests.gpu_util import compare_values, cuda, host, say
from tests.test_gpu_nav import compare_transport
from tests.test_gpu_solids import check, run_all
from tests.test_oracle_bool import COMPOSITES

pytestmark = pytest.mark.gpu

NAMES = list(COMPOSITES)
N_SMALL = (1 << 16) + 37


@pytest.fixture(scope="module")
def geo():
    import paper_1512_06637_amd as G
    g = G.Geometry(W.multi_solid_blob([COMPOSITES[k] for k in NAMES]))
    yield g
    g.close()


def mixed_tracks(name, n):
    """Thirds inside / outside / within 1e-6 mm of the surface, isotropic."""
    s = COMPOSITES[name]
    rng = np.random.default_rng(300 + NAMES.index(name))
    k = n // 3
    pin = W.sample_volume(s, rng, k)
    pout = W.sample_outside(s, rng, k)
    ps, nrm = W.sample_surface(s, rng, n - 2 * k)
    ps = ps + nrm * rng.uniform(-1e-6, 1e-6, n - 2 * k)[None, :]
    P = np.concatenate([pin, pout, ps], axis=1)[:, rng.permutation(n)]
    return W.Tracks(*P, *W.isotropic(rng, n))


def box_tracks(name, n):
    s = COMPOSITES[name]
    rng = np.random.default_rng(400 + NAMES.index(name))
    c, h = W.solid_extent(s)
    P = W.uniform_box_points(rng, n, c, 1.6 * h)
    return W.Tracks(*P, *W.isotropic(rng, n))


@pytest.mark.parametrize("name", NAMES)
def test_composite_parity_mixed(geo, name):
    say(f"[composite parity] {name} n={N_SMALL}")
    t = mixed_tracks(name, N_SMALL)
    check(name, COMPOSITES[name], t, run_all(geo, NAMES.index(name), t))


@pytest.mark.parametrize("name", NAMES)
def test_composite_parity_box_workload(geo, name):
    say(f"[composite parity, 1.6x extent] {name} n={N_SMALL}")
    t = box_tracks(name, N_SMALL)
    check(name, COMPOSITES[name], t, run_all(geo, NAMES.index(name), t))


@pytest.mark.parametrize("name", ["box_minus_hole", "pcon_minus_cons"])
def test_composite_parity_full_size_sampled(geo, name):
    """2^20 tracks in one launch; 20,000 sampled outputs recomputed by the oracle."""
    say(f"[composite parity, 2^20 sampled] {name}")
    t = box_tracks(name, 1 << 20)
    res = run_all(geo, NAMES.index(name), t)
    idx = np.sort(np.random.default_rng(31).choice(t.n, 20000, replace=False))
    check(name, COMPOSITES[name], t, res, idx)


def test_composite_fused_matches_oracle(geo):
    import torch
    name = "tubs_u_rot_box"
    t = mixed_tracks(name, 4099)
    lv = NAMES.index(name)
    a = [cuda(v) for v in t.arrays()]
    o = [torch.empty(t.n, dtype=torch.int8, device="cuda")] + [torch.empty(t.n, dtype=torch.float64, device="cuda")
                                                               for _ in range(3)]
    geo.solid_all(lv, *a, *o)
    torch.cuda.synchronize()
    s = COMPOSITES[name]
    code = O.inside(s, t.x, t.y, t.z)
    assert np.array_equal(host(o[0]), code)
    _, _, bad = compare_values(host(o[1]), O.safety(s, 0, t.x, t.y, t.z), what="fused safety")
    assert bad.size == 0
    for k, d in ((2, 0), (3, 1)):
        ref, diag = O.distance(s, d, t)
        ref = np.where(code == (O.INSIDE if d == 0 else O.OUTSIDE), -1.0, ref)
        _, _, bad = compare_values(host(o[k]), ref, diag, what=f"fused dist {d}")
        assert bad.size == 0


# ------------------------------------------------------------------ navigation
BLOB = W.composite_blob()


@pytest.fixture(scope="module")
def geos():
    import paper_1512_06637_amd as G
    g = G.Geometry(BLOB)
    og = O.Geometry(BLOB)
    yield g, og
    g.close()
    og.close()


def test_composite_locate_step_safety(geos):
    import paper_1512_06637_amd as G
    g, og = geos
    t = W.composite_tracks(20011)
    say(f"[composite navigation] locate / step / safety / inside n={t.n}")
    a = [cuda(v) for v in t.arrays()]
    pv = host(g.locate(*a[:3]))
    ref_pv = og.locate(t.x, t.y, t.z)
    assert np.array_equal(pv, ref_pv)
    assert np.bincount(pv + 1, minlength=11)[[2, 7, 8, 9, 10]].min() > 100
    p32 = cuda(pv.astype(np.int32))
    rst, rnx, _, rdg = og.step(t, pv)
    ok = (rdg & O.D_ILL) == 0
    for prec in (G.FP64, G.FP32_REFINE):
        st, nx = g.step(*a, p32, precision=prec)
        assert np.array_equal(host(nx)[ok], rnx[ok])
        _, _, bad = compare_values(host(st)[ok], rst[ok], what="composite step")
        assert bad.size == 0
        _, _, bad = compare_values(host(g.nav_safety(*a[:3], p32, precision=prec)), og.nav_safety(t.x, t.y, t.z, pv),
                                   what="composite nav safety")
        assert bad.size == 0
    assert np.array_equal(host(g.nav_inside(*a[:3], p32)), og.nav_inside(t.x, t.y, t.z, pv))


@pytest.mark.parametrize("n", [4099, 20011])
def test_composite_transport(geos, n):
    """Per-lane transport below 8,192 tracks, per-volume baskets above; both in
    full against the oracle, in FP64 and with the FP32 screens."""
    import paper_1512_06637_amd as G
    g, og = geos
    t = W.composite_tracks(n)
    say(f"[composite transport] n={n}")
    ref = og.transport(t)
    a = [cuda(v) for v in t.arrays()]
    for prec in (G.FP64, G.FP32_REFINE):
        assert compare_transport(g.transport(*a, precision=prec), ref) > 0.99 * n


# ------------------------------------------------- physics-limited and serving
COMPOSITE_MAT = {"density": np.array([1.0, 5.0]),
                 "sigma": np.array([[1e-4, 5e-5], [0.02, 0.01]]),  # mean free paths 1e4, 2e4 / 10, 20 mm
                 "lv_mat": np.array([0, 1, 1, 1, 1, 1, 1], np.int32)}


@pytest.mark.parametrize("n", [4099, 20011])
def test_composite_phys_transport(geos, n):
    """Physics-limited transport in the composite geometry (dense composites:
    many interactions inside them), per-lane and basket paths, against the
    oracle; the short-cut and the FP32 screens change nothing."""
    import paper_1512_06637_amd as G
    from tests.test_gpu_phys import _same, compare_phys
    g, og = geos
    g.set_materials(COMPOSITE_MAT["density"], COMPOSITE_MAT["sigma"], COMPOSITE_MAT["lv_mat"])
    t = W.composite_tracks(n)
    say(f"[composite phys transport] n={n}")
    a = [cuda(v) for v in t.arrays()]
    seed = W.PHYS_SEED + 1
    got = g.transport_phys(*a, seed, max_steps=256, shortcut=False)
    ref = og.transport_phys(t, COMPOSITE_MAT, seed, max_steps=256)
    assert compare_phys(got, ref) > 0.5 * n
    _same(got, g.transport_phys(*a, seed, max_steps=256, shortcut=True))
    _same(got, g.transport_phys(*a, seed, max_steps=256, shortcut=True, precision=G.FP32_REFINE))


def test_composite_serving(geos):
    """Mixed baskets served in shared rounds on the composite geometry equal
    the per-kind entry points and the oracle."""
    import paper_1512_06637_amd as G
    from tests.test_gpu_nav import STEP_REL
    from tests.test_gpu_serve import alone, check_equal, make_baskets, run_server
    g, og = geos
    t = W.composite_tracks(6000)
    pool = (t, og.locate(t.x, t.y, t.z).astype(np.int32))
    baskets = make_baskets(pool, 40, 23)
    say(f"[composite serve] {len(baskets)} baskets")
    with G.Server(g, slots=16, hbm_budget=64 << 20, nstreams=2) as srv:
        outs, _ = run_server(srv, baskets, pool)
    _, pv = pool
    for b, ob in zip(baskets, outs):
        got = G.unpack_result(b["kind"], ob, b["n"])
        check_equal(b["kind"], got, alone(g, b, pool))
        i = b["idx"]
        sub = t.take(i)
        if b["kind"] == G.Q_STEP:
            rs, rn, rf, rd = og.step(sub, pv[i], pstep=b["pstep"])
            ok = (rd & O.D_ILL) == 0
            assert np.array_equal(got[1][ok], rn[ok]) and np.array_equal(got[2][ok], rf[ok])
            assert np.all(np.abs(got[0] - rs)[ok] <= STEP_REL * np.maximum(1, rs[ok]) + 1e-12)
        elif b["kind"] == G.Q_SAFETY:
            _, _, bad = compare_values(got, og.nav_safety(sub.x, sub.y, sub.z, pv[i]), what="served safety")
            assert bad.size == 0
        else:
            assert np.array_equal(got, og.nav_inside(sub.x, sub.y, sub.z, pv[i]))
