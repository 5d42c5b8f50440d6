"""GPU parity of the daughter-candidate indexes on geometries built to reach
every branch, against the oracle's plain loop over all daughters.

* Nested tubes: ten identity-placed full tubes of unequal lengths, a solid
  core, placed out of radial order; starts uniform in the world with isotropic
  directions (one in eight parallel to the axis), so the radial walk runs
  outward and inward, from points radially inside a tube but beyond its ends,
  and with A = 0.
* Ring: sixteen boxes around the z axis inside a box mother; segments through
  the axis region take the culled loop, the others the phi sectors.
* Grid (25 boxes through the axis), big grid (81 boxes: two chunks of 64
  daughters) and bundle (12 tilted tubes): no index applies, so the culled
  loop runs, with group boxes for the grids.

Bar: the navigation bar of the detector tests (sequences, counts and flags
bit-exact for tracks the oracle does not flag; steps within 1e-12 relative +
1e-10 mm)."""
import numpy as np
import pytest

import oracle as O
from paper_1512_06637_amd import workloads as W
from tests.gpu_util import compare_values, cuda, host, say
from tests.test_gpu_nav import compare_transport

pytestmark = pytest.mark.gpu

CASES = {
    "nested_tubes": (W.nested_tubes_description, (390.0, 390.0, 390.0), (0.0, 0.0, 0.0)),
    "ring": (W.ring_description, (99.0, 99.0, 49.0), (0.0, 0.0, 10.0)),
    "grid": (W.grid_description, (119.0, 119.0, 59.0), (0.0, 0.0, 0.0)),
    "big_grid": (W.big_grid_description, (109.0, 109.0, 59.0), (0.0, 0.0, 0.0)),
    "bundle": (W.bundle_description, (119.0, 119.0, 89.0), (0.0, 0.0, 0.0)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    import paper_1512_06637_amd as G
    desc, half, centre = CASES[request.param]
    blob = W.make_blob(desc())
    g = G.Geometry(blob)
    og = O.Geometry(blob)
    yield request.param, g, og, half, centre
    g.close()
    og.close()


@pytest.mark.parametrize("n", [4099, 20011])
def test_index_transport(case, n):
    """Per-lane transport below 8,192 tracks, baskets above; FP64 and FP32
    screens; the index counters show which structure ran."""
    import paper_1512_06637_amd as G
    name, g, og, half, centre = case
    t = W.uniform_world_tracks(half, n, 1234 + n, centre)
    say(f"[index transport] {name} n={n}")
    ref = og.transport(t)
    a = [cuda(v) for v in t.arrays()]
    for prec in (G.FP64, G.FP32_REFINE):
        g.profile(work=True)
        got = g.transport(*a, precision=prec)
        _, _, w = g.profile_read()
        g.profile()
        assert compare_transport(got, ref) > 0.99 * n
        if n > 8192:  # basket path: counters of the step kernel
            say(f"  counters: radial {w[24]} lookups / {w[25]} bounds, phi {w[26]} lookups / {w[27]} sectors, "
                f"box tests {w[1]}")
            if name == "nested_tubes":
                assert w[24] > 0 and w[25] > 0 and w[26] == 0
            elif name == "ring":
                assert w[26] > 0 and w[27] >= w[26] and w[1] > 0  # box tests: the near-axis fallback ran
                assert w[24] == 0
            else:  # culled loop: box tests and bound checks of the daughter type
                t_d = 0 if name in ("grid", "big_grid") else 1  # box or tube daughters
                assert w[1] > 0 and w[2 + t_d] > 0 and w[8 + t_d] > 0 and w[24] == 0 and w[26] == 0


def test_index_step(case):
    """One ComputeStep from uniform starts (located by the library), against
    the oracle's step, FP64 and FP32 screens."""
    import paper_1512_06637_amd as G
    name, g, og, half, centre = case
    t = W.uniform_world_tracks(half, 30011, 77, centre)
    a = [cuda(v) for v in t.arrays()]
    pv = host(g.locate(*a[:3]))
    assert np.array_equal(pv, og.locate(t.x, t.y, t.z))
    inside = pv >= 0
    tt = t.take(np.nonzero(inside)[0])
    p = pv[inside].astype(np.int32)
    rst, rnx, _, rdg = og.step(tt, p)
    ok = (rdg & O.D_ILL) == 0
    b = [cuda(v) for v in tt.arrays()]
    for prec in (G.FP64, G.FP32_REFINE):
        st, nx = g.step(*b, cuda(p), precision=prec)
        assert np.array_equal(host(nx)[ok], rnx[ok]), name
        _, _, bad = compare_values(host(st)[ok], rst[ok], what=f"{name} step")
        assert bad.size == 0
    say(f"  {name}: {tt.n} steps compared, {int((~ok).sum())} flagged")
