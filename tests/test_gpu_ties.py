"""Exact ties of ComputeStep on the GPU, compared without excusing them: the
oracle marks such steps NEAR_TIE (two correct codes could order them
differently in general), but these ties are exact in FP64, so the reading --
lowest placement index among equal daughters, a daughter over an equal exit --
must be reproduced exactly by every daughter loop (plain, culled, phi sectors)
and by the per-lane and basket transports, in both precisions."""
import numpy as np
import pytest

import oracle as O
from paper_1512_06637_amd import workloads as W
from tests.gpu_util import cuda, host, say

pytestmark = pytest.mark.gpu

CASES = W.tie_cases()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_tie_step_and_transport(name, precision):
    import paper_1512_06637_amd as G
    lvs, p, d, k, st = CASES[name]
    blob = W.make_blob(lvs)
    g = G.Geometry(blob)
    og = O.Geometry(blob)
    say(f"[tie] {name} precision={precision}")
    t = W.tie_tracks(CASES[name], 64)
    pv0 = og.locate(t.x, t.y, t.z)
    gst, gnx = g.step(*[cuda(v) for v in t.arrays()], cuda(pv0), precision=precision)
    rs, rn, _, _ = og.step(t, pv0)
    assert np.array_equal(host(gnx), rn), (host(gnx)[:4], rn[:4])
    assert np.all(np.abs(host(gst) - rs) <= 1e-12 * np.maximum(1.0, rs))
    # whole transports: one lane per track (7 tracks) and per-volume baskets
    # (8,192 tracks), every step compared, ties included
    for n in (7, 8192):
        tt = W.tie_tracks(CASES[name], n)
        got = g.transport(*[cuda(v) for v in tt.arrays()], precision=precision)
        ref = og.transport(tt)
        ns = host(got["nsteps"])
        assert np.array_equal(ns, ref["nsteps"]), n
        assert np.array_equal(host(got["flags"]).astype(np.uint32), ref["flags"]), n
        m = int(ref["nsteps"][0])
        gp, gs = host(got["pv"]), host(got["step"])
        assert np.all(gp[:, :m + 1] == ref["pv"][:, :m + 1]), (n, gp[0, :m + 1], ref["pv"][0, :m + 1])
        assert np.all(np.abs(gs[:, :m] - ref["step"][:, :m]) <= 1e-12 * np.maximum(1.0, ref["step"][:, :m]) + 1e-12)
        say(f"  n={n}: sequence {ref['pv'][0, :m + 1].tolist()} reproduced")
    og.close()
    g.close()
