"""nav_transport_noalloc (the allocation-free transport, for callers that
cannot allocate device memory) against nav_transport: two calls in a row, the
second with fewer tracks, each bitwise equal to nav_transport's outputs on the
same inputs (the two share their kernels; the second call must not see the
first call's scratch contents), and the first also against the oracle; sizes
beyond the scratch's limit are refused before anything is enqueued."""
import numpy as np
import pytest

import oracle as O
from paper_1512_06637_amd import workloads as W
from tests.gpu_util import cuda, host, say, transport_bits_equal, transport_rows_compare

pytestmark = pytest.mark.gpu

MAX_TRACKS = 1 << 21


def _out(n, max_steps=128):
    import torch
    return {"pv": torch.full((n, max_steps + 1), -2, dtype=torch.int32, device="cuda"),
            "step": torch.full((n, max_steps), float("nan"), dtype=torch.float64, device="cuda"),
            "nsteps": torch.full((n,), -3, dtype=torch.int32, device="cuda"),
            "flags": torch.full((n,), -3, dtype=torch.int32, device="cuda")}


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_transport_twice(precision):
    import torch
    import paper_1512_06637_amd as G
    blob = W.detector_blob()
    g = G.Geometry(blob)
    og = O.Geometry(blob)
    for call, n in enumerate([300_007, 20_011]):
        t = W.config3_tracks(n)
        a = [cuda(v) for v in t.arrays()]
        say(f"[noalloc] call {call}: n={n} precision={precision}")
        got = g.transport(*a, out=_out(n), precision=precision, noalloc=True)
        ref = g.transport(*a, out=_out(n), precision=precision)
        torch.cuda.synchronize()
        assert transport_bits_equal(got, ref), (call, n)
        if call == 1:
            transport_rows_compare(got, og.transport(t), what=f"noalloc n={n}")
        say(f"  equal to nav_transport ({int(host(got['nsteps']).sum())} track-steps)")
    og.close()
    g.close()


def test_noalloc_refuses_beyond_scratch():
    import torch
    import paper_1512_06637_amd as G
    g = G.Geometry(W.detector_blob())
    n = MAX_TRACKS + 1
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    d = torch.ones(n, dtype=torch.float64, device="cuda")
    out = {"pv": torch.empty((n, 2), dtype=torch.int32, device="cuda"),
           "step": torch.empty((n, 1), dtype=torch.float64, device="cuda"),
           "nsteps": torch.empty(n, dtype=torch.int32, device="cuda"),
           "flags": torch.empty(n, dtype=torch.int32, device="cuda")}
    with pytest.raises(G.GVError) as e:
        g.transport(x, x, x, d, x, x, max_steps=1, out=out, noalloc=True)
    assert e.value.code == G.GV_EINVAL
    g.close()
