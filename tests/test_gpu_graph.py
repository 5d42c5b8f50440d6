"""HIP-graph replay of library calls (the measurement protocol captures solid
queries into a graph and replays it): every replay, with new inputs copied into
the captured buffers and eager work in between, equals an eager call, and the
eager call equals the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1512_06637_amd import workloads as W
from tests.gpu_util import compare_values, cuda, host, say

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    import torch
    import paper_1512_06637_amd as G
    sol = W.config_solids()
    g = G.Geometry(W.multi_solid_blob([sol["box"], sol["tubs"]]))
    t = W.config1_tracks("tubs", 4099)
    static = [cuda(v) for v in t.arrays()]
    o_din = torch.empty(t.n, dtype=torch.float64, device="cuda")
    o_saf = torch.empty(t.n, dtype=torch.float64, device="cuda")
    o_in = torch.empty(t.n, dtype=torch.int8, device="cuda")

    def calls():
        g.distance(1, G.TO_IN, *static, out=o_din)
        g.safety(1, *static[:3], out=o_saf)
        g.inside(0, *static[:3], out=o_in)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls()
    torch.cuda.current_stream().wait_stream(side)
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        calls()
    for r in range(4):
        perm = np.random.default_rng(100 + r).permutation(t.n)
        tr = t.take(perm)
        for dst, src in zip(static, tr.arrays()):
            dst.copy_(torch.from_numpy(src))
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        a = [cuda(v) for v in tr.arrays()]  # eager, on fresh buffers
        e_din = host(g.distance(1, G.TO_IN, *a))
        e_saf = host(g.safety(1, *a[:3]))
        e_in = host(g.inside(0, *a[:3]))
        torch.cuda.synchronize()
        assert np.array_equal(host(o_din).view(np.int64), e_din.view(np.int64)), r
        assert np.array_equal(host(o_saf).view(np.int64), e_saf.view(np.int64)), r
        assert np.array_equal(host(o_in), e_in), r
        if r == 0:
            ref, diag = O.distance(sol["tubs"], 0, tr)
            _, _, bad = compare_values(e_din, ref, diag, what="graph din", solid=sol["tubs"], tracks=tr)
            assert bad.size == 0
            assert np.array_equal(e_in, O.inside(sol["box"], tr.x, tr.y, tr.z))
        say(f"  replay {r}: equal to eager")
    g.close()
