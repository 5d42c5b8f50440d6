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
            _, _, bad = compare_values(e_din, ref, diag, what="graph din")
            assert bad.size == 0
            assert np.array_equal(e_in, O.inside(sol["box"], tr.x, tr.y, tr.z))
        say(f"  replay {r}: equal to eager")
    g.close()


@pytest.mark.parametrize("transport", [0, 1])
def test_transport_captured_in_graph_matches_eager(transport):
    """nav_transport (20,011 tracks; lane form, then basket form) only enqueues
    work, so it can be captured into a HIP graph once its workspace exists;
    every replay, with new inputs copied into the captured buffers and eager
    transports in between, equals the eager result bit for bit, and the eager
    result matches the oracle."""
    import torch
    import paper_1512_06637_amd as G
    blob = W.detector_blob()
    g = G.Geometry(blob)
    g.set_tuning(transport=transport)
    n = 20011
    t = W.config3_tracks(n)
    static = [cuda(v) for v in t.arrays()]
    max_steps = 128
    out = {"pv": torch.empty((n, max_steps + 1), dtype=torch.int32, device="cuda"),
           "step": torch.empty((n, max_steps), dtype=torch.float64, device="cuda"),
           "nsteps": torch.empty(n, dtype=torch.int32, device="cuda"),
           "flags": torch.empty(n, dtype=torch.int32, device="cuda")}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.transport(*static, out=out)  # sizes the workspace outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        g.transport(*static, out=out)
    og = O.Geometry(blob)
    for r in range(3):
        perm = np.random.default_rng(200 + r).permutation(n)
        tr = t.take(perm)
        for dst, src in zip(static, tr.arrays()):
            dst.copy_(torch.from_numpy(src))
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        e = g.transport(*[cuda(v) for v in tr.arrays()])  # eager, fresh buffers, same workspace
        torch.cuda.synchronize()
        ns = host(e["nsteps"])
        assert np.array_equal(host(out["nsteps"]), ns), r
        assert np.array_equal(host(out["flags"]), host(e["flags"])), r
        k = np.arange(max_steps)[None, :] < ns[:, None]
        kp = np.concatenate([np.ones((n, 1), bool), k], axis=1)
        assert np.array_equal(host(out["pv"])[kp], host(e["pv"])[kp]), r
        assert np.array_equal(host(out["step"])[k].view(np.int64), host(e["step"])[k].view(np.int64)), r
        if r == 0:
            ref = og.transport(tr)
            ok = (ref["diag"] & O.D_ILL) == 0
            same = (ns == ref["nsteps"]) & np.array([np.array_equal(host(e["pv"])[i, :ns[i] + 1],
                                                                     ref["pv"][i, :ns[i] + 1]) for i in range(n)])
            assert np.all(same[ok]), np.nonzero(~same & ok)[0][:10]
        say(f"  transport replay {r}: equal to eager ({int(ns.sum())} track-steps)")
    og.close()
    g.close()


@pytest.mark.parametrize("transport", [0, 1])
def test_transport_capture_without_workspace_is_refused(transport):
    """Under capture nothing may be allocated: a geometry that has never
    transported this many tracks refuses with GV_ESTATE (nothing recorded)."""
    import torch
    import paper_1512_06637_amd as G
    g = G.Geometry(W.detector_blob())
    g.set_tuning(transport=transport)
    n = 9000
    t = W.config3_tracks(n)
    a = [cuda(v) for v in t.arrays()]
    out = {"pv": torch.empty((n, 129), dtype=torch.int32, device="cuda"),
           "step": torch.empty((n, 128), dtype=torch.float64, device="cuda"),
           "nsteps": torch.empty(n, dtype=torch.int32, device="cuda"),
           "flags": torch.empty(n, dtype=torch.int32, device="cuda")}
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    err = None
    try:
        with torch.cuda.graph(gr):
            try:
                g.transport(*a, out=out)
            except G.GVError as e:
                err = e
    except Exception:
        pass  # an empty capture may itself be rejected by torch
    assert err is not None and err.code == G.GV_ESTATE, err
    torch.cuda.synchronize()
    got = g.transport(*a, out=out)  # eager afterwards still works
    torch.cuda.synchronize()
    assert int(host(got["nsteps"]).min()) > 0
    g.close()
