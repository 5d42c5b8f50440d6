"""Launch shapes never change a result: every shape the autotuner may pick
(and the stored choice) gives outputs bitwise equal to the defaults', for both
transport forms (FP64 and FP32_REFINE) and the solid-level queries; repeated
transports are bitwise equal (the atomics of the ordering, the work counter and
the regrouping only reorder work); and the roof probes compute what they
claim."""
import numpy as np
import pytest

from paper_1512_06637_amd import workloads as W
from tests.gpu_util import cuda, host, say

pytestmark = pytest.mark.gpu

BASKET = {"transport": 1}
SHAPES = [
    # lane form (default): orderings, register budgets, output staging, grid sizes
    {"sort_bits": 0},
    {"sort_bits": 3},
    {"sort_bits": 7},
    {"sort_key": 2},
    {"sort_key": 2, "sort_bits": 7},
    {"lane_waves": 3},
    {"lane_stage": 1},
    {"lane_stage": 1, "lane_waves": 3, "sort_bits": 0},
    {"lane_waves": 4, "lane_stage": 2, "sort_key": 2},
    {"lane_sched": 1},
    {"lane_sched": 1, "lane_waves": 3, "sort_bits": 0},
    {"lane_grid": 7},
    {"lane_grid": 300, "lane_waves": 3},
    # basket form: step and regrouping grids, direction cells, register budget
    dict(BASKET),
    dict(BASKET, step_grid=256),
    dict(BASKET, step_grid=1024, scatter_grid=64),
    dict(BASKET, scatter_grid=1024),
    dict(BASKET, cell_bits=0),
    dict(BASKET, cell_bits=4),
    dict(BASKET, step_waves=3),
    dict(BASKET, step_grid=97, scatter_grid=3, cell_bits=4, step_waves=3),
]
DEFAULTS = {"step_grid": 0, "scatter_grid": 0, "cell_bits": -1, "step_waves": 0, "transport": 0, "sort_bits": -1,
            "sort_key": 0, "lane_waves": 0, "lane_stage": 0, "lane_grid": 0, "lane_sched": 0}


def _bits(out):
    ns = host(out["nsteps"])
    n, ms = host(out["step"]).shape
    k = np.arange(ms)[None, :] < ns[:, None]
    kp = np.concatenate([np.ones((n, 1), bool), k], axis=1)
    return ns, host(out["flags"]), host(out["pv"])[kp], host(out["step"])[k].view(np.int64)


def _equal(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("precision", [0, 1])
def test_transport_shapes_and_repeats_bitwise(precision):
    import torch
    import paper_1512_06637_amd as G
    from paper_1512_06637_amd import tune
    g = G.Geometry(W.detector_blob(), tuned=False)
    t = W.config3_tracks(1 << 17)
    a = [cuda(v) for v in t.arrays()]
    say(f"[tune] transport n={t.n} precision={precision}")
    ref = _bits(g.transport(*a, precision=precision))
    for r in range(2):  # repeats with the default shape
        assert _equal(ref, _bits(g.transport(*a, precision=precision))), f"repeat {r}"
    stored = tune.stored_choice() or {}
    for sh in SHAPES + ([stored] if stored else []):
        g.set_tuning(**{**DEFAULTS, **sh})
        got = _bits(g.transport(*a, precision=precision))
        torch.cuda.synchronize()
        assert _equal(ref, got), sh
        say(f"  shape {sh}: bitwise equal")
    g.close()


@pytest.mark.parametrize("name", ["tubs", "pcon"])
def test_solid_lane_shapes_bitwise(name):
    import torch
    import paper_1512_06637_amd as G
    sol = W.config_solids()
    g = G.Geometry(W.multi_solid_blob([sol[name]]), tuned=False)
    t = W.config2_tracks(name, (1 << 16) + 37)
    a = [cuda(v) for v in t.arrays()]

    def run():
        o = [torch.empty(t.n, dtype=torch.int8, device="cuda")] + \
            [torch.empty(t.n, dtype=torch.float64, device="cuda") for _ in range(3)]
        g.solid_all(0, *a, *o)
        torch.cuda.synchronize()
        return [host(v).view(np.uint8) for v in o]

    ref = run()
    for sh in [{"solid_block": 64}, {"solid_block": 1024}, {"solid_grid": 7}, {"solid_block": 128, "solid_grid": 300}]:
        g.set_tuning(**{**{"solid_block": 0, "solid_grid": 0}, **sh})
        assert _equal(ref, run()), sh
    g.close()


def test_tuning_rejects_bad_fields():
    import paper_1512_06637_amd as G
    g = G.Geometry(W.detector_blob(), tuned=False)
    for bad in [{"step_grid": 5000}, {"cell_bits": 3}, {"solid_block": 100}, {"step_waves": 5}, {"transport": 3},
                {"sort_bits": 8}, {"sort_key": 3}, {"lane_waves": 2}, {"lane_stage": 3}, {"lane_sched": 3},
                {"lane_grid": -1}]:
        with pytest.raises(G.GVError):
            g.set_tuning(**bad)
    assert g.get_tuning()["step_grid"] == 0
    g.close()


def test_roof_probes_compute_what_they_claim():
    import torch
    import paper_1512_06637_amd as G
    n = (1 << 20) + 2
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    G.probe_stream(a, b, c, 0.5)
    torch.cuda.synchronize()
    assert torch.allclose(c, a + 0.5 * b, rtol=0, atol=1e-15)
    G.probe_stream(b, None, c)
    torch.cuda.synchronize()
    assert torch.equal(c, b)
    o = torch.empty(1 << 12, dtype=torch.float64, device="cuda")
    G.probe_fma64(o, 100)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(o).all())
