"""GPU tests of the serving engine (gv_server_*): baskets of mixed queries
answered in shared rounds give exactly what each basket gets alone from the
basket_* entry points, and those answers match the oracle; admission by slots
and HBM budget pushes back (GV_EAGAIN) and recovers."""
import numpy as np
import pytest

import oracle as O
from paper_1512_06637_amd import workloads as W
from tests.gpu_util import compare_values, cuda, host, say
from tests.test_gpu_nav import STEP_REL, states

pytestmark = pytest.mark.gpu

BLOB = W.detector_blob()


@pytest.fixture(scope="module")
def geos():
    import paper_1512_06637_amd as G
    g = G.Geometry(BLOB)
    og = O.Geometry(BLOB)
    yield g, og
    g.close()
    og.close()


@pytest.fixture(scope="module")
def pool(geos):
    _, og = geos
    t, pv = states(og, 6000, 21)
    return t, pv


def make_baskets(pool, count, seed, max_n=4096):
    import paper_1512_06637_amd as G
    t, pv = pool
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(np.clip(np.round(np.exp(rng.normal(np.log(256), np.log(4)))), 1, max_n))
        kind = [G.Q_STEP, G.Q_SAFETY, G.Q_INSIDE][rng.choice(3, p=[0.6, 0.3, 0.1])]
        prec = [G.FP64, G.FP32_REFINE][rng.integers(2)]
        idx = rng.integers(0, t.n, n)
        ps = rng.uniform(0, 300, n) if rng.random() < 0.5 else np.full(n, np.inf)
        out.append(dict(kind=kind, prec=prec, n=n, idx=idx, pstep=ps))
    return out


def pack(b, pool):
    import paper_1512_06637_amd as G
    t, pv = pool
    i = b["idx"]
    return G.pack_basket(b["kind"], t.x[i], t.y[i], t.z[i], pv[i], t.dx[i], t.dy[i], t.dz[i], b["pstep"])


def alone(g, b, pool):
    """The same basket through the per-kind entry point, on its own."""
    import torch
    import paper_1512_06637_amd as G
    t, pv = pool
    i = b["idx"]
    a = [cuda(v[i]) for v in t.arrays()]
    p = cuda(pv[i])
    if b["kind"] == G.Q_STEP:
        fl = torch.zeros(b["n"], dtype=torch.int32, device="cuda")
        st, nx = g.step(*a, p, pstep=cuda(b["pstep"]), out_flags=fl, precision=b["prec"])
        return host(st), host(nx), host(fl).view(np.uint32)
    if b["kind"] == G.Q_SAFETY:
        return host(g.nav_safety(*a[:3], p, precision=b["prec"]))
    return host(g.nav_inside(*a[:3], p))


def run_server(srv, baskets, pool):
    """Submits every basket (polling while the server pushes back), drains,
    and returns the output blocks and the number of GV_EAGAIN answers."""
    import paper_1512_06637_amd as G
    outs, tickets, again = [], {}, 0
    for j, b in enumerate(baskets):
        inb = pack(b, pool)
        ob = np.zeros(G.serve_out_bytes(b["kind"], b["n"]), np.uint8)
        outs.append(ob)
        while True:
            tk = srv.submit(b["kind"], b["prec"], b["n"], inb, ob)
            if tk is not None:
                tickets[tk] = j
                break
            again += 1
            for tkd, _ in srv.poll():
                tickets.pop(tkd)
    srv.drain()
    for tkd, _ in srv.poll(4096):
        tickets.pop(tkd)
    assert not tickets
    return outs, again


def check_equal(kind, got, ref):
    import paper_1512_06637_amd as G
    if kind == G.Q_STEP:
        assert np.array_equal(got[0].view(np.int64), ref[0].view(np.int64))
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
    elif kind == G.Q_SAFETY:
        assert np.array_equal(got.view(np.int64), ref.view(np.int64))
    else:
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("graphs", [True, False])
def test_serve_mixed_rounds_equal_alone(geos, pool, graphs):
    """Every basket served in a round of several (as one graph launch per round
    with the round's node parameters, or as plain copies and a launch) equals
    the same basket answered alone by basket_step / _nav_safety / _nav_inside,
    bit for bit, and the oracle."""
    import paper_1512_06637_amd as G
    g, og = geos
    baskets = make_baskets(pool, 60, 22)
    say(f"[serve] graphs={graphs}: {len(baskets)} baskets, {sum(b['n'] for b in baskets)} tracks")
    with G.Server(g, slots=16, hbm_budget=64 << 20, nstreams=2, graphs=graphs) as srv:
        outs, _ = run_server(srv, baskets, pool)
        st = srv.stats()
    say(f"  stats {st}")
    assert st["baskets"] == len(baskets) and st["admitted"] == 0 and st["in_bytes"] == 0
    assert st["max_round"] > 1  # some round served several baskets
    t, pv = pool
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


@pytest.mark.parametrize("graphs", [True, False])
def test_serve_backpressure(geos, pool, graphs):
    """A 16 MiB budget holds only a few 65,536-track step baskets (3.75 MiB of
    inputs each): the server answers GV_EAGAIN until rounds complete, the
    arenas wrap (rounds with two copy runs), and every basket is still answered
    exactly."""
    import paper_1512_06637_amd as G
    g, _ = geos
    rng = np.random.default_rng(23)
    t, pv = pool
    baskets = [dict(kind=G.Q_STEP, prec=G.FP64, n=65536, idx=rng.integers(0, t.n, 65536),
                    pstep=np.full(65536, np.inf)) for _ in range(6)]
    baskets += make_baskets(pool, 10, 24)
    with G.Server(g, slots=64, hbm_budget=16 << 20, nstreams=2, graphs=graphs) as srv:
        outs, again = run_server(srv, baskets, pool)
        big = np.zeros(G.serve_out_bytes(G.Q_STEP, 1 << 20), np.uint8)
        with pytest.raises(G.GVError) as e:
            srv.submit(G.Q_STEP, G.FP64, 1 << 20, np.zeros(G.serve_in_bytes(G.Q_STEP, 1 << 20), np.uint8), big)
        assert e.value.code == G.GV_EINVAL
    say(f"  GV_EAGAIN answers: {again}")
    assert again > 0
    for b, ob in zip(baskets, outs):
        check_equal(b["kind"], G.unpack_result(b["kind"], ob, b["n"]), alone(g, b, pool))


def test_serve_edges(geos, pool):
    """One-track baskets, invalid volume ids, an idle poll, slot limit 1."""
    import paper_1512_06637_amd as G
    g, _ = geos
    t, pv = pool
    with G.Server(g, slots=1, hbm_budget=1 << 20, nstreams=1) as srv:
        assert srv.poll() == []
        b = dict(kind=G.Q_STEP, prec=G.FP32_REFINE, n=1, idx=np.array([5]), pstep=np.array([np.inf]))
        ob = np.zeros(16, np.uint8)
        tk = srv.submit(G.Q_STEP, G.FP32_REFINE, 1, pack(b, pool), ob)
        assert tk is not None
        assert srv.submit(G.Q_INSIDE, G.FP64, 1, pack(dict(kind=G.Q_INSIDE, idx=np.array([5]), pstep=None), pool),
                          np.zeros(1, np.uint8)) is None  # the one slot is taken
        srv.drain()
        assert [x[0] for x in srv.poll()] == [tk]
        check_equal(G.Q_STEP, G.unpack_result(G.Q_STEP, ob, 1), alone(g, b, pool))
        bad = G.pack_basket(G.Q_STEP, t.x[:3], t.y[:3], t.z[:3], np.array([-1, 99999, 0], np.int32),
                            t.dx[:3], t.dy[:3], t.dz[:3])
        ob = np.zeros(48, np.uint8)
        srv.submit(G.Q_STEP, G.FP64, 3, bad, ob)
        srv.drain()
        srv.poll()
        st, nx, fl = G.unpack_result(G.Q_STEP, ob, 3)
        assert list(nx[:2]) == [-1, -1] and list(fl[:2]) == [4, 4] and list(st[:2]) == [0.0, 0.0]
