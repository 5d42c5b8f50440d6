"""Serving measurement: baskets of navigation queries arriving as a Poisson
stream at a resident detector geometry, answered by the library's serving
engine (gv_server_*), against a serial server that answers one basket at a time
with the per-kind entry points.

Workload (synthetic): basket sizes n = clip(round(exp(N(ln 1024, ln 4))), 16,
65536); query mix 60 % ComputeStep / 30 % NavSafety / 10 % volume Inside; track
states are mid-flight states (point, direction, placed volume) of origin
tracks of the layered detector, taken at a random step of their transport;
half of the step queries carry a physics limit drawn from U(0, 300) mm.
Offered load = a fraction of the engine's measured saturation rate (baskets/s);
latency = device completion of the basket's round (HIP events mapped to the
host clock) minus its arrival time on the host clock.

The serial form it is compared with is the same engine held to one slot and
one stream: every basket is its own round (copy in, one kernel, copy out) and
the next starts only when it has been returned, i.e. per-basket calls one
after another, with the same arrivals.

    python -m paper_1512_06637_amd.serve [--baskets 20000] [--loads 0.5 0.8 0.95]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import FP32_REFINE, FP64, Q_INSIDE, Q_SAFETY, Q_STEP, Geometry, Server, now, pack_basket, serve_out_bytes
from . import workloads as W

KINDS = (Q_STEP, Q_SAFETY, Q_INSIDE)
MIX = (0.6, 0.3, 0.1)


def state_pool(g, n=1 << 16, seed=5):
    """Mid-flight states: origin tracks transported by the library, each
    replayed on the host to a random step k (p += s d in FP64, the library's
    own update) and paired with the volume it is in after k steps."""
    import torch
    t = W.config3_tracks(n)
    a = [torch.from_numpy(v).to("cuda") for v in t.arrays()]
    r = g.transport(*a)
    ns = r["nsteps"].cpu().numpy()
    st = r["step"].cpu().numpy()
    pvs = r["pv"].cpu().numpy()
    rng = np.random.default_rng(seed)
    k = np.minimum(rng.integers(0, 80, n), np.maximum(ns - 1, 0))
    P = np.stack([t.x, t.y, t.z]).copy()
    D = np.stack([t.dx, t.dy, t.dz])
    for j in range(int(k.max())):
        m = j < k
        P[:, m] = P[:, m] + st[m, j][None, :] * D[:, m]
    pv = pvs[np.arange(n), k].astype(np.int32)
    return W.Tracks(*P, *D), pv


def make_baskets(pool, count, precision, seed):
    t, pv = pool
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(np.clip(np.round(np.exp(rng.normal(np.log(1024), np.log(4)))), 16, 65536))
        kind = KINDS[rng.choice(3, p=MIX)]
        i = rng.integers(0, t.n, n)
        ps = rng.uniform(0, 300, n) if rng.random() < 0.5 else None
        blk = pack_basket(kind, t.x[i], t.y[i], t.z[i], pv[i], t.dx[i], t.dy[i], t.dz[i], ps)
        out.append((kind, precision, n, blk, t.take(i), pv[i], ps))
    return out


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def saturation(srv, baskets, count):
    """Closed loop: keep the engine full; baskets/s, track-queries/s, track-steps/s."""
    t0 = now()
    sub = done = tracks = steps = 0
    while done < count:
        while sub < count:
            kind, prec, n, blk, *_ = baskets[sub % len(baskets)]
            if srv.submit(kind, prec, n, blk, np.empty(serve_out_bytes(kind, n), np.uint8)) is None:
                break
            sub += 1
            tracks += n
            steps += n if kind == Q_STEP else 0
        done += len(srv.poll())
    dt = now() - t0
    return {"baskets_per_s": count / dt, "track_queries_per_s": tracks / dt, "track_steps_per_s": steps / dt}


def open_loop(srv, baskets, count, rate, seed):
    """Poisson arrivals at `rate` baskets/s; returns latency percentiles."""
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1.0 / rate, count))
    t0 = now() + 0.01
    arr = arr + t0
    backlog = []  # arrived, not yet admitted
    ticket_arrival = {}
    lat = []
    tracks = 0
    i = 0
    while len(lat) < count:
        tn = now()
        while i < count and arr[i] <= tn:
            backlog.append(i)
            i += 1
        while backlog:
            j = backlog[0]
            kind, prec, n, blk, *_ = baskets[j % len(baskets)]
            tk = srv.submit(kind, prec, n, blk, np.empty(serve_out_bytes(kind, n), np.uint8))
            if tk is None:
                break
            ticket_arrival[tk] = arr[j]
            tracks += n
            backlog.pop(0)
        for tk, td in srv.poll():
            lat.append(td - ticket_arrival.pop(tk))
    span = now() - t0
    lat_ms = np.array(lat) * 1e3
    return {"offered_baskets_per_s": rate, "achieved_track_queries_per_s": tracks / span,
            "p50_ms": _pct(lat_ms, 50), "p99_ms": _pct(lat_ms, 99), "max_ms": float(lat_ms.max())}


def run(g, loads=(0.5, 0.8, 0.95), precisions=(FP64, FP32_REFINE), n_baskets=20000, serial=True,
        slots=64, hbm_budget=256 << 20, nstreams=2, distinct=256, graphs=True):
    """graphs: rounds as graph launches (the engine's default); the other
    launch form's saturation is measured beside it."""
    pool = state_pool(g)
    res = {"slots": slots, "hbm_budget": hbm_budget, "nstreams": nstreams, "baskets_per_point": n_baskets,
           "rounds_as": "graph launches" if graphs else "plain copies and launch", "points": []}
    for prec in precisions:
        bk = make_baskets(pool, distinct, prec, seed=31 + prec)
        with Server(g, slots, hbm_budget, nstreams, graphs=not graphs) as other:
            saturation(other, bk, min(1000, n_baskets))
            other_sat = saturation(other, bk, min(5000, n_baskets))
        with Server(g, slots, hbm_budget, nstreams, graphs=graphs) as srv:
            saturation(srv, bk, min(2000, n_baskets))  # warm-up
            sat = saturation(srv, bk, min(5000, n_baskets))
            pts = []
            for L in loads:
                r = open_loop(srv, bk, n_baskets, L * sat["baskets_per_s"], seed=41)
                r["load"] = L
                pts.append(r)
            st = srv.stats()
        point = {"precision": "fp64" if prec == FP64 else "fp32_refine", "saturation": sat,
                 "loads": pts, "rounds": st["rounds"], "largest_round": st["max_round"],
                 "saturation_other_launch_form": other_sat}
        if serial:
            # the serial form: one basket per round, one round at a time
            with Server(g, 1, hbm_budget, 1, graphs=graphs) as one:
                saturation(one, bk, min(500, n_baskets))
                ssat = saturation(one, bk, min(2000, n_baskets))
                spts = []
                for L in loads:
                    r = open_loop(one, bk, min(n_baskets, 2000), L * sat["baskets_per_s"], seed=41)
                    r["load"] = L
                    spts.append(r)
            point["serial"] = {"saturation": ssat, "loads": spts,
                               "batching_speedup": sat["baskets_per_s"] / ssat["baskets_per_s"]}
        res["points"].append(point)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--baskets", type=int, default=20000)
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 0.8, 0.95])
    ap.add_argument("--budget-mib", type=int, default=256)
    ap.add_argument("--no-serial", action="store_true")
    ap.add_argument("--streams", type=int, default=2)
    ap.add_argument("--slots", type=int, default=64)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    g = Geometry(W.detector_blob())
    t0 = time.perf_counter()
    r = run(g, loads=args.loads, n_baskets=args.baskets, serial=not args.no_serial,
            hbm_budget=args.budget_mib << 20, nstreams=args.streams, slots=args.slots)
    r["wall_s"] = time.perf_counter() - t0
    g.close()
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
