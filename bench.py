"""Benchmark: FP64 basket navigation through the layered detector on one MI355X.

Workload (one "step" of this benchmark = one nav_transport call over the whole
batch): 2^20 straight tracks starting uniformly in [-1, 1]^3 mm with isotropic
directions, transported through the layered detector (world box 4 x 4 x 6 m,
20 tube layers x 64 box modules, 1,301 placed volumes) until they leave the
world, recording every track's volume sequence and step lengths.  Inputs are
resident in HBM before timing starts.

Metric: track-steps/s = (track-steps the batch takes) / (device time per call).
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def cpu_baseline(blob, tracks, target_s=12.0, max_s=30.0):
    """The CPU oracle on a bounded sample of the same workload (the first tracks,
    in chunks, until about target_s seconds of work), on this host's cores.
    Returns (the baseline record, the oracle's outputs for the sample)."""
    import numpy as np

    import oracle as O

    threads = O.default_threads()
    og = O.Geometry(blob)
    done_tracks = done_steps = 0
    spent = 0.0
    chunk = 8192
    start = 0
    parts = []
    while spent < target_s and start < tracks.n:
        idx = np.arange(start, min(start + chunk, tracks.n))
        t0 = time.perf_counter()
        r = og.transport(tracks.take(idx), threads=threads)
        spent += time.perf_counter() - t0
        parts.append(r)
        done_tracks += idx.size
        done_steps += int(r["nsteps"].sum())
        start += idx.size
        if spent < target_s / 4:
            chunk *= 2
        if spent > max_s:
            break
    og.close()
    ref = {k: np.concatenate([r[k] for r in parts]) for k in parts[0]}
    return ({"value": done_steps / spent, "unit": "track-steps/s", "cores": threads, "kind": "oracle",
             "sample": f"first {done_tracks} of the {tracks.n} tracks ({done_steps} track-steps, {spent:.1f} s)"},
            ref)


# Navigation steps: both codes advance the global point p += s d in FP64; after
# k steps the points differ by up to about k ulp(|p|) (ulp(2048 mm) = 4.5e-13
# mm, k <= 84 here), and a step measured from a shifted point shifts by as much
# over the cosine of the hit angle.  Same bar as the navigation parity tests.
STEP_REL, STEP_ABS = 1e-12, 1e-10


def oracle_parity(ref, out):
    """The GPU transport's outputs against the oracle's on the oracle's sample
    (its first m tracks): volume sequences, step counts and flags bit-exact for
    tracks the oracle does not flag as ill-conditioned (those are counted and
    the first listed), step lengths within STEP_REL relative + STEP_ABS."""
    import numpy as np

    import oracle as O

    m = ref["nsteps"].shape[0]
    ns = out["nsteps"][:m].cpu().numpy()
    fl = out["flags"][:m].cpu().numpy().astype(np.uint32)
    pv = out["pv"][:m].cpu().numpy()
    st = out["step"][:m].cpu().numpy()
    ok = (ref["diag"] & O.D_ILL) == 0
    rn = ref["nsteps"]
    bad_len = (ns != rn) | (fl != ref["flags"])
    k = np.arange(pv.shape[1])[None, :]
    seq_bad = ((pv != ref["pv"]) & (k <= rn[:, None])).any(axis=1)
    mk = k[:, :-1] < rn[:, None]
    with np.errstate(invalid="ignore"):
        err = np.where(mk, np.abs(st - ref["step"]), 0.0)
        tol = STEP_REL * np.maximum(1.0, np.abs(np.where(mk, ref["step"], 0.0))) + STEP_ABS
    step_bad = (mk & ~(err <= tol)).any(axis=1)
    bad = bad_len | seq_bad | step_bad
    flagged = np.nonzero(~ok)[0]
    return {"tracks": int(m), "track_steps": int(rn.sum()), "mismatched_tracks": int((bad & ok).sum()),
            "sequence_mismatches": int(((bad_len | seq_bad) & ok).sum()),
            "flagged_tracks": int(flagged.size), "flagged_first": [int(i) for i in flagged[:20]],
            "flagged_that_differ": int((bad & ~ok).sum()),
            "max_step_err_mm": float(err[ok].max()) if ok.any() else None,
            "bar": f"sequences, counts, flags exact; steps |d| <= {STEP_REL} max(1 mm, |ref|) + {STEP_ABS} mm"}


def roof_probes():
    """What this GPU reaches on the two roofs, measured in this process: a
    stream triad c = a + s b and a copy over 3 x 512 MiB arrays (beyond the
    256 MB last-level cache), and eight independent FP64 FMA chains per lane on
    2^19 lanes.  Medians of 5 timed calls after a warm-up."""
    import torch

    import paper_1512_06637_amd as G

    n = 1 << 26  # 512 MiB per array
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)

    def med(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        ts.sort()
        return ts[len(ts) // 2]

    t_triad = med(lambda: G.probe_stream(a, b, c, 0.5))
    t_copy = med(lambda: G.probe_stream(a, None, c))
    del a, b, c
    lanes, iters = 1 << 19, 8192
    out = torch.empty(lanes, dtype=torch.float64, device="cuda")
    t_fma = med(lambda: G.probe_fma64(out, iters))
    fmas = 8.0 * iters * lanes
    return {"hbm_triad_GBs": 24.0 * n / t_triad / 1e9, "hbm_copy_GBs": 16.0 * n / t_copy / 1e9,
            "fp64_fma_Tlane_ops": fmas / t_fma / 1e12, "fp64_TFLOPs": 2 * fmas / t_fma / 1e12,
            "nominal": {"hbm_GBs": R_PEAK_HBM_GBS, "fp64_Tlane_ops": R_PEAK_FP64_TOPS},
            "method": "triad/copy over 3 x 512 MiB float64 arrays; 8 FMA chains x 8192 on 2^19 lanes; "
                      "median of 5 after warm-up"}


R_PEAK_HBM_GBS = 8000.0
R_PEAK_FP64_TOPS = 256 * 64 * 2.4e9 / 1e12


def kernel_sources_sha256():
    """Hash of the HIP sources and the C-ABI header (file names and bytes)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1512_06637_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "include", "gvgeom.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (k_lane_transport or k_bt_step) on this
    workload from the committed counter summary, or None when the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_detector_2p20_traffic.txt")
    try:
        txt = open(path).read()
    except OSError:
        return None
    sha = val = None
    for line in txt.splitlines():
        if "sha256" in line:
            sha = line.split("sha256")[1].split()[0]
        if line.startswith("traffic_bytes_per_launch:"):
            val = float(line.split(":")[1])
    return val if sha == kernel_sources_sha256() else None


def graph_ms(fn, calls, replays):
    """Per-call device time of `fn(c)`, c = 0 .. calls-1, captured once into a
    HIP graph and replayed: launch overhead of the host stays out."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for c in range(calls):
            fn(c)
    torch.cuda.current_stream().wait_stream(side)
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        for c in range(calls):
            fn(c)
    gr.replay()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(replays):
        gr.replay()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / (replays * calls)


def solids_leg(copies=8, replays=10):
    """The six solids, 2^20 tracks each (a third inside, a third outside, a third
    within 1e-6 mm of the surface): every query separately and fused, cycling
    over `copies` distinct input/output sets (384 MiB of inputs, beyond the
    256 MB last-level cache) so the bytes come from HBM."""
    import torch

    import paper_1512_06637_amd as G
    from paper_1512_06637_amd import roofline as R
    from paper_1512_06637_amd import workloads as W

    names = W.CONFIG2_SOLIDS
    sol = W.config_solids()
    g = G.Geometry(W.multi_solid_blob([sol[k] for k in names]))
    res = {}
    for lv, name in enumerate(names):
        t = W.config2_tracks(name)
        n = t.n
        base = [torch.from_numpy(v).to("cuda") for v in t.arrays()]
        sets = [[v.clone() for v in base] for _ in range(copies)]
        outs = [{"c": torch.empty(n, dtype=torch.int8, device="cuda"),
                 "s": torch.empty(n, dtype=torch.float64, device="cuda"),
                 "a": torch.empty(n, dtype=torch.float64, device="cuda"),
                 "b": torch.empty(n, dtype=torch.float64, device="cuda")} for _ in range(copies)]
        calls = {
            "inside": lambda c: g.inside(lv, *sets[c][:3], out=outs[c]["c"]),
            "safety": lambda c: g.safety(lv, *sets[c][:3], out=outs[c]["s"]),
            "dist_in": lambda c: g.distance(lv, G.TO_IN, *sets[c], out=outs[c]["a"]),
            "dist_out": lambda c: g.distance(lv, G.TO_OUT, *sets[c], out=outs[c]["b"]),
            "fused": lambda c: g.solid_all(lv, *sets[c], outs[c]["c"], outs[c]["s"], outs[c]["a"], outs[c]["b"]),
        }
        r = {}
        for q, f in calls.items():
            ms = graph_ms(f, copies, replays)
            gbs = n * R.SOLID_BYTES[q] / (ms * 1e-3) / 1e9
            ops = None
            if name == "pcon":  # the walk's own work, counted in one call of the query
                g.profile(work=True)
                f(0)
                _, _, work = g.profile_read()
                g.profile()
                ops = R.pcon_ops(q, n, work)
                r.setdefault("walk_counts", {})[q] = work[28:33]
            r[q] = {"us_per_call": ms * 1e3, "tracks_per_s": n / (ms * 1e-3), "GB_s": gbs}
            r[q].update(R.solid_roofline(name, q, n, ms * 1e3, ops=ops))
        r["separate_vs_fused_time"] = sum(r[q]["us_per_call"] for q in ("inside", "safety", "dist_in", "dist_out")) \
            / r["fused"]["us_per_call"]
        res[name] = r
        del sets, outs, base
    g.close()
    return res


def composites_leg(args, copies=4, replays=10, n=1 << 20):
    """Composite solids.  (1) The fused solid-level query of each of the eight
    composites over 2^20 tracks uniform in 1.6 times its bounding box, cycling
    over `copies` input sets.  (2) Transport in the composite geometry (four
    composites, one with daughters, and a tube segment in a 600 mm cube): 2^20
    tracks starting around its volumes, to world exit, FP64; the oracle's rate
    on the first 2^16 of them beside it."""
    import torch

    import oracle as O
    import paper_1512_06637_amd as G
    from paper_1512_06637_amd import workloads as W

    comps = W.composite_solids()
    names = list(comps)
    g = G.Geometry(W.multi_solid_blob([comps[k] for k in names]))
    res = {"solids": {}}
    for lv, name in enumerate(names):
        t = W.composite_box_tracks(comps[name], n, 500 + lv)
        base = [torch.from_numpy(v).to("cuda") for v in t.arrays()]
        sets = [[v.clone() for v in base] for _ in range(copies)]
        outs = [[torch.empty(n, dtype=torch.int8, device="cuda")]
                + [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)] for _ in range(copies)]
        ms = graph_ms(lambda c: g.solid_all(lv, *sets[c], *outs[c]), copies, replays)
        res["solids"][name] = {"fused_us_per_call": ms * 1e3, "tracks_per_s": n / (ms * 1e-3)}
        del sets, outs, base
    g.close()
    blob = W.composite_blob()
    g = G.Geometry(blob)
    t = W.composite_tracks(n)
    a = [torch.from_numpy(v).to("cuda") for v in t.arrays()]
    for _ in range(args.warmup):
        out = g.transport(*a)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        out = g.transport(*a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    total = int(out["nsteps"].sum())
    g.close()
    og = O.Geometry(blob)
    k = 1 << 16
    t0 = time.perf_counter()
    r = og.transport(t.take(slice(0, k)))
    cpu_s = time.perf_counter() - t0
    og.close()
    res["transport"] = {"tracks": n, "track_steps": total, "ms_per_call": ms, "track_steps_per_s": total / (ms * 1e-3),
                        "flags_nonzero": int((out["flags"] != 0).sum()),
                        "oracle_track_steps_per_s": int(r["nsteps"].sum()) / cpu_s,
                        "oracle_cores": O.default_threads(), "oracle_sample": f"first {k} tracks"}
    return res


def protocol_leg(replays=50, calls=100):
    """The paper's measurement protocol: DistanceToOut of points inside the box
    and the tube segment, N = 2^4 .. 2^20, per-call time over 5,000 graph-replayed
    calls."""
    import torch

    import paper_1512_06637_amd as G
    from paper_1512_06637_amd import workloads as W

    sol = W.config_solids()
    g = G.Geometry(W.multi_solid_blob([sol["box"], sol["tubs"]]))
    res = {}
    for lv, name in enumerate(("box", "tubs")):
        pts = []
        full = W.config1_inside_points(name, 1 << 20)
        for e in range(4, 21, 2):
            n = 1 << e
            a = [torch.from_numpy(v[:n].copy()).to("cuda") for v in full.arrays()]
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            ms = graph_ms(lambda c: g.distance(lv, G.TO_OUT, *a, out=out), calls, max(1, replays // max(1, n >> 16)))
            pts.append({"n": n, "us_per_call": ms * 1e3, "tracks_per_s": n / (ms * 1e-3)})
        res[name] = pts
    g.close()
    return res


def cpu_baseline_solids(protocol, max_s=1.0):
    """The oracle on the same inputs: DistanceToIn / DistanceToOut of the full
    solid set on 2^16-track samples, and the protocol sweep's DistanceToOut for
    each N (repeated up to `max_s` seconds)."""
    import oracle as O
    from paper_1512_06637_amd import workloads as W

    threads = O.default_threads()
    sol = W.config_solids()
    full = {}
    for name in W.CONFIG2_SOLIDS:
        t = W.config2_tracks(name).take(slice(0, 1 << 16))
        r = {}
        for q, d in (("dist_in", 0), ("dist_out", 1)):
            t0 = time.perf_counter()
            O.distance(sol[name], d, t, threads=threads)
            r[q + "_tracks_per_s"] = t.n / (time.perf_counter() - t0)
        full[name] = r
    proto = {}
    for name, pts in protocol.items():
        allp = W.config1_inside_points(name, 1 << 20)
        out = []
        for p in pts:
            t = allp.take(slice(0, p["n"]))
            k, t0 = 0, time.perf_counter()
            while True:
                O.distance(sol[name], 1, t, threads=threads)
                k += 1
                el = time.perf_counter() - t0
                if el > max_s or (k >= 3 and el > 0.05):
                    break
            cpu = k * p["n"] / el
            out.append({"n": p["n"], "tracks_per_s": cpu, "gpu_speedup": p["tracks_per_s"] / cpu})
        proto[name] = out
    return {"kind": "oracle", "cores": threads, "solids_sample": "first 2^16 tracks of each solid's set",
            "solids": full, "protocol": proto}


def _time_calls(fn, calls):
    """Device time per call of `fn` over `calls` calls, HIP events on the current
    stream (the one the library launches on)."""
    import torch
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(calls):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / calls


def phys_leg(g, a, args, max_steps=256):
    """Physics-limited transport of the same tracks (synthetic materials: mean
    free paths 60-400 mm in the modules, 5e3-1e5 mm in the layers, 2e5-1e6 mm
    in the world), with and without the safety short-cut."""
    import torch

    from paper_1512_06637_amd import workloads as W

    m = W.detector_materials()
    g.set_materials(m["density"], m["sigma"], m["lv_mat"])
    n = a[0].shape[0]
    out = {"pv": torch.empty((n, max_steps + 1), dtype=torch.int32, device="cuda"),
           "step": torch.empty((n, max_steps), dtype=torch.float64, device="cuda"),
           "proc": torch.empty((n, max_steps), dtype=torch.int8, device="cuda"),
           "nsteps": torch.empty(n, dtype=torch.int32, device="cuda"),
           "flags": torch.empty(n, dtype=torch.int32, device="cuda")}
    res = {}
    for short in (True, False):
        run = lambda: g.transport_phys(*a, W.PHYS_SEED, max_steps=max_steps, out=out, shortcut=short)  # noqa: E731
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        ms = _time_calls(run, args.steps)
        g.profile(work=True)
        run()
        _, _, work = g.profile_read()
        g.profile()
        total = int(out["nsteps"].sum())
        res["shortcut" if short else "no_shortcut"] = {
            "ms_per_step": ms, "track_steps_per_s": total / (ms * 1e-3), "track_steps": total,
            "physics_limited_steps": work[22], "shortcut_steps": work[23]}
    return res


def fp32_leg(g, a, ref, max_steps, args, ms64, oracle_ref=None):
    """The same workload with precision FP32_REFINE (FP32 daughter screens, FP64
    distances): time per call, whether every output equals the FP64 run's, the
    oracle parity of its outputs, and the share of culled track-steps whose
    screens ran in FP32."""
    import torch

    import paper_1512_06637_amd as G

    n = ref["nsteps"].shape[0]
    out = {k: torch.empty_like(v) for k, v in ref.items()}
    run = lambda: g.transport(*a, max_steps=max_steps, out=out, precision=G.FP32_REFINE)  # noqa: E731
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    ms = _time_calls(run, args.steps)
    g.profile(events=True)
    run()
    step_ms, _, _ = g.profile_read()
    g.profile(work=True)
    run()
    _, _, work = g.profile_read()
    g.profile()
    run()
    torch.cuda.synchronize()
    ns = ref["nsteps"]
    k = torch.arange(max_steps, device=ns.device)[None, :]
    m = k < ns[:, None].long()
    mp = torch.cat([torch.ones((n, 1), dtype=torch.bool, device=ns.device), m], dim=1)
    same = (torch.equal(ns, out["nsteps"]) and torch.equal(ref["flags"], out["flags"])
            and torch.equal(ref["pv"][mp], out["pv"][mp])
            and torch.equal(ref["step"][m].view(torch.int64), out["step"][m].view(torch.int64)))
    total = int(ns.sum())
    r = {"ms_per_step": ms, "value": total / (ms * 1e-3), "speedup_vs_fp64": ms64 / ms,
         "kernel_ms_per_transport": step_ms, "identical_to_fp64": bool(same),
         "fp32_screened_frac": work[20] / max(1, work[20] + work[21]),
         "daughter_box_tests": work[1], "dist_in_box_tube": work[8:10]}
    if oracle_ref is not None:
        r["oracle_parity"] = oracle_parity(oracle_ref, out)
    return r


def serving_leg(baskets=3000):
    """The serving engine (continuous batching: slots 64, HBM budget 256 MiB,
    2 streams) and the same engine serving one basket at a time (1 slot, 1
    stream: the serial per-basket form), FP64 and FP32_REFINE, Poisson arrivals
    at 0.5 / 0.8 / 0.95 of the batching engine's saturation rate; `baskets`
    baskets per point."""
    import paper_1512_06637_amd as G
    from paper_1512_06637_amd import serve as S
    from paper_1512_06637_amd import workloads as W

    g = G.Geometry(W.detector_blob())
    try:
        return S.run(g, n_baskets=baskets)
    finally:
        g.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-screen + FP64-refine leg")
    ap.add_argument("--no-solids", action="store_true", help="skip the solid-level legs")
    ap.add_argument("--no-phys", action="store_true", help="skip the physics-limited transport leg")
    ap.add_argument("--no-composites", action="store_true", help="skip the composite-solid legs")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-probes", action="store_true", help="skip the HBM and FP64 roof probes")
    ap.add_argument("--transport", choices=["tuned", "lane", "basket"], default="tuned",
                    help="transport form of the navigation legs: the stored tuning's (default), or forced")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 256 MiB device to device (a kernel of known traffic for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "tracks are independent, so more GPUs would each transport a contiguous shard", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1512_06637_amd as G
    from paper_1512_06637_amd import roofline as R
    from paper_1512_06637_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    blob = W.detector_blob()
    tracks = W.config3_tracks(args.n)
    g = G.Geometry(blob)
    if args.transport != "tuned":
        g.set_tuning(**dict(g.get_tuning(), transport=1 if args.transport == "basket" else 2))
    a = [torch.from_numpy(v).to("cuda") for v in tracks.arrays()]
    max_steps = 128
    n = tracks.n
    out = {
        "pv": torch.empty((n, max_steps + 1), dtype=torch.int32, device="cuda"),
        "step": torch.empty((n, max_steps), dtype=torch.float64, device="cuda"),
        "nsteps": torch.empty(n, dtype=torch.int32, device="cuda"),
        "flags": torch.empty(n, dtype=torch.int32, device="cuda"),
    }
    run = lambda: g.transport(*a, max_steps=max_steps, out=out)  # noqa: E731
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = _time_calls(run, args.steps)
    wall = time.perf_counter() - t0

    # the transport kernel alone (the persistent lane kernel, or each launch of
    # the basket form's per-step kernel): HIP events around its launches, on
    # the stream the library launches on, over the same number of calls
    lane_form = g.get_tuning()["transport"] != 1
    kernel = "k_lane_transport" if lane_form else "k_bt_step"
    g.profile(events=True)
    for _ in range(args.steps):
        run()
    step_ms_total, launches, _ = g.profile_read()
    # operation counts: one call of the basket form's counting instance (every
    # track takes the same steps, with the same daughter work, in both forms)
    g.profile(work=True)
    run()
    _, _, work = g.profile_read()
    g.profile()
    run()  # outputs of the production kernels for the parity check below
    torch.cuda.synchronize()
    step_ms = step_ms_total / args.steps  # transport-kernel time per transport
    launches_per = launches / args.steps
    launch_ms = step_ms_total / max(1, launches)

    ns = out["nsteps"].cpu().numpy()
    pv = out["pv"].cpu().numpy()
    flags = out["flags"].cpu().numpy()
    total_steps = int(ns.sum())
    world, layer, module = R.detector_step_classes(pv, ns)
    del pv
    ops_plain = R.detector_ops(world, layer, module)
    ops = R.detector_ops_culled(world, layer, module, work)
    alg_bytes = R.transport_bytes(n, total_steps)
    design_bytes = alg_bytes + 8 * n if lane_form else total_steps * R.STEP_DESIGN_BYTES
    intensity = ops / alg_bytes
    balance = R.PEAK_FP64_OPS / R.PEAK_HBM
    achieved = ops / (step_ms * 1e-3)  # = ops per launch / average launch duration
    traffic = measured_traffic(kernel)
    roofs = None if args.no_probes else roof_probes()
    roofline = {
        "bound": "alu" if intensity > balance else "hbm",
        "kernel": kernel,
        "achieved": achieved / 1e12,
        "peak": R.PEAK_FP64_OPS / 1e12,
        "unit": "T FP64 lane-ops/s (an FMA counts 1; peak = 256 CU x 64 lanes x 2.4 GHz = 78.6 TFLOP/s)",
        "frac": achieved / R.PEAK_FP64_OPS,
        "traffic": traffic,
        "ops_per_transport": ops,
        "ops_per_launch": ops / launches_per,
        "launches_per_transport": launches_per,
        "avg_launch_ms": launch_ms,
        "kernel_ms_per_transport": step_ms,
        "algorithmic_bytes_per_transport": alg_bytes,
        "ops_per_algorithmic_byte": intensity,
        "machine_balance_ops_per_byte": balance,
        "frac_measured_fp64_roof": achieved / (roofs["fp64_fma_Tlane_ops"] * 1e12) if roofs else None,
        "hbm": {"algorithmic_GBs": alg_bytes / (ms * 1e-3) / 1e9,
                "frac_algorithmic": alg_bytes / (ms * 1e-3) / R.PEAK_HBM,
                "design_bytes_per_launch": design_bytes / launches_per,
                "measured_traffic_per_launch": traffic,
                "measured_traffic_over_algorithmic": (traffic * launches_per / alg_bytes) if traffic else None,
                "frac_measured_traffic": (traffic / (launch_ms * 1e-3) / R.PEAK_HBM) if traffic else None},
        "accounting": "ops = the culled navigator's own work from its operation counters x the per-operation "
                      "table of roofline.py; bytes = inputs once + outputs once (transport_bytes); design bytes = "
                      "those plus the lane form's direction keys and order (8 B per track), or the basket form's "
                      "152 B per track-step",
    }
    res = {
        "metric": "track-steps/s",
        "value": total_steps / (ms * 1e-3),
        "unit": "track-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "layered-detector navigation FP64: 2^20 origin tracks to world exit, 1301 PVs",
                   "tracks": n, "track_steps": total_steps, "max_steps": max_steps,
                   "steps_world_layer_module": [world, layer, module]},
        "roofline": roofline,
        "roofs": roofs,
        "tuning": g.get_tuning(),
        "work": {"plain_navigator_ops": ops_plain, "culled_ops": ops, "daughter_box_tests": work[1],
                 "bound_checks_box_tube": work[2:4], "dist_in_box_tube": work[8:10], "steps": work[0],
                 "radial_lookups": work[24], "radial_bounds": work[25], "phi_lookups": work[26],
                 "phi_sectors_read": work[27]},
        "wall_s": wall,
        "flags_nonzero": int((flags != 0).sum()),
    }
    oracle_ref = None
    if not args.no_cpu_baseline:
        res["cpu_baseline"], oracle_ref = cpu_baseline(blob, tracks)
        res["oracle_parity"] = oracle_parity(oracle_ref, out)
    if not args.no_fp32:
        res["fp32_refine"] = fp32_leg(g, a, out, max_steps, args, ms, oracle_ref)
    del oracle_ref
    if not args.no_phys:
        res["physics_limited"] = phys_leg(g, a, args)
    g.close()
    del out, a
    if not args.no_serving:
        res["serving"] = serving_leg()
    if not args.no_solids:
        res["solids"] = solids_leg()
        res["protocol"] = protocol_leg()
        if not args.no_cpu_baseline:
            res["cpu_baseline_solids"] = cpu_baseline_solids(res["protocol"])
    if not args.no_composites:
        res["composites"] = composites_leg(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
