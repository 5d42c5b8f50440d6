"""Algorithmic work accounting for the roofline figures of the benchmark.

An "op" is one FP64 VALU lane operation of the minimal per-track formulation:
add, sub, mul, fma, min, max and compare count 1 each, and so do a division and
a square root (which cost several instructions on CDNA).  The per-step figures
are those of the plain navigator: the mother's DistanceToOut plus, for every
daughter, the placement transform and its DistanceToIn (Sec. III.A/III.C).

Peak: MI355X has 256 CUs x 4 SIMDs x 16 FP64 lanes at 2.4 GHz = 39.32e12 FP64
lane-ops/s (78.6 TFLOP/s when every op is an FMA).  HBM3E peak 8 TB/s.
"""
PEAK_FP64_OPS = 256 * 64 * 2.4e9  # 39.32e12 lane-ops/s
PEAK_HBM = 8.0e12  # B/s

TRANSFORM = 21      # p_loc = R^T (p - t): 3 sub + 9 mul/fma; d_loc = R^T d: 9
BOX_DIST_IN = 33    # inside test 6, three slabs 24, clip + chord test 3
BOX_DIST_OUT = 16   # inside test 6, three exit planes 9, clamp 1
TUBE_DIST_IN = 53   # inside test 9, outer cylinder 16, z slab 6, inner cylinder 12, pieces 10
TUBE_DIST_OUT = 53
SELECT = 1          # running minimum over candidates, per candidate
STEP_FIXED = 9      # final selection (3) + advance p += s d (6)

# ops per ComputeStep by the class of the current volume in the layered detector
OPS_WORLD_STEP = TRANSFORM + BOX_DIST_OUT + 20 * (TRANSFORM + TUBE_DIST_IN + SELECT) + STEP_FIXED
OPS_LAYER_STEP = TRANSFORM + TUBE_DIST_OUT + 64 * (TRANSFORM + BOX_DIST_IN + SELECT) + STEP_FIXED
OPS_MODULE_STEP = TRANSFORM + BOX_DIST_OUT + STEP_FIXED

# Design traffic of one basket step of one track (k_bt_step): its list entry
# (4), its 64-byte record read and rewritten (128), the staged step length and
# next volume (12), its next bucket and its place in the next list (8).  This is
# what the basket design moves, not what the method needs: the algorithmic
# bytes of a transport are transport_bytes() below (inputs once, outputs once).
STEP_DESIGN_BYTES = 4 + 128 + 12 + 8


# bytes that must move per track of a transport: the SoA start state in
# (6 doubles) and the outputs (start PV, per step one int32 PV and one double
# step, nsteps, flags)
def transport_bytes(n_tracks: int, n_steps_total: int) -> int:
    return n_tracks * (48 + 4 + 4 + 4) + n_steps_total * (4 + 8)


def detector_step_classes(pv_rows, nsteps, n_modules=64):
    """Counts of steps taken from the world, a layer and a module, read from the
    transport's own PV sequences (PV 0 world, 1 + 65 i layer i, else module)."""
    import numpy as np

    pv = np.asarray(pv_rows)
    ns = np.asarray(nsteps)
    k = np.arange(pv.shape[1] - 1)[None, :]
    cur = pv[:, :-1]
    valid = k < ns[:, None]
    stride = n_modules + 1
    world = int(np.sum(valid & (cur == 0)))
    layer = int(np.sum(valid & (cur > 0) & ((cur - 1) % stride == 0)))
    module = int(np.sum(valid)) - world - layer
    return world, layer, module


def detector_ops(world, layer, module) -> float:
    """Plain navigator: every daughter's DistanceToIn at every step."""
    return float(world) * OPS_WORLD_STEP + float(layer) * OPS_LAYER_STEP + float(module) * OPS_MODULE_STEP


# Culled navigator (the daughter loops that run): a bounding-box test per
# daughter (6 fma, 6 min/max per axis pair, 4 to combine, 3 compares, 1 select),
# then per candidate the point transform (12) and the child's SafetyToIn bound,
# then for survivors the direction transform (9), DistanceToIn and the select.
AABB_TEST = 20
RAY_SETUP = 6  # three reciprocals and three products per step
SAFETY_IN = {0: 5, 1: 9}        # box, tube (by daughter solid type)
DIST_IN = {0: BOX_DIST_IN, 1: TUBE_DIST_IN}
DIST_OUT = {"world": BOX_DIST_OUT, "layer": TUBE_DIST_OUT, "module": BOX_DIST_OUT}


# Radial walk (an LV whose daughters are concentric tubes, the detector's
# world): per step rho^2, A, B (9), the count of tubes with rmin^2 <= rho^2
# over the world's 20 tubes (2 each), the holding test (1) and the test that
# the ray leaves a held tube at once (4); per crossing bound C, the
# discriminant, a square root, the stable root and the margin test (12).
RADIAL_LOOKUP = 9 + 2 * 20 + 1 + 4
RADIAL_BOUND = 12
# Phi sectors (the detector's layers): per step the segment end (4), the
# closest approach to the axis (13), its guard (7), two pseudo-angles (8 each,
# with a division), the turning sense (3) and two sector indices (4); per
# sector read one OR and one compare.
PHI_LOOKUP = 4 + 13 + 7 + 16 + 3 + 4
PHI_SECTOR = 2


def detector_ops_culled(world, layer, module, work) -> float:
    """Operation count of the culled navigator from the library's work counters
    ([0] steps, [1] box tests, [2+t] bound checks, [8+t] culled DistanceToIn,
    [14+t] plain DistanceToIn, t = daughter solid type, [24] radial lookups,
    [25] radial crossing bounds, [26] phi-sector lookups, [27] sectors read)."""
    fixed = TRANSFORM + STEP_FIXED
    ops = world * (fixed + DIST_OUT["world"] + RAY_SETUP) + layer * (fixed + DIST_OUT["layer"] + RAY_SETUP)
    ops += module * (fixed + DIST_OUT["module"])
    ops += work[1] * AABB_TEST
    for t in (0, 1):
        ops += work[2 + t] * (12 + SAFETY_IN[t])
        ops += work[8 + t] * (9 + DIST_IN[t] + SELECT)
        ops += work[14 + t] * (TRANSFORM + DIST_IN[t] + SELECT)
    if len(work) > 25:
        ops += work[24] * RADIAL_LOOKUP + work[25] * RADIAL_BOUND
    if len(work) > 27:
        ops += work[26] * PHI_LOOKUP + work[27] * PHI_SECTOR
    return float(ops)


# Solid-level queries: algorithmic FP64 lane-ops per track of the minimal
# per-track formulation (same op definition as above; a division or a square
# root counts 1), per solid and query.  Box and tube segment are the counts
# above; the others are estimates of their formulas (cone: two normalised
# cone terms and a z slab; sphere shell: one radius; Trd: two normalised slab
# pairs; polycone with 10 z-planes: the section search and, per section, a
# cone quadric for the distances and a point-segment distance for the exact
# meridian safety).  Fused = all four answers from one read of the track.
SOLID_OPS = {
    "box": {"inside": 7, "safety": 7, "dist_in": BOX_DIST_IN, "dist_out": BOX_DIST_OUT},
    "tubs": {"inside": 16, "safety": 22, "dist_in": TUBE_DIST_IN, "dist_out": TUBE_DIST_OUT},
    "cons": {"inside": 14, "safety": 14, "dist_in": 60, "dist_out": 45},
    "sphere": {"inside": 6, "safety": 7, "dist_in": 25, "dist_out": 20},
    "trd": {"inside": 12, "safety": 12, "dist_in": 45, "dist_out": 20},
    "pcon": {"inside": 20, "safety": 199, "dist_in": 370, "dist_out": 315},
}

# Polycone (the full-set polycone: 10 z-planes, rmin 0), from the walk's own
# work counters (gv_profile_read [28..32]); the dist_in / dist_out entries of
# SOLID_OPS above are the full walk over all 9 sections.
#   inside: section search over the 8 inner planes (8), r (3 + 1 root), the
#     cone term and its normalisation (5), the two caps and their max (3) = 20;
#   safety: r (4), per side segment (9) and cap (2) of the meridian polygon the
#     point-segment squared distance with its precomputed 1/|e|^2 (15) and the
#     running minimum (1), two hollowness tests per side, one final root
#     = 4 + 11 * 16 + 9 * 2 + 1 = 199;
#   per walked section: the z slab (6; the reciprocal of dz once per walk), the
#     outer cone quadric (rz 2, A 4, B 4, C 4, discriminant 3, root 1, q 2, two
#     divisions 2, min/max 2, clip to the slab 2 = 26), the pieces (8), the
#     merge and early-stop tests (4) = 44;
#   per walk: the section search again (8), direction set-up and the
#     reciprocal of dz (4), the return (3) = 15;
#   DistanceToIn of an outside point also tests the bounding cylinder first
#     (its quadric 20, z slab 6, interval and test 4 = 30).
PCON_INSIDE = 20
PCON_SAFETY = 199
PCON_SECTION = 44
PCON_WALK = 15
PCON_REJECT = 30


def pcon_ops(query: str, n: int, work) -> float:
    """Operation count of a polycone query over n tracks from the walk counters
    of that call ([28] DistanceToIn sections, [29] DistanceToOut sections, [30]
    bounding-cylinder rejects, [31] DistanceToIn walks, [32] DistanceToOut
    walks).  The fused query computes the inside code once."""
    sec_in, sec_out, rej, w_in, w_out = (float(v) for v in work[28:33])
    din = (rej + w_in) * PCON_REJECT + w_in * PCON_WALK + sec_in * PCON_SECTION
    dout = w_out * PCON_WALK + sec_out * PCON_SECTION
    if query == "inside":
        return n * float(PCON_INSIDE)
    if query == "safety":
        return n * float(PCON_INSIDE + PCON_SAFETY)
    if query == "dist_in":
        return n * float(PCON_INSIDE) + din
    if query == "dist_out":
        return n * float(PCON_INSIDE) + dout
    return n * float(PCON_INSIDE + PCON_SAFETY) + din + dout
for _v in SOLID_OPS.values():
    _v["fused"] = _v["inside"] + _v["safety"] + _v["dist_in"] + _v["dist_out"]

# Algorithmic HBM bytes per track of the solid-level queries: inputs read (3 or
# 6 doubles) and outputs written (int8 code, doubles).
SOLID_BYTES = {"inside": 24 + 1, "safety": 24 + 8, "dist_in": 48 + 8, "dist_out": 48 + 8, "fused": 48 + 25}


def solid_roofline(solid: str, query: str, n: int, us_per_call: float, hbm_peak=PEAK_HBM, alu_peak=PEAK_FP64_OPS,
                   ops=None):
    """Both fractions of one solid-level call and the roof that bounds it (the
    larger of the two roofline times).  ops: the call's operation count when
    it is measured (polycone walks), else the SOLID_OPS table's per track."""
    ops = SOLID_OPS[solid][query] * n if ops is None else ops
    byt = SOLID_BYTES[query] * n
    s = us_per_call * 1e-6
    t_alu, t_hbm = ops / alu_peak, byt / hbm_peak
    return {"bound": "alu" if t_alu > t_hbm else "hbm", "frac_alu": ops / s / alu_peak,
            "frac_hbm": byt / s / hbm_peak, "frac": max(t_alu, t_hbm) / s, "ops_per_track": ops / n,
            "bytes_per_track": SOLID_BYTES[query]}
