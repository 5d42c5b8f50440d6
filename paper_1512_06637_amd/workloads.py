"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle's tests.

This module only *describes* geometries and *draws* inputs.  It holds none of the
method's arithmetic: no Inside classification with tolerance, no distances, no
safeties, no navigation.  Both sides (the HIP library and the CPU oracle) parse the
geometry blob written here with their own parsers and derive their own constants.

Geometry model (paper Sec. III.B: elementary solids, coordinate transforms, and a
hierarchy that builds the detector as an ordered system of building blocks):

* a logical volume (LV) = one elementary solid + an ordered list of daughter
  placements (child LV, rotation R, translation t), with x_mother = R x_child + t;
* placed volumes (PVs) are the expansion of that tree from the world LV in DFS
  pre-order, so PV 0 is the world and a PV id is a full navigation state.

Blob layout (little endian, version 1):

  header, 32 B : magic b"GVGEOM\\0\\1", u32 version, u32 n_lv, u32 n_place,
                 u32 n_param, u32 world_lv, u32 reserved
  LV table     : n_lv x {i32 solid_type, i32 param_off, i32 param_cnt,
                         i32 place_off, i32 place_cnt, i32 pad[3]}      (32 B)
  placements   : n_place x {i32 child_lv, i32 pad, f64 R[9] (row major), f64 t[3]} (104 B)
  params       : n_param x f64

Solid types and parameters (lengths in mm, angles in rad):
  0 box      dx dy dz                                  (half-lengths)
  1 tubs     rmin rmax dz sphi dphi                    (dz half-length)
  2 cons     rmin1 rmax1 rmin2 rmax2 dz sphi dphi      (radii at -dz / +dz)
  3 sphere   rmin rmax                                 (full shell)
  4 trd      dx1 dx2 dy1 dy2 dz                        (half-widths at -dz / +dz)
  5 pcon     nz z[nz] rmin[nz] rmax[nz]                (full phi)
  6 bool     op tA nA A[nA] tC nC C[nC] R[9] t[3]      (composite of two solids of
             types 0-5: op 0 union, 1 A minus C, 2 intersection; A at the
             composite's origin, C placed by x = R x_C + t, R row major)

Track sets follow the paper's workload of randomly placed particles with random
directions (Sec. III.C speed test); the concrete recipes are the five benchmark
configurations of this project.
"""
from __future__ import annotations

import hashlib
import math
import struct
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1512066370
MAGIC = b"GVGEOM\x00\x01"
VERSION = 1

BOX, TUBS, CONS, SPHERE, TRD, PCON, BOOL = 0, 1, 2, 3, 4, 5, 6
UNION, SUBTRACTION, INTERSECTION = 0, 1, 2
SOLID_NAMES = {BOX: "box", TUBS: "tubs", CONS: "cons", SPHERE: "sphere", TRD: "trd", PCON: "pcon", BOOL: "bool"}
TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------- solids
@dataclass
class Solid:
    type: int
    params: list

    @property
    def name(self) -> str:
        return SOLID_NAMES[self.type]


def box(dx, dy, dz):
    return Solid(BOX, [dx, dy, dz])


def tubs(rmin, rmax, dz, sphi=0.0, dphi=TWO_PI):
    return Solid(TUBS, [rmin, rmax, dz, sphi, dphi])


def cons(rmin1, rmax1, rmin2, rmax2, dz, sphi=0.0, dphi=TWO_PI):
    return Solid(CONS, [rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi])


def sphere(rmin, rmax):
    return Solid(SPHERE, [rmin, rmax])


def trd(dx1, dx2, dy1, dy2, dz):
    return Solid(TRD, [dx1, dx2, dy1, dy2, dz])


def pcon(z, rmin, rmax):
    z, rmin, rmax = list(map(float, z)), list(map(float, rmin)), list(map(float, rmax))
    assert len(z) == len(rmin) == len(rmax) >= 2
    return Solid(PCON, [float(len(z))] + z + rmin + rmax)


def boolean(op, a: Solid, c: Solid, R=None, t=(0.0, 0.0, 0.0)) -> Solid:
    """Composite op(A, C) of two elementary solids; C placed by x = R x_C + t."""
    assert a.type != BOOL and c.type != BOOL and op in (UNION, SUBTRACTION, INTERSECTION)
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
    return Solid(BOOL, [float(op), float(a.type), float(len(a.params))] + [float(v) for v in a.params]
                 + [float(c.type), float(len(c.params))] + [float(v) for v in c.params]
                 + [float(v) for v in R.reshape(9)] + [float(v) for v in np.asarray(t, dtype=np.float64)])


def bool_parts(s: Solid):
    """(op, A, C, R, t) of a composite."""
    q = s.params
    op, at = int(q[0]), 1
    parts = []
    for _ in range(2):
        typ, n = int(q[at]), int(q[at + 1])
        parts.append(Solid(typ, list(q[at + 2:at + 2 + n])))
        at += 2 + n
    R = np.asarray(q[at:at + 9], dtype=np.float64).reshape(3, 3)
    t = np.asarray(q[at + 9:at + 12], dtype=np.float64)
    return op, parts[0], parts[1], R, t


def pcon_arrays(s: Solid):
    nz = int(s.params[0])
    a = np.asarray(s.params[1:], dtype=np.float64)
    return a[:nz], a[nz:2 * nz], a[2 * nz:3 * nz]


# The six configuration solids.  Box and tube segment are the paper's speed-test
# bodies; cone, sphere shell, trapezoid and polycone complete the basic set.
def polycone_radii() -> np.ndarray:
    """rmax of the 10-plane polycone, uniform in [5, 50] mm, drawn from the
    full-solid-set configuration's seed stream (first spawned child)."""
    ss = np.random.SeedSequence(SEED_BASE + 2)
    rng = np.random.Generator(np.random.PCG64(ss.spawn(1)[0]))
    return rng.uniform(5.0, 50.0, size=10)


def config_solids(hollow_pcon: bool = False) -> dict:
    zs = -90.0 + 20.0 * np.arange(10)
    rmax = polycone_radii()
    rmin = 0.3 * rmax if hollow_pcon else np.zeros(10)
    return {
        "box": box(10.0, 20.0, 30.0),
        "tubs": tubs(5.0, 15.0, 20.0, 0.0, 1.5 * math.pi),
        "cons": cons(2.0, 8.0, 4.0, 12.0, 25.0),
        "sphere": sphere(10.0, 30.0),
        "trd": trd(10.0, 20.0, 15.0, 25.0, 30.0),
        "pcon": pcon(zs, rmin, rmax),
    }


def solid_extent(s: Solid):
    """Axis-aligned bounding box (centre, half-lengths) of a solid's local frame."""
    p = s.params
    if s.type == BOX:
        return np.zeros(3), np.array(p[:3])
    if s.type == TUBS:
        return np.zeros(3), np.array([p[1], p[1], p[2]])
    if s.type == CONS:
        r = max(p[1], p[3])
        return np.zeros(3), np.array([r, r, p[4]])
    if s.type == SPHERE:
        return np.zeros(3), np.array([p[1]] * 3)
    if s.type == TRD:
        return np.zeros(3), np.array([max(p[0], p[1]), max(p[2], p[3]), p[4]])
    if s.type == PCON:
        z, _, rmax = pcon_arrays(s)
        r = float(rmax.max())
        return np.array([0.0, 0.0, 0.5 * (z[0] + z[-1])]), np.array([r, r, 0.5 * (z[-1] - z[0])])
    if s.type == BOOL:
        op, a, c, R, t = bool_parts(s)
        ca, ha = solid_extent(a)
        cc, hc = solid_extent(c)
        cc = R @ cc + t
        hc = np.abs(R) @ hc
        lo_a, hi_a, lo_c, hi_c = ca - ha, ca + ha, cc - hc, cc + hc
        if op == UNION:
            lo, hi = np.minimum(lo_a, lo_c), np.maximum(hi_a, hi_c)
        elif op == INTERSECTION and np.all(np.maximum(lo_a, lo_c) < np.minimum(hi_a, hi_c)):
            lo, hi = np.maximum(lo_a, lo_c), np.minimum(hi_a, hi_c)
        else:
            lo, hi = lo_a, hi_a
        return 0.5 * (lo + hi), 0.5 * (hi - lo)
    raise ValueError(s.type)


# --------------------------------------------------------------------------- geometry
@dataclass
class LV:
    solid: Solid
    placements: list = field(default_factory=list)  # (child_lv, R[3x3], t[3])
    name: str = ""


def rot_z(phi: float) -> np.ndarray:
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def make_blob(lvs: list, world_lv: int = 0) -> bytes:
    params, lv_rows, pl_rows = [], [], []
    for lv in lvs:
        off = len(params)
        params.extend(float(v) for v in lv.solid.params)
        lv_rows.append((lv.solid.type, off, len(lv.solid.params), len(pl_rows), len(lv.placements)))
        for child, R, t in lv.placements:
            pl_rows.append((child, np.asarray(R, dtype=np.float64).reshape(9), np.asarray(t, dtype=np.float64)))
    out = bytearray()
    out += MAGIC
    out += struct.pack("<6I", VERSION, len(lvs), len(pl_rows), len(params), world_lv, 0)
    for typ, off, cnt, poff, pcnt in lv_rows:
        out += struct.pack("<8i", typ, off, cnt, poff, pcnt, 0, 0, 0)
    for child, R, t in pl_rows:
        out += struct.pack("<2i", child, 0)
        out += R.astype("<f8").tobytes() + t.astype("<f8").tobytes()
    out += np.asarray(params, dtype="<f8").tobytes()
    return bytes(out)


def single_solid_blob(s: Solid) -> bytes:
    return make_blob([LV(s, [], s.name)])


def multi_solid_blob(solids: list) -> bytes:
    """One LV per solid, no placements (LV i = solids[i]); used by solid-level queries."""
    return make_blob([LV(s, [], s.name) for s in solids])


# Layered detector: world box 4 x 4 x 6 m, 20 concentric full tube layers between
# r = 50 and ~1942.5 mm, each holding 64 box modules rotated about z.
N_LAYERS = 20
N_MODULES = 64
WORLD_HALF = (2000.0, 2000.0, 3000.0)


def layer_rmin(i: int) -> float:
    return 50.0 + 97.5 * i


def detector_description():
    """Returns (lvs, info) for the layered detector.  LV 0 world; LV 1+2i layer i;
    LV 2+2i the module box of layer i."""
    lvs = [LV(box(*WORLD_HALF), [], "world")]
    info = {"layers": []}
    for i in range(N_LAYERS):
        rmin = layer_rmin(i)
        rmax = rmin + 40.0
        rc = rmin + 20.0
        hy = 0.8 * (rc - 15.0) * math.tan(math.pi / N_MODULES)
        layer_lv = len(lvs)
        module_lv = layer_lv + 1
        lvs.append(LV(tubs(rmin, rmax, 2500.0), [], f"layer{i}"))
        lvs.append(LV(box(15.0, hy, 2450.0), [], f"module{i}"))
        for k in range(N_MODULES):
            phi = TWO_PI * k / N_MODULES
            R = rot_z(phi)
            t = np.array([rc * math.cos(phi), rc * math.sin(phi), 0.0])
            lvs[layer_lv].placements.append((module_lv, R, t))
        lvs[0].placements.append((layer_lv, np.eye(3), np.zeros(3)))
        info["layers"].append({"rmin": rmin, "rmax": rmax, "rc": rc, "hy": hy})
    return lvs, info


def detector_materials() -> dict:
    """Synthetic materials of the layered detector for physics-limited steps:
    number density n and cross sections sigma of three processes per material,
    so that the mean free paths 1 / (n sigma) are 2e5, 5e5, 1e6 mm in the world,
    5e3, 2e4, 1e5 mm in the layers and 60, 150, 400 mm in the modules."""
    density = np.array([1.0, 1.0, 8.0])
    sigma = np.array([[5e-6, 2e-6, 1e-6],
                      [2e-4, 5e-5, 1e-5],
                      [1.0 / 480.0, 1.0 / 1200.0, 1.0 / 3200.0]])
    lv_mat = np.array([0] + [1, 2] * N_LAYERS, np.int32)  # world, then (layer, module) per layer
    return {"density": density, "sigma": sigma, "lv_mat": lv_mat}


PHYS_SEED = SEED_BASE + 6  # key of the physics draws of the detector workload


def detector_blob() -> bytes:
    return make_blob(detector_description()[0])


def _rot(axis, ang):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + math.sin(ang) * K + (1.0 - math.cos(ang)) * K @ K


def composite_solids() -> dict:
    """Eight composites: the three operations, every elementary part type,
    rotated and translated placements, touching parts (two cubes sharing a
    face) and a part that cuts through (a bore)."""
    return {
        "box_u_box": boolean(UNION, box(10, 10, 10), box(10, 10, 10), t=(20, 0, 0)),
        "box_minus_hole": boolean(SUBTRACTION, box(20, 20, 20), tubs(0, 5, 30)),
        "sphere_n_cube": boolean(INTERSECTION, sphere(0, 12), box(10, 10, 10)),
        "cube_n_rot_cube": boolean(INTERSECTION, box(10, 10, 10), box(10, 10, 10), R=rot_z(math.pi / 4)),
        "tubs_u_rot_box": boolean(UNION, tubs(5, 15, 20, 0.3, 1.2 * math.pi), box(4, 9, 25),
                                  R=_rot((1, 2, 3), 0.7), t=(8, -3, 2)),
        "pcon_minus_cons": boolean(SUBTRACTION, config_solids()["pcon"], cons(0, 6, 0, 14, 30),
                                   R=_rot((0, 1, 0), 0.4), t=(3, 0, -20)),
        "trd_n_sphere": boolean(INTERSECTION, trd(10, 20, 15, 25, 30), sphere(8, 28), t=(2, -3, 5)),
        "sphere_u_trd": boolean(UNION, sphere(10, 30), trd(5, 12, 6, 14, 20), R=_rot((1, 0, 1), 1.1), t=(25, 5, 0)),
    }


def composite_box_tracks(s: Solid, n: int, seed: int) -> Tracks:
    """Points uniform in the box 1.6 times a solid's bounding box, isotropic."""
    rng = np.random.default_rng(seed)
    c, h = solid_extent(s)
    P = uniform_box_points(rng, n, c, 1.6 * h)
    return Tracks(*P, *isotropic(rng, n))


# Composite-solid setup: a 600 mm world cube holding five volumes, four of them
# composites (one with daughters of its own), the fifth an elementary tube.
def composite_description():
    """LV 0 world; LV 1 a 120 mm cube with a radius-20 bore along z holding four
    small boxes in its wall; LV 2 a sphere shell united with a tilted Trd; LV 3
    a sphere clipped by a cube; LV 4 a tube segment (elementary); LV 5 a
    polycone with a tilted cone cut out; LV 6 the small box."""
    lvs = [LV(box(300.0, 300.0, 300.0), [], "world")]
    lvs.append(LV(boolean(SUBTRACTION, box(60.0, 60.0, 60.0), tubs(0.0, 20.0, 80.0)), [], "bored_cube"))
    lvs.append(LV(boolean(UNION, sphere(10.0, 40.0), trd(8.0, 16.0, 9.0, 20.0, 30.0), R=_rot((1, 0, 1), 1.1),
                          t=(35.0, 5.0, 0.0)), [], "shell_and_trd"))
    lvs.append(LV(boolean(INTERSECTION, sphere(0.0, 55.0), box(45.0, 45.0, 45.0)), [], "clipped_sphere"))
    lvs.append(LV(tubs(10.0, 50.0, 60.0, 0.3, 1.4 * math.pi), [], "tube_segment"))
    z = -90.0 + 20.0 * np.arange(10)
    lvs.append(LV(boolean(SUBTRACTION, pcon(z, np.zeros(10), polycone_radii() + 15.0), cons(0.0, 6.0, 0.0, 14.0, 30.0),
                          R=_rot((0, 1, 0), 0.4), t=(3.0, 0.0, -20.0)), [], "cut_polycone"))
    lvs.append(LV(box(5.0, 5.0, 5.0), [], "insert"))
    for sx, sy in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        lvs[1].placements.append((6, rot_z(0.3 * sx), np.array([40.0 * sx, 40.0 * sy, 10.0 * sy])))
    lvs[0].placements += [(1, _rot((0, 0, 1), 0.2), np.array([-170.0, 0.0, 0.0])),
                          (2, _rot((1, 1, 0), 0.6), np.array([160.0, 20.0, 0.0])),
                          (3, np.eye(3), np.array([0.0, 170.0, 60.0])),
                          (4, _rot((1, 0, 0), 0.5), np.array([0.0, -160.0, 0.0])),
                          (5, np.eye(3), np.array([0.0, 0.0, -150.0]))]
    return lvs


def composite_blob() -> bytes:
    return make_blob(composite_description())


COMPOSITE_CENTRES = np.array([[-170.0, 0.0, 0.0], [160.0, 20.0, 0.0], [0.0, 170.0, 60.0], [0.0, -160.0, 0.0],
                              [0.0, 0.0, -150.0]])


def composite_tracks(n: int) -> Tracks:
    """Each start is uniform in the 160 mm cube around one of the five placed
    volumes (chosen uniformly), directions isotropic."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7))
    c = COMPOSITE_CENTRES[rng.integers(0, len(COMPOSITE_CENTRES), n)].T
    p = c + rng.uniform(-80.0, 80.0, (3, n))
    return Tracks(p[0].copy(), p[1].copy(), p[2].copy(), *isotropic(rng, n))


# Index-structure setups.  Nested tubes: a world cube holding 10 identity-
# placed full tubes with disjoint radial ranges (the innermost a solid
# cylinder) and unequal lengths, placed out of radial order.  Ring: a world
# cube holding a box that holds 16 small boxes on a ring of radius 60 mm around
# the z axis, turned to face the axis.
def nested_tubes_description():
    lvs = [LV(box(400.0, 400.0, 400.0), [], "world")]
    order = [3, 0, 7, 1, 9, 4, 2, 8, 5, 6]
    for i in order:
        rmin = 0.0 if i == 0 else 20.0 + 30.0 * i
        rmax = rmin + 18.0 if i else 12.0
        dz = 150.0 + 20.0 * ((i * 7) % 5)
        lvs[0].placements.append((len(lvs), np.eye(3), np.zeros(3)))
        lvs.append(LV(tubs(rmin, rmax, dz), [], f"tube{i}"))
    return lvs


def ring_description():
    lvs = [LV(box(200.0, 200.0, 200.0), [], "world"), LV(box(100.0, 100.0, 50.0), [], "holder"),
           LV(box(6.0, 9.0, 40.0), [], "block")]
    lvs[0].placements.append((1, np.eye(3), np.array([0.0, 0.0, 10.0])))
    for k in range(16):
        phi = TWO_PI * k / 16 + 0.1
        lvs[1].placements.append((2, rot_z(phi), np.array([60.0 * math.cos(phi), 60.0 * math.sin(phi), 0.0])))
    return lvs


def grid_description():
    """A world cube holding a box that holds a 5 x 5 grid of boxes in the xy
    plane, centred on the z axis (no phi index: the middle one surrounds the
    axis), so the culled loop with group boxes runs."""
    lvs = [LV(box(200.0, 200.0, 200.0), [], "world"), LV(box(120.0, 120.0, 60.0), [], "holder"),
           LV(box(12.0, 9.0, 40.0), [], "cell")]
    lvs[0].placements.append((1, np.eye(3), np.zeros(3)))
    for i in range(5):
        for j in range(5):
            lvs[1].placements.append((2, rot_z(0.2 * (i - j)), np.array([40.0 * (i - 2), 40.0 * (j - 2), 4.0 * (i - j)])))
    return lvs


def big_grid_description():
    """A 9 x 9 grid of boxes in a box mother, through the z axis: 81 box
    daughters, so the culled loop runs over two chunks of 64 daughters (with
    group boxes) and the box a track has just left can sit in either."""
    lvs = [LV(box(200.0, 200.0, 200.0), [], "world"), LV(box(110.0, 110.0, 60.0), [], "holder"),
           LV(box(8.0, 6.0, 40.0), [], "cell")]
    lvs[0].placements.append((1, np.eye(3), np.zeros(3)))
    for i in range(9):
        for j in range(9):
            lvs[1].placements.append((2, rot_z(0.15 * (i - j) / 4.0),
                                      np.array([22.0 * (i - 4), 22.0 * (j - 4), 4.0 * (i - j) / 2.0])))
    return lvs


def bundle_description():
    """A world cube holding a box that holds 12 tilted tubes in two planes of
    3 x 2, two of them on the z axis (no phi index: the culled loop runs over
    tube daughters)."""
    lvs = [LV(box(200.0, 200.0, 200.0), [], "world"), LV(box(120.0, 120.0, 90.0), [], "holder"),
           LV(tubs(4.0, 14.0, 30.0), [], "pipe")]
    lvs[0].placements.append((1, np.eye(3), np.zeros(3)))
    k = 0
    for z in (-45.0, 45.0):
        for x in (-70.0, 0.0, 70.0):
            for y in (-75.0, 0.0):
                axis = (math.cos(1.3 * k), math.sin(1.3 * k), 0.4)
                lvs[1].placements.append((2, _rot(axis, 0.3 + 0.02 * k), np.array([x, y, z])))
                k += 1
    return lvs


# Constructed exact ties of ComputeStep (the paper fixes no tie-break; the
# readings are: among daughters entered at the same distance the lowest
# placement index wins, and a daughter entered exactly where the mother is
# left wins over the exit).  Each case: (LV list, start point, unit direction,
# index of the daughter that must be entered, step length).  Overlapping or
# protruding daughters are what makes a tie exact; the arithmetic of every
# case is exact in FP64 (axis-aligned slabs at integer coordinates, or two
# daughters with identical placements and parameters).
def tie_cases() -> dict:
    cases = {}
    a, b = box(10.0, 10.0, 10.0), box(5.0, 20.0, 20.0)  # entered at x = 40 from the origin
    e = np.eye(3)
    ray = (np.array([0.0, 3.0, -2.0]), np.array([1.0, 0.0, 0.0]))
    # two daughters entered at the same distance: plain loop (2 daughters)
    lvs = [LV(box(100.0, 100.0, 100.0), [(1, e, [50.0, 0.0, 0.0]), (2, e, [45.0, 0.0, 0.0])]), LV(a), LV(b)]
    cases["daughters_plain"] = (lvs, *ray, 0, 40.0)
    lvs = [LV(box(100.0, 100.0, 100.0), [(2, e, [45.0, 0.0, 0.0]), (1, e, [50.0, 0.0, 0.0])]), LV(a), LV(b)]
    cases["daughters_plain_swapped"] = (lvs, *ray, 0, 40.0)
    # the same among 10 box daughters (culled loop with its box screen and
    # SafetyToIn bound): the tied pair at indices 3 and 7
    small = box(2.0, 2.0, 2.0)
    pl = [(3, e, np.array([-80.0 + 18.0 * k, -80.0, 0.0])) for k in range(10)]
    pl[3] = (1, e, np.array([50.0, 0.0, 0.0]))
    pl[7] = (2, e, np.array([45.0, 0.0, 0.0]))
    lvs = [LV(box(100.0, 100.0, 100.0), pl), LV(box(10.0, 10.0, 10.0)), LV(box(10.0, 10.0, 10.0)), LV(small)]
    # both tied daughters are the same size here: b's slab also starts at 40
    lvs[2] = LV(box(5.0, 10.0, 10.0))
    cases["daughters_culled"] = (lvs, *ray, 3, 40.0)
    # phi sectors: 8 boxes on a ring around the z axis inside a holder, the
    # box at index 2 placed again at index 6 (identical placement); the ray
    # runs radially towards it, off the axis by 3 mm
    ring = []
    for k in range(8):
        phi = TWO_PI * k / 8 + 0.1
        ring.append((2, rot_z(phi), np.array([60.0 * math.cos(phi), 60.0 * math.sin(phi), 0.0])))
    ring[6] = ring[2]
    lvs = [LV(box(200.0, 200.0, 200.0), [(1, e, np.zeros(3))]), LV(box(100.0, 100.0, 50.0), ring),
           LV(box(6.0, 9.0, 40.0))]
    phi2 = TWO_PI * 2 / 8 + 0.1
    u = np.array([math.cos(phi2), math.sin(phi2), 0.0])
    v = np.array([-math.sin(phi2), math.cos(phi2), 0.0])
    cases["daughters_phi"] = (lvs, 20.0 * u + 3.0 * v, u, 2, None)
    # a daughter entered exactly where the mother is left (it protrudes
    # through the mother's face x = 100): the daughter wins
    lvs = [LV(box(100.0, 100.0, 100.0), [(1, e, [110.0, 0.0, 0.0])]), LV(a)]
    cases["exit_plain"] = (lvs, *ray, 0, 100.0)
    pl = [(2, e, np.array([-80.0 + 18.0 * k, -80.0, 0.0])) for k in range(10)]
    pl[5] = (1, e, np.array([110.0, 0.0, 0.0]))
    lvs = [LV(box(100.0, 100.0, 100.0), pl), LV(a), LV(small)]
    cases["exit_culled"] = (lvs, *ray, 5, 100.0)
    return cases


def tie_tracks(case, n: int = 1) -> Tracks:
    """n copies of a tie case's ray."""
    _, p, d, _, _ = case
    return Tracks(*[np.full(n, float(v)) for v in (*p, *d)])


def uniform_world_tracks(half, n: int, seed: int, centre=(0.0, 0.0, 0.0)) -> Tracks:
    """Starts uniform in the box centre +- half (mm), isotropic directions; one
    track in eight is parallel to the z axis."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = uniform_box_points(rng, n, np.asarray(centre, dtype=np.float64), np.broadcast_to(np.asarray(half, dtype=np.float64), (3,)))
    dx, dy, dz = isotropic(rng, n)
    par = np.arange(n) % 8 == 3
    dx[par], dy[par], dz[par] = 0.0, 0.0, np.where(rng.random(int(par.sum())) < 0.5, 1.0, -1.0)
    return Tracks(p[0].copy(), p[1].copy(), p[2].copy(), dx, dy, dz)


def expand_pvs(lvs: list, world_lv: int = 0):
    """DFS pre-order expansion: list of (lv, parent_pv, R_global, t_global, depth).
    Global transforms are composed here only for test brute force and generators."""
    out = []

    def rec(lv, parent, Rg, tg, depth):
        me = len(out)
        out.append((lv, parent, Rg, tg, depth))
        for child, R, t in lvs[lv].placements:
            rec(child, me, Rg @ np.asarray(R), Rg @ np.asarray(t) + tg, depth + 1)

    rec(world_lv, -1, np.eye(3), np.zeros(3), 0)
    return out


# --------------------------------------------------------------------------- tracks
@dataclass
class Tracks:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    dx: np.ndarray
    dy: np.ndarray
    dz: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return [self.x, self.y, self.z, self.dx, self.dy, self.dz]

    def take(self, idx) -> "Tracks":
        return Tracks(*[np.ascontiguousarray(a[idx]) for a in self.arrays()])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in self.arrays():
            h.update(np.ascontiguousarray(a, dtype="<f8").tobytes())
        return h.hexdigest()


def rng_for(config: int, stream: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence(SEED_BASE + config)
    return np.random.Generator(np.random.PCG64(ss.spawn(stream + 2)[stream + 1]))


def isotropic(rng: np.random.Generator, n: int):
    """cos(theta) ~ U(-1,1), phi ~ U(0,2pi), renormalised in FP64."""
    ct = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, TWO_PI, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct])
    d /= np.sqrt((d * d).sum(axis=0))
    return d[0].copy(), d[1].copy(), d[2].copy()


def uniform_box_points(rng, n, centre, half):
    p = rng.uniform(-1.0, 1.0, (3, n)) * np.asarray(half)[:, None] + np.asarray(centre)[:, None]
    return p


CONFIG1_SOLIDS = ("box", "tubs")


def config1_tracks(name: str, n: int = 65536) -> Tracks:
    """Positions uniform in a box twice the solid's extent, isotropic directions."""
    s = config_solids()[name]
    rng = rng_for(1, CONFIG1_SOLIDS.index(name))
    c, h = solid_extent(s)
    p = uniform_box_points(rng, n, c, 2.0 * h)
    dx, dy, dz = isotropic(rng, n)
    return Tracks(p[0].copy(), p[1].copy(), p[2].copy(), dx, dy, dz)


def config1_inside_points(name: str, n: int) -> Tracks:
    """Paper-protocol sweep: points inside the body (drawn by parametric sampling)."""
    s = config_solids()[name]
    rng = rng_for(1, 10 + CONFIG1_SOLIDS.index(name))
    p = sample_volume(s, rng, n)
    dx, dy, dz = isotropic(rng, n)
    return Tracks(p[0].copy(), p[1].copy(), p[2].copy(), dx, dy, dz)


CONFIG2_SOLIDS = ("box", "tubs", "cons", "sphere", "trd", "pcon")


def config2_tracks(name: str, n: int = 1 << 20, hollow_pcon: bool = False) -> Tracks:
    """floor(n/3) inside, floor(n/3) outside, the rest within 1e-6 mm of the surface
    (area-uniform surface point moved along its outward normal by U(-1e-6, 1e-6)),
    shuffled; isotropic directions."""
    s = config_solids(hollow_pcon)[name]
    rng = rng_for(2, 1 + CONFIG2_SOLIDS.index(name))
    n_in = n // 3
    n_out = n // 3
    n_surf = n - n_in - n_out
    pin = sample_volume(s, rng, n_in)
    pout = sample_outside(s, rng, n_out)
    psurf, nrm = sample_surface(s, rng, n_surf)
    psurf = psurf + nrm * rng.uniform(-1e-6, 1e-6, n_surf)[None, :]
    p = np.concatenate([pin, pout, psurf], axis=1)
    perm = rng.permutation(n)
    p = p[:, perm]
    dx, dy, dz = isotropic(rng, n)
    return Tracks(p[0].copy(), p[1].copy(), p[2].copy(), dx, dy, dz)


def config3_tracks(n: int = 1 << 20) -> Tracks:
    """Starts uniform in the cube [-1, 1]^3 mm around the origin, isotropic directions."""
    rng = rng_for(3, 0)
    p = rng.uniform(-1.0, 1.0, (3, n))
    dx, dy, dz = isotropic(rng, n)
    return Tracks(p[0].copy(), p[1].copy(), p[2].copy(), dx, dy, dz)


# --------------------------------------------------------------------------- sampling
# Parametric samplers: they draw points by construction from the solid's
# parameter domain.  `_member` is a zero-tolerance membership predicate used only
# to reject the outside third of the full-solid-set workload; it decides which
# points are drawn, never any expected value.

def _phi_range(sphi, dphi):
    return sphi, min(dphi, TWO_PI)


def _sample_z_linear_density(rng, n, z0, z1, f0, f1):
    """z in [z0, z1] with density proportional to the linear function f (f0 at z0, f1 at z1)."""
    u = rng.uniform(0.0, 1.0, n)
    if abs(f1 - f0) < 1e-14 * max(abs(f0), abs(f1), 1.0):
        return z0 + u * (z1 - z0)
    # invert the CDF of a linear density
    a = f0
    b = f1 - f0
    # F(s) = (a s + b s^2 / 2) / (a + b/2), s in [0,1]
    tot = a + 0.5 * b
    s = (-a + np.sqrt(a * a + 2.0 * b * tot * u)) / b
    return z0 + s * (z1 - z0)


def _sample_z_quadratic_density(rng, n, z0, z1, dens):
    """Rejection sampling of z in [z0,z1] with density dens(z) >= 0 (vectorised)."""
    zz = np.linspace(z0, z1, 257)
    dmax = float(np.max(dens(zz))) * 1.0001 + 1e-300
    out = np.empty(0)
    while out.size < n:
        m = max(2 * (n - out.size), 1024)
        z = rng.uniform(z0, z1, m)
        keep = rng.uniform(0.0, dmax, m) < dens(z)
        out = np.concatenate([out, z[keep]])
    return out[:n]


def sample_volume(s: Solid, rng, n: int) -> np.ndarray:
    p = s.params
    if s.type == BOOL:  # rejection from the bounding box
        c, h = solid_extent(s)
        out = np.empty((3, 0))
        while out.shape[1] < n:
            P = uniform_box_points(rng, 4 * (n - out.shape[1]) + 1024, c, h)
            out = np.concatenate([out, P[:, _member(s, P)]], axis=1)
        return out[:, :n]
    if s.type == BOX:
        return rng.uniform(-1, 1, (3, n)) * np.array(p[:3])[:, None]
    if s.type in (TUBS, CONS):
        if s.type == TUBS:
            rmin1 = rmin2 = p[0]
            rmax1 = rmax2 = p[1]
            dz, sphi, dphi = p[2], p[3], p[4]
        else:
            rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi = p
        Ri = lambda z: rmin1 + (rmin2 - rmin1) * (z + dz) / (2 * dz)
        Ro = lambda z: rmax1 + (rmax2 - rmax1) * (z + dz) / (2 * dz)
        z = _sample_z_quadratic_density(rng, n, -dz, dz, lambda z: Ro(z) ** 2 - Ri(z) ** 2)
        r = np.sqrt(rng.uniform(Ri(z) ** 2, Ro(z) ** 2))
        s0, dp = _phi_range(sphi, dphi)
        ph = s0 + rng.uniform(0, 1, n) * dp
        return np.stack([r * np.cos(ph), r * np.sin(ph), z])
    if s.type == SPHERE:
        rmin, rmax = p
        rho = np.cbrt(rng.uniform(rmin ** 3, rmax ** 3, n))
        u = np.stack(isotropic(rng, n))
        return u * rho[None, :]
    if s.type == TRD:
        dx1, dx2, dy1, dy2, dz = p
        X = lambda z: dx1 + (dx2 - dx1) * (z + dz) / (2 * dz)
        Y = lambda z: dy1 + (dy2 - dy1) * (z + dz) / (2 * dz)
        z = _sample_z_quadratic_density(rng, n, -dz, dz, lambda z: X(z) * Y(z))
        x = rng.uniform(-1, 1, n) * X(z)
        y = rng.uniform(-1, 1, n) * Y(z)
        return np.stack([x, y, z])
    if s.type == PCON:
        zs, rmin, rmax = pcon_arrays(s)
        h = np.diff(zs)
        vol = np.pi * h / 3.0 * (rmax[:-1] ** 2 + rmax[:-1] * rmax[1:] + rmax[1:] ** 2
                                 - rmin[:-1] ** 2 - rmin[:-1] * rmin[1:] - rmin[1:] ** 2)
        sec = rng.choice(len(h), size=n, p=vol / vol.sum())
        out = np.empty((3, n))
        for j in range(len(h)):
            m = sec == j
            k = int(m.sum())
            if k == 0:
                continue
            Ri = lambda z, j=j: rmin[j] + (rmin[j + 1] - rmin[j]) * (z - zs[j]) / h[j]
            Ro = lambda z, j=j: rmax[j] + (rmax[j + 1] - rmax[j]) * (z - zs[j]) / h[j]
            z = _sample_z_quadratic_density(rng, k, zs[j], zs[j + 1], lambda z: Ro(z) ** 2 - Ri(z) ** 2)
            r = np.sqrt(rng.uniform(Ri(z) ** 2, Ro(z) ** 2))
            ph = rng.uniform(0, TWO_PI, k)
            out[:, m] = np.stack([r * np.cos(ph), r * np.sin(ph), z])
        return out
    raise ValueError(s.type)


def _member(s: Solid, P: np.ndarray) -> np.ndarray:
    x, y, z = P
    p = s.params
    if s.type == BOX:
        return (np.abs(x) <= p[0]) & (np.abs(y) <= p[1]) & (np.abs(z) <= p[2])
    if s.type in (TUBS, CONS):
        if s.type == TUBS:
            rmin1 = rmin2 = p[0]
            rmax1 = rmax2 = p[1]
            dz, sphi, dphi = p[2], p[3], p[4]
        else:
            rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi = p
        r = np.hypot(x, y)
        f = (z + dz) / (2 * dz)
        ok = (np.abs(z) <= dz) & (r <= rmax1 + (rmax2 - rmax1) * f) & (r >= rmin1 + (rmin2 - rmin1) * f)
        if dphi < TWO_PI:
            ph = np.mod(np.arctan2(y, x) - sphi, TWO_PI)
            ok &= ph <= dphi
        return ok
    if s.type == SPHERE:
        rho = np.sqrt(x * x + y * y + z * z)
        return (rho >= p[0]) & (rho <= p[1])
    if s.type == TRD:
        dx1, dx2, dy1, dy2, dz = p
        f = (z + dz) / (2 * dz)
        return (np.abs(z) <= dz) & (np.abs(x) <= dx1 + (dx2 - dx1) * f) & (np.abs(y) <= dy1 + (dy2 - dy1) * f)
    if s.type == PCON:
        zs, rmin, rmax = pcon_arrays(s)
        r = np.hypot(x, y)
        ok = (z >= zs[0]) & (z <= zs[-1])
        ro = np.interp(z, zs, rmax)
        ri = np.interp(z, zs, rmin)
        return ok & (r <= ro) & (r >= ri)
    if s.type == BOOL:
        op, a, c, R, t = bool_parts(s)
        ma, mc = _member(a, P), _member(c, R.T @ (P - t[:, None]))
        return (ma | mc) if op == UNION else ((ma & ~mc) if op == SUBTRACTION else (ma & mc))
    raise ValueError(s.type)


def sample_outside(s: Solid, rng, n: int) -> np.ndarray:
    c, h = solid_extent(s)
    out = np.empty((3, 0))
    while out.shape[1] < n:
        m = 2 * (n - out.shape[1]) + 1024
        P = uniform_box_points(rng, m, c, 2.0 * h)
        out = np.concatenate([out, P[:, ~_member(s, P)]], axis=1)
    return out[:, :n]


def _faces(s: Solid):
    """List of (area, sampler(rng, k) -> (P[3,k], N[3,k])) for every boundary face."""
    p = s.params
    faces = []
    if s.type == BOX:
        h = np.array(p[:3])
        for ax in range(3):
            o1, o2 = [a for a in range(3) if a != ax]
            for sg in (-1.0, 1.0):
                def smp(rng, k, ax=ax, o1=o1, o2=o2, sg=sg):
                    P = np.empty((3, k))
                    P[ax] = sg * h[ax]
                    P[o1] = rng.uniform(-h[o1], h[o1], k)
                    P[o2] = rng.uniform(-h[o2], h[o2], k)
                    N = np.zeros((3, k))
                    N[ax] = sg
                    return P, N
                faces.append((4.0 * h[o1] * h[o2], smp))
        return faces
    if s.type in (TUBS, CONS):
        if s.type == TUBS:
            rmin1 = rmin2 = p[0]
            rmax1 = rmax2 = p[1]
            dz, sphi, dphi = p[2], p[3], p[4]
        else:
            rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi = p
        s0, dp = _phi_range(sphi, dphi)
        for (r1, r2, sg) in ((rmax1, rmax2, 1.0), (rmin1, rmin2, -1.0)):
            if r1 == 0.0 and r2 == 0.0:
                continue
            b = (r2 - r1) / (2 * dz)
            slant = math.sqrt(1.0 + b * b)
            area = dp * 0.5 * (r1 + r2) * 2 * dz * slant

            def smp(rng, k, r1=r1, r2=r2, sg=sg, b=b, slant=slant):
                z = _sample_z_linear_density(rng, k, -dz, dz, r1, r2)
                R = r1 + (r2 - r1) * (z + dz) / (2 * dz)
                ph = s0 + rng.uniform(0, 1, k) * dp
                P = np.stack([R * np.cos(ph), R * np.sin(ph), z])
                N = sg * np.stack([np.cos(ph), np.sin(ph), -b * np.ones(k)]) / slant
                return P, N
            faces.append((area, smp))
        for (zc, ri, ro, sg) in ((-dz, rmin1, rmax1, -1.0), (dz, rmin2, rmax2, 1.0)):
            area = 0.5 * dp * (ro * ro - ri * ri)
            if area <= 0.0:
                continue

            def smp(rng, k, zc=zc, ri=ri, ro=ro, sg=sg):
                r = np.sqrt(rng.uniform(ri * ri, ro * ro, k))
                ph = s0 + rng.uniform(0, 1, k) * dp
                P = np.stack([r * np.cos(ph), r * np.sin(ph), np.full(k, zc)])
                N = np.zeros((3, k))
                N[2] = sg
                return P, N
            faces.append((area, smp))
        if dphi < TWO_PI:
            pe = sphi + dphi
            for (ph0, nrm) in ((sphi, (math.sin(sphi), -math.cos(sphi))), (pe, (-math.sin(pe), math.cos(pe)))):
                area = 0.5 * ((rmax1 - rmin1) + (rmax2 - rmin2)) * 2 * dz

                def smp(rng, k, ph0=ph0, nrm=nrm):
                    z = _sample_z_linear_density(rng, k, -dz, dz, rmax1 - rmin1, rmax2 - rmin2)
                    f = (z + dz) / (2 * dz)
                    ri = rmin1 + (rmin2 - rmin1) * f
                    ro = rmax1 + (rmax2 - rmax1) * f
                    r = rng.uniform(ri, ro)
                    P = np.stack([r * math.cos(ph0), r * math.sin(ph0), z])
                    N = np.zeros((3, k))
                    N[0], N[1] = nrm
                    return P, N
                faces.append((area, smp))
        return faces
    if s.type == SPHERE:
        for (R, sg) in ((p[1], 1.0), (p[0], -1.0)):
            if R <= 0.0:
                continue

            def smp(rng, k, R=R, sg=sg):
                u = np.stack(isotropic(rng, k))
                return u * R, sg * u
            faces.append((4 * math.pi * R * R, smp))
        return faces
    if s.type == TRD:
        dx1, dx2, dy1, dy2, dz = p
        for (zc, hx, hy, sg) in ((-dz, dx1, dy1, -1.0), (dz, dx2, dy2, 1.0)):
            def smp(rng, k, zc=zc, hx=hx, hy=hy, sg=sg):
                P = np.stack([rng.uniform(-hx, hx, k), rng.uniform(-hy, hy, k), np.full(k, zc)])
                N = np.zeros((3, k))
                N[2] = sg
                return P, N
            faces.append((4 * hx * hy, smp))
        for ax, (a1, a2, o1, o2) in ((0, (dx1, dx2, dy1, dy2)), (1, (dy1, dy2, dx1, dx2))):
            t = (a2 - a1) / (2 * dz)
            slant = math.sqrt(1 + t * t)
            area = (o1 + o2) * 2 * dz * slant
            for sg in (-1.0, 1.0):
                def smp(rng, k, ax=ax, a1=a1, a2=a2, o1=o1, o2=o2, t=t, slant=slant, sg=sg):
                    z = _sample_z_linear_density(rng, k, -dz, dz, o1, o2)
                    f = (z + dz) / (2 * dz)
                    A = a1 + (a2 - a1) * f
                    O = o1 + (o2 - o1) * f
                    P = np.empty((3, k))
                    P[ax] = sg * A
                    P[1 - ax] = rng.uniform(-1, 1, k) * O
                    P[2] = z
                    N = np.zeros((3, k))
                    N[ax] = sg / slant
                    N[2] = -t / slant
                    return P, N
                faces.append((area, smp))
        return faces
    if s.type == PCON:
        zs, rmin, rmax = pcon_arrays(s)
        for j in range(len(zs) - 1):
            h = zs[j + 1] - zs[j]
            for (R, sg) in ((rmax, 1.0), (rmin, -1.0)):
                r1, r2 = R[j], R[j + 1]
                if r1 == 0.0 and r2 == 0.0:
                    continue
                b = (r2 - r1) / h
                slant = math.sqrt(1 + b * b)
                area = math.pi * (r1 + r2) * h * slant

                def smp(rng, k, j=j, r1=r1, r2=r2, b=b, slant=slant, sg=sg, h=h):
                    z = _sample_z_linear_density(rng, k, zs[j], zs[j + 1], r1, r2)
                    Rz = r1 + (r2 - r1) * (z - zs[j]) / h
                    ph = rng.uniform(0, TWO_PI, k)
                    P = np.stack([Rz * np.cos(ph), Rz * np.sin(ph), z])
                    N = sg * np.stack([np.cos(ph), np.sin(ph), -b * np.ones(k)]) / slant
                    return P, N
                faces.append((area, smp))
        for (zc, ri, ro, sg) in ((zs[0], rmin[0], rmax[0], -1.0), (zs[-1], rmin[-1], rmax[-1], 1.0)):
            def smp(rng, k, zc=zc, ri=ri, ro=ro, sg=sg):
                r = np.sqrt(rng.uniform(ri * ri, ro * ro, k))
                ph = rng.uniform(0, TWO_PI, k)
                P = np.stack([r * np.cos(ph), r * np.sin(ph), np.full(k, zc)])
                N = np.zeros((3, k))
                N[2] = sg
                return P, N
            faces.append((math.pi * (ro * ro - ri * ri), smp))
        return faces
    raise ValueError(s.type)


def _bool_surface(s: Solid, rng, n: int):
    """Points of the components' faces that lie on the composite's boundary
    (membership differs 1e-7 mm to either side), with outward normals."""
    op, a, c, R, t = bool_parts(s)
    P, N = np.empty((3, 0)), np.empty((3, 0))
    while P.shape[1] < n:
        m = 2 * (n - P.shape[1]) + 1024
        pa, na = sample_surface(a, rng, m)
        pc, nc = sample_surface(c, rng, m)
        Q = np.concatenate([pa, R @ pc + t[:, None]], axis=1)
        M = np.concatenate([na, R @ nc], axis=1)
        e = 1e-7
        inn, out = _member(s, Q - e * M), _member(s, Q + e * M)
        keep = inn != out
        M = np.where(inn, M, -M)
        P = np.concatenate([P, Q[:, keep]], axis=1)
        N = np.concatenate([N, M[:, keep]], axis=1)
    sel = rng.permutation(P.shape[1])[:n]
    return P[:, sel], N[:, sel]


def sample_surface(s: Solid, rng, n: int):
    if s.type == BOOL:
        return _bool_surface(s, rng, n)
    faces = _faces(s)
    areas = np.array([a for a, _ in faces])
    pick = rng.choice(len(faces), size=n, p=areas / areas.sum())
    P = np.empty((3, n))
    N = np.empty((3, n))
    for i, (_, smp) in enumerate(faces):
        m = pick == i
        k = int(m.sum())
        if k:
            P[:, m], N[:, m] = smp(rng, k)
    return P, N
