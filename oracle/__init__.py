"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 CPU implementation of the geometry queries and the step
selection of the paper (Sec. III.A, III.B, III.C), written independently of the
HIP library: the two share no code, headers, tables or helpers.  Only `tests/`,
`__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py` may import it;
the product path never does.

Functions pinned by the tests in tests/test_oracle_*.py.  Safety values away
from the cases where the chosen lower-bound formula equals the exact distance
are "parity unpinned" beyond the invariant 0 <= Safety <= true distance.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

OUTSIDE, SURFACE, INSIDE = 0, 1, 2
F_OVERFLOW, F_STUCK, F_LOCATE_FAIL = 1, 2, 4
D_NEAR_TIE, D_GRAZE, D_ZERO_STEP, D_BAND_EDGE, D_NO_EXIT = 16, 32, 64, 128, 256
D_COND = 512  # solid-level hit whose FP64 conditioning exceeds the 1e-12 bar (or_hit_cond)
# decisions two correct FP64 codes may take differently (the oracle's own pins
# exclude only these; D_COND hits still meet the closed forms there)
D_DECIDE = D_NEAR_TIE | D_GRAZE | D_ZERO_STEP | D_BAND_EDGE | D_NO_EXIT
D_ILL = D_DECIDE | D_COND

_P = C.c_void_p
_I64 = C.c_int64


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        sig = {
            "orc_solid_check": (C.c_int, [C.c_int, _P, C.c_int]),
            "orc_solid_signed": (C.c_int, [C.c_int, _P, C.c_int, _I64, _P, _P, _P, _P, C.c_int]),
            "orc_solid_inside": (C.c_int, [C.c_int, _P, C.c_int, _I64, _P, _P, _P, _P, C.c_int]),
            "orc_solid_safety": (C.c_int, [C.c_int, _P, C.c_int, C.c_int, _I64, _P, _P, _P, _P, C.c_int]),
            "orc_solid_distance": (C.c_int, [C.c_int, _P, C.c_int, C.c_int, _I64] + [_P] * 8 + [C.c_int]),
            "orc_solid_roots": (C.c_int, [C.c_int, _P, C.c_int, _P, _P, _P, C.c_int]),
            "orc_geom_load": (_P, [_P, _I64, C.POINTER(C.c_int)]),
            "orc_geom_free": (None, [_P]),
            "orc_geom_info": (C.c_int, [_P, _P]),
            "orc_geom_pv_table": (C.c_int, [_P, _P, _P, _P]),
            "orc_to_local": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P]),
            "orc_locate": (C.c_int, [_P, _I64, _P, _P, _P, _P, C.c_int]),
            "orc_step": (C.c_int, [_P, _I64] + [_P] * 12 + [C.c_int]),
            "orc_nav_safety": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, C.c_int]),
            "orc_nav_inside": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, C.c_int]),
            "orc_transport": (C.c_int, [_P, _I64] + [_P] * 7 + [C.c_int] + [_P] * 5 + [C.c_int]),
            "orc_max_threads": (C.c_int, []),
            "orc_philox": (None, [_P, _P, _P]),
            "orc_uniform": (C.c_double, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]),
            "orc_phys_length": (C.c_int, [C.c_int, C.c_int, _P, _P, _I64, _P, C.c_uint64, _P, _P, _P, _P]),
            "orc_transport_phys": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _I64] + [_P] * 7
                                   + [C.c_int, C.c_uint64] + [_P] * 7 + [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _params(solid):
    return _f64(np.asarray(solid.params, dtype=np.float64))


def solid_ok(solid) -> bool:
    p = _params(solid)
    return lib().orc_solid_check(solid.type, _ptr(p), p.size) == 0


def signed(solid, x, y, z, threads=None):
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = np.empty(x.shape[0], np.float64)
    p = _params(solid)
    rc = lib().orc_solid_signed(solid.type, _ptr(p), p.size, x.shape[0], _ptr(x), _ptr(y), _ptr(z),
                                _ptr(out), threads or default_threads())
    assert rc == 0
    return out


def inside(solid, x, y, z, threads=None):
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = np.empty(x.shape[0], np.int8)
    p = _params(solid)
    rc = lib().orc_solid_inside(solid.type, _ptr(p), p.size, x.shape[0], _ptr(x), _ptr(y), _ptr(z),
                                _ptr(out), threads or default_threads())
    assert rc == 0
    return out


def safety(solid, mode, x, y, z, threads=None):
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = np.empty(x.shape[0], np.float64)
    p = _params(solid)
    rc = lib().orc_solid_safety(solid.type, _ptr(p), p.size, mode, x.shape[0], _ptr(x), _ptr(y),
                                _ptr(z), _ptr(out), threads or default_threads())
    assert rc == 0
    return out


def distance(solid, direction, tracks, threads=None):
    """direction 0 = DistanceToIn, 1 = DistanceToOut; returns (dist, diag)."""
    a = [_f64(v) for v in tracks.arrays()]
    n = a[0].shape[0]
    out = np.empty(n, np.float64)
    diag = np.zeros(n, np.uint32)
    p = _params(solid)
    rc = lib().orc_solid_distance(solid.type, _ptr(p), p.size, direction, n, *[_ptr(v) for v in a],
                                  _ptr(out), _ptr(diag), threads or default_threads())
    assert rc == 0
    return out, diag


def roots(solid, p3, d3):
    p = _params(solid)
    pp, dd = _f64(p3), _f64(d3)
    buf = np.empty(512, np.float64)
    n = lib().orc_solid_roots(solid.type, _ptr(p), p.size, _ptr(pp), _ptr(dd), _ptr(buf), 512)
    return np.sort(buf[:n])


class Geometry:
    """Oracle-side placed-volume tree parsed from a geometry blob."""

    def __init__(self, blob: bytes):
        self._blob = bytes(blob)
        st = C.c_int(0)
        buf = C.create_string_buffer(self._blob, len(self._blob))
        self._h = lib().orc_geom_load(buf, len(self._blob), C.byref(st))
        if not self._h:
            raise ValueError(f"oracle: geometry blob rejected (status {st.value})")
        info = np.zeros(4, np.int32)
        lib().orc_geom_info(self._h, _ptr(info))
        self.n_lv, self.n_pv, self.max_depth, self.world_lv = (int(v) for v in info)

    def close(self):
        if self._h:
            lib().orc_geom_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pv_table(self):
        lv = np.empty(self.n_pv, np.int32)
        par = np.empty(self.n_pv, np.int32)
        dep = np.empty(self.n_pv, np.int32)
        lib().orc_geom_pv_table(self._h, _ptr(lv), _ptr(par), _ptr(dep))
        return lv, par, dep

    def to_local(self, x, y, z, pv):
        x, y, z = _f64(x), _f64(y), _f64(z)
        pv = np.ascontiguousarray(pv, np.int32)
        out = np.empty((x.shape[0], 3), np.float64)
        assert lib().orc_to_local(self._h, x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(pv), _ptr(out)) == 0
        return out

    def locate(self, x, y, z, threads=None):
        x, y, z = _f64(x), _f64(y), _f64(z)
        out = np.empty(x.shape[0], np.int32)
        lib().orc_locate(self._h, x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(out), threads or default_threads())
        return out

    def step(self, tracks, pv, pstep=None, threads=None):
        a = [_f64(v) for v in tracks.arrays()]
        n = a[0].shape[0]
        pv = np.ascontiguousarray(pv, np.int32)
        ps = None if pstep is None else _f64(pstep)
        st = np.empty(n, np.float64)
        nx = np.empty(n, np.int32)
        fl = np.zeros(n, np.uint32)
        dg = np.zeros(n, np.uint32)
        rc = lib().orc_step(self._h, n, *[_ptr(v) for v in a], _ptr(pv), _ptr(ps), _ptr(st), _ptr(nx),
                            _ptr(fl), _ptr(dg), threads or default_threads())
        assert rc == 0
        return st, nx, fl, dg

    def nav_safety(self, x, y, z, pv, threads=None):
        x, y, z = _f64(x), _f64(y), _f64(z)
        pv = np.ascontiguousarray(pv, np.int32)
        out = np.empty(x.shape[0], np.float64)
        assert lib().orc_nav_safety(self._h, x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(pv), _ptr(out),
                                    threads or default_threads()) == 0
        return out

    def nav_inside(self, x, y, z, pv, threads=None):
        x, y, z = _f64(x), _f64(y), _f64(z)
        pv = np.ascontiguousarray(pv, np.int32)
        out = np.empty(x.shape[0], np.int8)
        assert lib().orc_nav_inside(self._h, x.shape[0], _ptr(x), _ptr(y), _ptr(z), _ptr(pv), _ptr(out),
                                    threads or default_threads()) == 0
        return out

    def transport(self, tracks, start_pv=None, max_steps=128, threads=None):
        """Returns dict(pv[n, max_steps+1], step[n, max_steps], nsteps, flags, diag).
        Entries past a track's last step hold -2 / NaN."""
        a = [_f64(v) for v in tracks.arrays()]
        n = a[0].shape[0]
        sp = None if start_pv is None else np.ascontiguousarray(start_pv, np.int32)
        pv = np.full((n, max_steps + 1), -2, np.int32)
        stp = np.full((n, max_steps), np.nan, np.float64)
        ns = np.zeros(n, np.int32)
        fl = np.zeros(n, np.uint32)
        dg = np.zeros(n, np.uint32)
        rc = lib().orc_transport(self._h, n, *[_ptr(v) for v in a], _ptr(sp), max_steps, _ptr(pv), _ptr(stp),
                                 _ptr(ns), _ptr(fl), _ptr(dg), threads or default_threads())
        assert rc == 0
        return {"pv": pv, "step": stp, "nsteps": ns, "flags": fl, "diag": dg}

    def transport_phys(self, tracks, materials, seed, start_pv=None, max_steps=128, track_id=None, threads=None):
        """Physics-limited transport (materials: dict density[n_mat], sigma[n_mat][n_proc],
        lv_mat[n_lv]); adds proc[n, max_steps] (int8: process of a physics-limited
        step, -1 for a boundary step; -2 past the last step).  track_id: the
        counters of the tracks' draws (default 0 .. n-1)."""
        a = [_f64(v) for v in tracks.arrays()]
        n = a[0].shape[0]
        den = _f64(materials["density"])
        sig = np.ascontiguousarray(materials["sigma"], np.float64)
        lvm = np.ascontiguousarray(materials["lv_mat"], np.int32)
        sp = None if start_pv is None else np.ascontiguousarray(start_pv, np.int32)
        pv = np.full((n, max_steps + 1), -2, np.int32)
        stp = np.full((n, max_steps), np.nan, np.float64)
        pr = np.full((n, max_steps), -2, np.int8)
        ns = np.zeros(n, np.int32)
        fl = np.zeros(n, np.uint32)
        dg = np.zeros(n, np.uint32)
        tid = None if track_id is None else np.ascontiguousarray(track_id, np.uint32)
        rc = lib().orc_transport_phys(self._h, den.shape[0], sig.shape[1], _ptr(den), _ptr(sig), _ptr(lvm), n,
                                      *[_ptr(v) for v in a], _ptr(sp), max_steps, int(seed), _ptr(tid), _ptr(pv),
                                      _ptr(stp),
                                      _ptr(pr), _ptr(ns), _ptr(fl), _ptr(dg), threads or default_threads())
        assert rc == 0
        return {"pv": pv, "step": stp, "proc": pr, "nsteps": ns, "flags": fl, "diag": dg}


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: four 32-bit words from counter[4] and key[2]."""
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(o))
    return o


def uniform(seed, track, step, proc):
    return lib().orc_uniform(int(seed), int(track), int(step), int(proc))


def phys_length(materials, mat, seed, track, step):
    """Shortest sampled interaction length (and its process) per entry."""
    den = _f64(materials["density"])
    sig = np.ascontiguousarray(materials["sigma"], np.float64)
    mat = np.ascontiguousarray(mat, np.int32)
    tr = np.ascontiguousarray(track, np.uint32)
    st = np.ascontiguousarray(step, np.uint32)
    out = np.empty(mat.shape[0], np.float64)
    pr = np.empty(mat.shape[0], np.int32)
    rc = lib().orc_phys_length(den.shape[0], sig.shape[1], _ptr(den), _ptr(sig), mat.shape[0], _ptr(mat), int(seed),
                               _ptr(tr), _ptr(st), _ptr(out), _ptr(pr))
    assert rc == 0
    return out, pr
