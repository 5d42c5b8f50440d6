"""Python binding of libgvgeom.so -- the MI355X basket geometry library.

Argument marshalling only: every query runs in the HIP kernels behind the C-ABI of
include/gvgeom.h.  torch supplies device memory (tensors on "cuda") and the
current HIP stream; it computes nothing here.  There is no CPU fallback: if the
library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgvgeom.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gvgeom.h")

GV_OK, GV_EINVAL, GV_ENOMEM, GV_EHIP, GV_EFORMAT, GV_ESTATE, GV_EAGAIN = 0, -1, -2, -3, -4, -5, -6
Q_STEP, Q_SAFETY, Q_INSIDE = 0, 1, 2
SERVE_GRAPH = 1
OUTSIDE, SURFACE, INSIDE = 0, 1, 2
TO_IN, TO_OUT = 0, 1
SAFETY_AUTO, SAFETY_IN, SAFETY_OUT = 0, 1, 2
FP64, FP32_REFINE = 0, 1
WORK_N = 33  # work counters returned by gv_profile_read (28 transport, 5 polycone)
PROF_EVENTS, PROF_WORK = 1, 2
TUNING_FIELDS = ("step_grid", "scatter_grid", "cell_bits", "solid_block", "solid_grid", "step_waves",
                 "transport", "sort_bits", "sort_key", "lane_waves", "lane_stage", "lane_grid", "lane_sched")


class _Tuning(C.Structure):
    _fields_ = [(f, C.c_int32) for f in TUNING_FIELDS]
PHYS_SAFETY_SHORTCUT = 1
FLAG_OVERFLOW, FLAG_STUCK, FLAG_LOCATE_FAIL = 1, 2, 4

_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_SIGS = {
    "geom_load": [_P, C.c_size_t, C.POINTER(_P)],
    "geom_free": [_P],
    "geom_info": [_P, _P],
    "basket_inside": [_P, _I32, _I64, _P, _P, _P, _P, _P],
    "basket_safety": [_P, _I32, _I32, _I64, _P, _P, _P, _P, _P, _I32, _P],
    "basket_distance": [_P, _I32, _I32, _I64] + [_P] * 7 + [_I32, _P],
    "basket_solid_all": [_P, _I32, _I64] + [_P] * 10 + [_P],
    "basket_locate": [_P, _I64, _P, _P, _P, _P, _P],
    "basket_step": [_P, _I64] + [_P] * 11 + [_I32, _P],
    "basket_nav_safety": [_P, _I64, _P, _P, _P, _P, _P, _I32, _P],
    "basket_nav_inside": [_P, _I64, _P, _P, _P, _P, _P, _P],
    "nav_transport": [_P, _I64] + [_P] * 7 + [_I32] + [_P] * 4 + [_I32, _P],
    "nav_transport_noalloc": [_P, _I64] + [_P] * 7 + [_I32] + [_P] * 4 + [_I32, _P],
    "gv_profile": [_P, C.c_int],
    "gv_profile_read": [_P, _P, _P, _P],
    "gv_set_tuning": [_P, _P],
    "gv_probe_stream": [_P, _P, _P, C.c_double, _I64, _P],
    "gv_probe_fma64": [_P, _I64, _I32, _P],
    "gv_get_tuning": [_P, _P],
    "geom_set_materials": [_P, _I32, _I32, _P, _P, _P],
    "nav_transport_phys": [_P, _I64] + [_P] * 7 + [_I32, C.c_uint64] + [_P] * 5 + [_I32, _I32, _P],
    "gv_server_create": [_P, _I32, _I64, _I32, _I32, C.POINTER(_P)],
    "gv_server_submit": [_P, _I32, _I32, _I64, _P, _P, _P],
    "gv_server_poll": [_P, _I32, _P, _P, _P],
    "gv_server_drain": [_P],
    "gv_server_stats": [_P, _P],
    "gv_server_destroy": [_P],
}

_lib = None


class GVError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


def lib():
    """Load libgvgeom.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        # torch ships its own libamdhip64.so.7; loading it first lets the library
        # bind to that runtime by SONAME, so the process holds one HIP runtime
        # and torch's device pointers and streams are valid in our launches.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.gv_last_error.restype = C.c_char_p
        L.gv_last_error.argtypes = []
        L.gv_now.restype = C.c_double
        L.gv_now.argtypes = []
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared by include/gvgeom.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|double|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def _check(fn, rc):
    if rc != GV_OK:
        raise GVError(fn, rc, lib().gv_last_error().decode(errors="replace"))


def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dev(t, dtype, name, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor on the GPU")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: tensor must live on the GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _opt(t, dtype, name, numel=None):
    return None if t is None else _dev(t, dtype, name, numel)


def _n(*ts):
    """Common length of the basket arrays; every array must hold exactly n elements."""
    n = ts[0].numel()
    for t in ts[1:]:
        if t is not None and t.numel() != n:
            raise ValueError(f"basket arrays differ in length ({t.numel()} != {n})")
    return n


class Geometry:
    """A geometry resident on the current GPU (geom_load / geom_free)."""

    def __init__(self, blob: bytes, tuned: bool = True):
        """tuned: apply the launch shapes the autotuner stored for this GPU's
        architecture (paper_1512_06637_amd/tuned.json), if any."""
        h = C.c_void_p()
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check("geom_load", lib().geom_load(buf, len(blob), C.byref(h)))
        self._h = h
        counts = (C.c_int32 * 4)()
        _check("geom_info", lib().geom_info(self._h, counts))
        self.n_lv, self.n_pv, self.max_depth, self.world_lv = list(counts)
        if tuned:
            from . import tune
            choice = tune.stored_choice()
            if choice:
                self.set_tuning(**choice)

    def get_tuning(self) -> dict:
        t = _Tuning()
        _check("gv_get_tuning", lib().gv_get_tuning(self._h, C.byref(t)))
        return {f: getattr(t, f) for f in TUNING_FIELDS}

    def set_tuning(self, **fields):
        """Launch shapes (gvgeom.h gv_tuning); fields not given keep their value.
        None of them changes a result."""
        cur = self.get_tuning()
        for k, v in fields.items():
            if k not in cur:
                raise KeyError(f"unknown tuning field {k!r}")
            cur[k] = int(v)
        t = _Tuning(*[cur[f] for f in TUNING_FIELDS])
        _check("gv_set_tuning", lib().gv_set_tuning(self._h, C.byref(t)))

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check("geom_free", lib().geom_free(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ----------------------------------------------------------- solid level
    def inside(self, lv, x, y, z, out=None):
        torch = _torch()
        n = _n(x, y, z, out)
        out = torch.empty(n, dtype=torch.int8, device=x.device) if out is None else out
        f64 = torch.float64
        _check("basket_inside", lib().basket_inside(self._h, lv, n, _dev(x, f64, "x"), _dev(y, f64, "y"),
                                                    _dev(z, f64, "z"), _dev(out, torch.int8, "out"), _stream()))
        return out

    def safety(self, lv, x, y, z, side=SAFETY_AUTO, out=None, out_inside=None, precision=FP64):
        torch = _torch()
        n = _n(x, y, z, out, out_inside)
        out = torch.empty(n, dtype=torch.float64, device=x.device) if out is None else out
        f64 = torch.float64
        _check("basket_safety", lib().basket_safety(
            self._h, lv, side, n, _dev(x, f64, "x"), _dev(y, f64, "y"), _dev(z, f64, "z"), _dev(out, f64, "out"),
            _opt(out_inside, torch.int8, "out_inside"), precision, _stream()))
        return out

    def distance(self, lv, direction, x, y, z, dx, dy, dz, out=None, precision=FP64):
        torch = _torch()
        n = _n(x, y, z, dx, dy, dz, out)
        out = torch.empty(n, dtype=torch.float64, device=x.device) if out is None else out
        f64 = torch.float64
        a = [_dev(v, f64, nm) for v, nm in zip((x, y, z, dx, dy, dz), ("x", "y", "z", "dx", "dy", "dz"))]
        _check("basket_distance", lib().basket_distance(self._h, lv, direction, n, *a, _dev(out, f64, "out"),
                                                        precision, _stream()))
        return out

    def solid_all(self, lv, x, y, z, dx, dy, dz, out_inside=None, out_safety=None, out_din=None, out_dout=None):
        torch = _torch()
        n = _n(x, y, z, dx, dy, dz, out_inside, out_safety, out_din, out_dout)
        f64 = torch.float64
        a = [_dev(v, f64, nm) for v, nm in zip((x, y, z, dx, dy, dz), ("x", "y", "z", "dx", "dy", "dz"))]
        _check("basket_solid_all", lib().basket_solid_all(
            self._h, lv, n, *a, _opt(out_inside, torch.int8, "out_inside"), _opt(out_safety, f64, "out_safety"),
            _opt(out_din, f64, "out_din"), _opt(out_dout, f64, "out_dout"), _stream()))

    # ------------------------------------------------------------ navigation
    def locate(self, x, y, z, out=None):
        torch = _torch()
        n = _n(x, y, z, out)
        out = torch.empty(n, dtype=torch.int32, device=x.device) if out is None else out
        f64 = torch.float64
        _check("basket_locate", lib().basket_locate(self._h, n, _dev(x, f64, "x"), _dev(y, f64, "y"),
                                                    _dev(z, f64, "z"), _dev(out, torch.int32, "out"), _stream()))
        return out

    def step(self, x, y, z, dx, dy, dz, pv, pstep=None, out_step=None, out_next=None, out_flags=None,
             precision=FP64):
        torch = _torch()
        n = _n(x, y, z, dx, dy, dz, pv, pstep, out_step, out_next, out_flags)
        f64 = torch.float64
        out_step = torch.empty(n, dtype=f64, device=x.device) if out_step is None else out_step
        out_next = torch.empty(n, dtype=torch.int32, device=x.device) if out_next is None else out_next
        a = [_dev(v, f64, nm) for v, nm in zip((x, y, z, dx, dy, dz), ("x", "y", "z", "dx", "dy", "dz"))]
        _check("basket_step", lib().basket_step(
            self._h, n, *a, _dev(pv, torch.int32, "pv"), _opt(pstep, f64, "pstep"), _dev(out_step, f64, "out_step"),
            _dev(out_next, torch.int32, "out_next"), _opt(out_flags, torch.int32, "out_flags"), precision,
            _stream()))
        return out_step, out_next

    def nav_safety(self, x, y, z, pv, out=None, precision=FP64):
        torch = _torch()
        n = _n(x, y, z, pv, out)
        f64 = torch.float64
        out = torch.empty(n, dtype=f64, device=x.device) if out is None else out
        _check("basket_nav_safety", lib().basket_nav_safety(
            self._h, n, _dev(x, f64, "x"), _dev(y, f64, "y"), _dev(z, f64, "z"), _dev(pv, torch.int32, "pv"),
            _dev(out, f64, "out"), precision, _stream()))
        return out

    def nav_inside(self, x, y, z, pv, out=None):
        torch = _torch()
        n = _n(x, y, z, pv, out)
        f64 = torch.float64
        out = torch.empty(n, dtype=torch.int8, device=x.device) if out is None else out
        _check("basket_nav_inside", lib().basket_nav_inside(
            self._h, n, _dev(x, f64, "x"), _dev(y, f64, "y"), _dev(z, f64, "z"), _dev(pv, torch.int32, "pv"),
            _dev(out, torch.int8, "out"), _stream()))
        return out

    def profile(self, events=False, work=False):
        """events: time every per-step kernel launch of basket transports with HIP
        events (production kernels); work: run the instance that keeps operation
        counters.  profile() turns both off."""
        flags = (PROF_EVENTS if events else 0) | (PROF_WORK if work else 0)
        _check("gv_profile", lib().gv_profile(self._h, flags))

    def profile_read(self):
        """(step-kernel ms, launches, work counts: [0] steps, [1] bounding-box tests,
        [2+t] lower-bound checks, [8+t] culled DistanceToIn, [14+t] plain DistanceToIn,
        t = daughter solid type, [20] culled track-steps screened in FP32, [21] culled
        track-steps screened in FP64, [22] physics-limited steps, [23] of which taken
        by the safety short-cut, [24] radial-order lookups, [25] radial crossing
        bounds, [26] phi-sector lookups, [27] sectors read; then the polycone
        queries' [28] DistanceToIn sections computed, [29] DistanceToOut sections
        computed, [30] DistanceToIn bounding-cylinder rejects, [31] DistanceToIn
        walks, [32] DistanceToOut walks)."""
        ms = C.c_double(0.0)
        launches = C.c_int64(0)
        work = (C.c_uint64 * WORK_N)()
        _check("gv_profile_read", lib().gv_profile_read(self._h, C.byref(ms), C.byref(launches), work))
        return ms.value, launches.value, list(work)

    def set_materials(self, density, sigma, lv_material):
        """Materials for physics-limited transport (host arrays)."""
        import numpy as np
        den = np.ascontiguousarray(density, np.float64)
        sig = np.ascontiguousarray(sigma, np.float64)
        lvm = np.ascontiguousarray(lv_material, np.int32)
        if sig.ndim != 2 or sig.shape[0] != den.shape[0]:
            raise ValueError("sigma must be [n_mat][n_proc]")
        _check("geom_set_materials", lib().geom_set_materials(
            self._h, den.shape[0], sig.shape[1], C.c_void_p(den.ctypes.data), C.c_void_p(sig.ctypes.data),
            C.c_void_p(lvm.ctypes.data)))

    def transport_phys(self, x, y, z, dx, dy, dz, seed, start_pv=None, max_steps=128, out=None, shortcut=True,
                       precision=FP64):
        """Physics-limited transport; dict as transport() plus proc [n, max_steps] int8."""
        torch = _torch()
        n = _n(x, y, z, dx, dy, dz, start_pv)
        f64 = torch.float64
        if out is None:
            out = {
                "pv": torch.full((n, max_steps + 1), -2, dtype=torch.int32, device=x.device),
                "step": torch.full((n, max_steps), float("nan"), dtype=f64, device=x.device),
                "proc": torch.full((n, max_steps), -2, dtype=torch.int8, device=x.device),
                "nsteps": torch.empty(n, dtype=torch.int32, device=x.device),
                "flags": torch.empty(n, dtype=torch.int32, device=x.device),
            }
        a = [_dev(v, f64, nm) for v, nm in zip((x, y, z, dx, dy, dz), ("x", "y", "z", "dx", "dy", "dz"))]
        _check("nav_transport_phys", lib().nav_transport_phys(
            self._h, n, *a, _opt(start_pv, torch.int32, "start_pv"), max_steps, int(seed),
            _dev(out["pv"], torch.int32, "pv", n * (max_steps + 1)), _dev(out["step"], f64, "step", n * max_steps),
            _opt(out.get("proc"), torch.int8, "proc", n * max_steps), _dev(out["nsteps"], torch.int32, "nsteps", n),
            _dev(out["flags"], torch.int32, "flags", n), PHYS_SAFETY_SHORTCUT if shortcut else 0, precision,
            _stream()))
        return out

    def transport(self, x, y, z, dx, dy, dz, start_pv=None, max_steps=128, out=None, precision=FP64,
                  noalloc=False):
        """Returns dict(pv [n, max_steps+1] int32, step [n, max_steps] f64, nsteps, flags).
        noalloc: call nav_transport_noalloc (library scratch, no allocation;
        `out` must then be given to allocate nothing here either)."""
        torch = _torch()
        n = _n(x, y, z, dx, dy, dz, start_pv)
        f64 = torch.float64
        if out is None:
            out = {
                "pv": torch.full((n, max_steps + 1), -2, dtype=torch.int32, device=x.device),
                "step": torch.full((n, max_steps), float("nan"), dtype=f64, device=x.device),
                "nsteps": torch.empty(n, dtype=torch.int32, device=x.device),
                "flags": torch.empty(n, dtype=torch.int32, device=x.device),
            }
        a = [_dev(v, f64, nm) for v, nm in zip((x, y, z, dx, dy, dz), ("x", "y", "z", "dx", "dy", "dz"))]
        fn = "nav_transport_noalloc" if noalloc else "nav_transport"
        _check(fn, getattr(lib(), fn)(
            self._h, n, *a, _opt(start_pv, torch.int32, "start_pv"), max_steps,
            _dev(out["pv"], torch.int32, "pv", n * (max_steps + 1)), _dev(out["step"], f64, "step", n * max_steps),
            _dev(out["nsteps"], torch.int32, "nsteps", n), _dev(out["flags"], torch.int32, "flags", n), precision,
            _stream()))
        return out


# ------------------------------------------------------------ roof probes
def probe_stream(a, b, c, s=1.0):
    """c = a + s b (b None: c = a) on device float64 tensors of one even length."""
    torch = _torch()
    n = _n(a, b, c)
    _check("gv_probe_stream", lib().gv_probe_stream(
        _dev(a, torch.float64, "a"), _opt(b, torch.float64, "b"), _dev(c, torch.float64, "c"), float(s), n,
        _stream()))


def probe_fma64(out, iters):
    """out: device float64 tensor, one element per lane (multiple of 256)."""
    torch = _torch()
    _check("gv_probe_fma64", lib().gv_probe_fma64(_dev(out, torch.float64, "out"), out.numel(), int(iters),
                                                  _stream()))


# ------------------------------------------------------------------ serving
def serve_in_bytes(kind, n):
    return (60 if kind == Q_STEP else 28) * n


def serve_out_bytes(kind, n):
    return (16 if kind == Q_STEP else 8 if kind == Q_SAFETY else 1) * n


def pack_basket(kind, x, y, z, pv, dx=None, dy=None, dz=None, pstep=None):
    """Host byte block of one basket in the serving layout (numpy uint8)."""
    import numpy as np
    n = len(x)
    f = [np.ascontiguousarray(v, np.float64) for v in (x, y, z)]
    if kind == Q_STEP:
        ps = np.full(n, np.inf) if pstep is None else pstep
        f += [np.ascontiguousarray(v, np.float64) for v in (dx, dy, dz, ps)]
    parts = [v.view(np.uint8) for v in f] + [np.ascontiguousarray(pv, np.int32).view(np.uint8)]
    out = np.concatenate(parts)
    assert out.size == serve_in_bytes(kind, n)
    return out


def unpack_result(kind, buf, n):
    """Views of a basket's output block: (step, next_pv, flags), safety, or code."""
    import numpy as np
    if kind == Q_STEP:
        return (buf[:8 * n].view(np.float64), buf[8 * n:12 * n].view(np.int32), buf[12 * n:16 * n].view(np.uint32))
    if kind == Q_SAFETY:
        return buf[:8 * n].view(np.float64)
    return buf[:n].view(np.int8)


def now():
    """Seconds on the clock of Server.poll's completion times."""
    return lib().gv_now()


class Server:
    """Serving engine over a resident Geometry (gv_server_* of include/gvgeom.h).
    Input and output blocks are host numpy uint8 arrays in the serving layout;
    an output block must stay alive until poll() returns its ticket."""

    def __init__(self, geometry, slots=64, hbm_budget=256 << 20, nstreams=2, graphs=True):
        """graphs: every round is one launch of a per-stream HIP graph (GV_SERVE_GRAPH)."""
        self._g = geometry
        h = C.c_void_p()
        _check("gv_server_create", lib().gv_server_create(geometry._h, slots, hbm_budget, nstreams,
                                                          SERVE_GRAPH if graphs else 0, C.byref(h)))
        self._h = h
        self._keep = {}  # ticket -> output buffer (kept alive until returned)

    def submit(self, kind, precision, n, inbuf, outbuf):
        """Ticket, or None when the server is full now (GV_EAGAIN)."""
        import numpy as np
        assert inbuf.dtype == np.uint8 and inbuf.flags.c_contiguous and inbuf.size == serve_in_bytes(kind, n)
        assert outbuf.dtype == np.uint8 and outbuf.flags.c_contiguous and outbuf.size == serve_out_bytes(kind, n)
        t = C.c_uint64(0)
        rc = lib().gv_server_submit(self._h, kind, precision, n, C.c_void_p(inbuf.ctypes.data),
                                    C.c_void_p(outbuf.ctypes.data), C.byref(t))
        if rc == GV_EAGAIN:
            return None
        _check("gv_server_submit", rc)
        self._keep[t.value] = outbuf
        return t.value

    def poll(self, max_n=1024):
        """[(ticket, device completion time)] of baskets finished since the last poll."""
        tk = (C.c_uint64 * max_n)()
        td = (C.c_double * max_n)()
        cnt = C.c_int32(0)
        _check("gv_server_poll", lib().gv_server_poll(self._h, max_n, tk, td, C.byref(cnt)))
        out = [(tk[i], td[i]) for i in range(cnt.value)]
        for t, _ in out:
            self._keep.pop(t, None)
        return out

    def drain(self):
        _check("gv_server_drain", lib().gv_server_drain(self._h))

    def stats(self):
        v = (C.c_int64 * 8)()
        _check("gv_server_stats", lib().gv_server_stats(self._h, v))
        keys = ("admitted", "waiting", "rounds", "baskets", "tracks", "max_round", "in_bytes", "out_bytes")
        return dict(zip(keys, list(v)))

    def close(self):
        if self._h:
            rc = lib().gv_server_destroy(self._h)
            self._h = None
            _check("gv_server_destroy", rc)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
