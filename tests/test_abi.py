"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/gvgeom.h declares, and rejects bad arguments on the host side
before touching the device."""
import ctypes as C

import pytest

import paper_1512_06637_amd as G
from paper_1512_06637_amd import workloads as W


def test_exports_every_declared_symbol():
    names = G.header_functions()
    assert {"geom_load", "basket_distance", "basket_safety", "basket_step", "nav_transport"} <= set(names)
    L = G.lib()
    for n in names:
        assert hasattr(L, n), n


def _load(blob):
    h = C.c_void_p()
    buf = C.create_string_buffer(blob, len(blob))
    rc = G.lib().geom_load(buf, len(blob), C.byref(h))
    return rc, G.lib().gv_last_error().decode()


@pytest.mark.parametrize("mutate,expect", [
    (lambda b: b"XXXXXXXX" + b[8:], "magic"),
    (lambda b: b[:-8], "size"),
    (lambda b: b[:8] + (7).to_bytes(4, "little") + b[12:], "version"),
])
def test_geom_load_rejects_malformed_blob(mutate, expect):
    rc, msg = _load(mutate(W.detector_blob()))
    assert rc == G.GV_EFORMAT and expect in msg


def test_geom_load_rejects_bad_solid_and_cycles():
    rc, msg = _load(W.single_solid_blob(W.tubs(10.0, 5.0, 1.0)))
    assert rc == G.GV_EFORMAT and "tube" in msg
    lv = W.LV(W.box(1.0, 1.0, 1.0))
    lv.placements.append((0, [[1, 0, 0], [0, 1, 0], [0, 0, 1]], [0, 0, 0]))
    rc, msg = _load(W.make_blob([lv]))
    assert rc == G.GV_EFORMAT and "cycle" in msg


def test_null_handle_and_negative_n_are_rejected():
    L = G.lib()
    assert L.basket_distance(None, 0, 0, 10, *([None] * 7), 0, None) == G.GV_EINVAL
    assert "NULL" in L.gv_last_error().decode()
    assert L.nav_transport(None, -1, *([None] * 7), 128, *([None] * 4), 0, None) == G.GV_EINVAL
    assert L.geom_free(None) == G.GV_OK
    assert L.geom_load(None, 0, None) == G.GV_EINVAL


def test_server_argument_checks_need_no_gpu():
    """The serving entry points reject bad handles and arguments on the host."""
    L = G.lib()
    h = C.c_void_p()
    assert L.gv_server_create(None, 64, 256 << 20, 2, G.SERVE_GRAPH, C.byref(h)) == G.GV_EINVAL
    assert L.gv_server_create(None, 64, 256 << 20, 2, 0, None) == G.GV_EINVAL
    cnt = C.c_int32(0)
    assert L.gv_server_submit(None, 0, 0, 10, None, None, None) == G.GV_EINVAL
    assert L.gv_server_poll(None, 0, None, None, C.byref(cnt)) == G.GV_EINVAL
    assert L.gv_server_drain(None) == G.GV_EINVAL
    assert L.gv_server_stats(None, None) == G.GV_EINVAL
    assert L.gv_server_destroy(None) == G.GV_OK
    t0 = L.gv_now()
    assert L.gv_now() >= t0 > 0.0

