"""Host-side work accounting behind the benchmark's roofline figures: step
classes read from PV sequences, and the culled navigator's operation count
reducing to the plain navigator's when its counters describe the plain loop."""
import numpy as np

from paper_1512_06637_amd import roofline as R


def test_step_classes_from_sequences():
    # detector PV numbering: 0 world, 1 + 65 i layer i, the 64 PVs after it its modules
    garbage = 999
    pv = np.array([
        [0, 1, 5, 1, 0, -1, garbage],        # world, layer 0, module, layer 0, world
        [66, 70, 66, -1, garbage, garbage, garbage],  # layer 1, module of layer 1, layer 1
        [3, -1, garbage, garbage, garbage, garbage, garbage],  # one module step
        [0, garbage, garbage, garbage, garbage, garbage, garbage],  # no step taken
    ])
    nsteps = np.array([5, 3, 1, 0])
    assert R.detector_step_classes(pv, nsteps) == (2, 4, 3)


def test_culled_count_with_plain_counters_is_the_plain_count():
    """A world step evaluating every one of the 20 tube daughters through the
    plain loop, a layer step evaluating all 64 box modules, and a module step
    (no daughters) cost what the plain navigator costs, plus the ray set-up the
    culled loop does once per step in a volume with daughters."""
    w = [0] * 28
    w[14 + 1] = 20
    assert R.detector_ops_culled(1, 0, 0, w) == R.detector_ops(1, 0, 0) + R.RAY_SETUP
    w = [0] * 28
    w[14 + 0] = 64
    assert R.detector_ops_culled(0, 1, 0, w) == R.detector_ops(0, 1, 0) + R.RAY_SETUP
    assert R.detector_ops_culled(0, 0, 1, [0] * 28) == R.detector_ops(0, 0, 1)


def test_counts_are_linear_and_culling_is_cheaper():
    w = [0] * 28
    w[1] = 23          # box tests of a culled world step
    w[2 + 1] = 12      # tube bounds
    w[8 + 1] = 2       # tube DistanceToIn after culling
    one = R.detector_ops_culled(1, 0, 0, w)
    assert R.detector_ops_culled(3, 0, 0, [3 * v for v in w]) == 3 * one
    assert one < R.detector_ops(1, 0, 0)
    # index lookups add their own terms
    w2 = list(w)
    w2[24], w2[25], w2[26], w2[27] = 1, 2, 1, 3
    extra = R.RADIAL_LOOKUP + 2 * R.RADIAL_BOUND + R.PHI_LOOKUP + 3 * R.PHI_SECTOR
    assert R.detector_ops_culled(1, 0, 0, w2) == one + extra


def test_byte_figures():
    assert R.STEP_DESIGN_BYTES == 152
    # 2 tracks, 5 steps: 2 x (48 in + start PV + nsteps + flags) + 5 x (PV + step)
    assert R.transport_bytes(2, 5) == 2 * 60 + 5 * 12


def test_polycone_ops_from_walk_counters():
    """The polycone's operation count follows its walk counters: no walk (every
    ray rejected or every point on the wrong side) leaves the inside test (and
    the reject); each walked section adds PCON_SECTION; the fused count is the
    inside test once, the safety and both distance parts."""
    n = 10
    w = [0] * 33
    assert R.pcon_ops("inside", n, w) == n * R.PCON_INSIDE
    assert R.pcon_ops("safety", n, w) == n * (R.PCON_INSIDE + R.PCON_SAFETY)
    w[30] = 4  # four rejected rays
    assert R.pcon_ops("dist_in", n, w) == n * R.PCON_INSIDE + 4 * R.PCON_REJECT
    w[31], w[28] = 3, 7  # three walks over seven sections in all
    din = (4 + 3) * R.PCON_REJECT + 3 * R.PCON_WALK + 7 * R.PCON_SECTION
    assert R.pcon_ops("dist_in", n, w) == n * R.PCON_INSIDE + din
    w[32], w[29] = 2, 5
    dout = 2 * R.PCON_WALK + 5 * R.PCON_SECTION
    assert R.pcon_ops("dist_out", n, w) == n * R.PCON_INSIDE + dout
    assert R.pcon_ops("fused", n, w) == n * (R.PCON_INSIDE + R.PCON_SAFETY) + din + dout
    # the full walk over all 9 sections is at most the table's estimate
    assert R.PCON_INSIDE + R.PCON_REJECT + R.PCON_WALK + 9 * R.PCON_SECTION <= R.SOLID_OPS["pcon"]["dist_in"] + 100
