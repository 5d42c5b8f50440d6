"""Helpers for the GPU parity tests (comparison rules against the oracle)."""
import sys

import numpy as np

import oracle as O

# FP64 distances and safeties: |got - ref| <= 1e-12 max(|ref|, 1 mm); the
# sentinels -1 (wrong side) and +inf (miss) must match exactly.
REL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


FLAGGED = []  # (what, number flagged, first ids), printed at the end of the session


def record_flagged(what, ids):
    """Tracks the oracle flags as ill-conditioned are listed, not counted: keep
    them for the session's summary."""
    ids = np.asarray(ids)
    if ids.size:
        FLAGGED.append((what, int(ids.size), [int(i) for i in ids[:12]]))


def compare_values(got, ref, diag=None, rel=REL, what=""):
    """Returns (n_checked, flagged_and_different, bad_indices).  Tracks whose
    oracle diagnostic marks them ill-conditioned (D_ILL: near ties, grazes,
    band edges, and solid-level hits whose FP64 conditioning exceeds the bar)
    are listed in the session summary, not counted; every other value must
    meet the plain bar |got - ref| <= rel max(|ref|, 1 mm), sentinels exact."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    ok = np.ones(ref.shape, bool) if diag is None else (diag & O.D_ILL) == 0
    sent = (ref == -1.0) | np.isinf(ref)
    bad_sent = sent & (got != ref)
    fin = ~sent
    with np.errstate(invalid="ignore"):
        err = np.abs(got - ref)
    bad_val = fin & ~(err <= rel * np.maximum(np.abs(ref), 1.0))
    bad = (bad_sent | bad_val)
    flagged = np.nonzero(bad & ~ok)[0]
    record_flagged(f"{what} (flagged, differ)", flagged)
    if diag is not None:
        record_flagged(f"{what} (flagged)", np.nonzero(~ok)[0])
    real = np.nonzero(bad & ok)[0]
    if real.size:
        i = real[0]
        say(f"  {what}: {real.size} mismatches, first i={i} got={got[i]!r} ref={ref[i]!r}")
    return int(ok.sum()), flagged, real


# Navigation steps: both codes advance the global point p += s d in FP64; after
# k steps the points differ by up to ~k ulp(|p|) (ulp(2048 mm) = 4.5e-13 mm, k
# <= 84 on the detector, so ~4e-11 mm), and a step measured from a shifted point
# shifts by as much over the cosine of the hit angle.
STEP_REL = 1e-12
STEP_ABS = 1e-10


def transport_rows_compare(got, ref, idx=None, what="transport", proc=False, chunk=1 << 16):
    """Every track of a GPU transport against the oracle's, vectorised:
    sequences, step counts, flags (and processes) bit-exact for tracks the
    oracle does not flag as ill-conditioned (those are listed); steps within
    STEP_REL relative (1 mm floor) + STEP_ABS.  got: the binding's dict of
    device tensors (rows idx of it when given); ref: the oracle's dict.
    Returns (well-conditioned tracks, worst step error)."""
    gns = host(got["nsteps"])
    gfl = host(got["flags"]).astype(np.uint32)
    if idx is not None:
        gns, gfl = gns[idx], gfl[idx]
    rns = np.asarray(ref["nsteps"])
    n, ms = np.asarray(ref["step"]).shape
    ok = (np.asarray(ref["diag"]) & O.D_ILL) == 0
    bad = (gns != rns) | (gfl != np.asarray(ref["flags"]).astype(np.uint32))
    worst = 0.0
    k = np.arange(ms)[None, :]
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        if idx is None:
            rows = slice(a, b)
        else:
            import torch
            rows = torch.as_tensor(np.asarray(idx)[a:b], device=got["pv"].device)
        gpv = host(got["pv"][rows])
        gst = host(got["step"][rows])
        rpv = np.asarray(ref["pv"][a:b])
        rst = np.asarray(ref["step"][a:b])
        m = k < rns[a:b, None]
        bad[a:b] |= gpv[:, 0] != rpv[:, 0]
        bad[a:b] |= np.any((gpv[:, 1:] != rpv[:, 1:]) & m, axis=1)
        with np.errstate(invalid="ignore"):
            err = np.where(m, np.abs(gst - rst), 0.0)
            lim = STEP_REL * np.maximum(1.0, np.abs(rst)) + STEP_ABS
        bad[a:b] |= np.any(m & ~(err <= lim), axis=1)
        if proc:
            bad[a:b] |= np.any((host(got["proc"][rows]) != np.asarray(ref["proc"][a:b])) & m, axis=1)
        good = ~bad[a:b]
        if good.any():
            worst = max(worst, float(np.max(err[good])))
    flagged = np.nonzero(bad & ~ok)[0]
    record_flagged(f"{what} (flagged, differ)", flagged)
    record_flagged(f"{what} (flagged)", np.nonzero(~ok)[0])
    real = np.nonzero(bad & ok)[0]
    say(f"  {what}: {n} tracks, {int(ok.sum())} well-conditioned, {int(rns.sum())} track-steps, "
        f"worst |dstep| {worst:.3e} mm, {flagged.size} flagged differ")
    assert real.size == 0, (what, real[:10].tolist())
    return int(ok.sum()), worst


def transport_bits_equal(a, b, proc=False):
    """Two GPU transports' outputs bit for bit (entries past each track's last
    step are not outputs and are skipped)."""
    import torch
    if not (torch.equal(a["nsteps"], b["nsteps"]) and torch.equal(a["flags"], b["flags"])):
        return False
    ns = a["nsteps"].long()
    k = torch.arange(a["step"].shape[1], device=ns.device)[None, :]
    m = k < ns[:, None]
    mp = torch.cat([torch.ones_like(m[:, :1]), m], dim=1)
    if not torch.equal(a["pv"][mp], b["pv"][mp]):
        return False
    if not torch.equal(a["step"][m].view(torch.int64), b["step"][m].view(torch.int64)):
        return False
    return not proc or torch.equal(a["proc"][m], b["proc"][m])


_ORACLE_CACHE = {}


def oracle_detector_transport(og, key, fn):
    """The oracle's transport of a large workload, computed once per session
    (several tests compare against the same 2^20-track result)."""
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = fn(og)
    return _ORACLE_CACHE[key]
