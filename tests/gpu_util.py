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
