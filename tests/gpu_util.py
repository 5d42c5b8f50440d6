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


EPS = 2.0 ** -52


def conditioning_allowance(solid, tracks, ref):
    """Difference two correct FP64 evaluations of a hit distance may show: the
    inputs and intermediate products carry a few ulp of the coordinate scale L,
    and the hit distance moves by that over |cos theta|, theta being the angle
    between the ray and the surface normal at the hit.  The normal is the
    central-difference gradient of the oracle's signed term at the hit point;
    L = (|p|^2 + |q|^2) / max(1 mm, |q|) also covers the C = |p|^2 - R^2 term of
    quadric surfaces (q is the hit point)."""
    P = np.stack([tracks.x, tracks.y, tracks.z])
    D = np.stack([tracks.dx, tracks.dy, tracks.dz])
    Q = P + ref[None, :] * D
    h = 1e-6 * np.maximum(1.0, np.abs(Q).max(axis=0))
    grad = np.empty_like(Q)
    for k in range(3):
        e = np.zeros_like(Q)
        e[k] = h
        sp = O.signed(solid, *(Q + e))
        sm = O.signed(solid, *(Q - e))
        grad[k] = (sp - sm) / (2.0 * h)
    nrm = np.linalg.norm(grad, axis=0)
    cos = np.abs((grad * D).sum(axis=0)) / np.maximum(nrm, 1e-300)
    qn = np.linalg.norm(Q, axis=0)
    L = (np.linalg.norm(P, axis=0) ** 2 + qn ** 2) / np.maximum(1.0, qn)
    return 16.0 * EPS * L / np.maximum(cos, 1e-300)


def compare_values(got, ref, diag=None, rel=REL, what="", solid=None, tracks=None):
    """Returns (n_checked, n_flagged, bad_indices) where flagged tracks carry an
    oracle ill-conditioning diagnostic and are listed, not counted.  With solid
    and tracks given, a finite distance outside the plain bar is re-checked
    with the conditioning allowance of the hit."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    ok = np.ones(ref.shape, bool) if diag is None else (diag & O.D_ILL) == 0
    sent = (ref == -1.0) | np.isinf(ref)
    bad_sent = sent & (got != ref)
    fin = ~sent
    with np.errstate(invalid="ignore"):
        err = np.abs(got - ref)
    bad_val = fin & ~(err <= rel * np.maximum(np.abs(ref), 1.0))
    if solid is not None and bad_val.any():
        idx = np.nonzero(bad_val)[0]
        allow = conditioning_allowance(solid, tracks.take(idx), ref[idx])
        within = err[idx] <= rel * np.maximum(np.abs(ref[idx]), 1.0) + allow
        if within.any():
            say(f"  {what}: {int(within.sum())} ill-conditioned hits within their conditioning allowance "
                f"(worst uses {float(np.max(err[idx][within] / allow[within])):.2f} of it)")
        bad_val[idx[within]] = False
    bad = (bad_sent | bad_val)
    flagged = np.nonzero(bad & ~ok)[0]
    real = np.nonzero(bad & ok)[0]
    if real.size:
        i = real[0]
        say(f"  {what}: {real.size} mismatches, first i={i} got={got[i]!r} ref={ref[i]!r}")
    return int(ok.sum()), flagged, real
