"""Optimality-criteria design update (test oracle, FP64).

Section 3.2 (eq. kkt, eq. update): with B_e = -s~_e / lambda (the volume
derivative is one per cell, since all cells have equal volume and the
constraint counts cells), move limit m and damping eta,

    rho_new_e = clamp(rho_e * B_e^eta, max(rho_min, rho_e - m), min(1, rho_e + m)).

Section 3.2.1: lambda is found by bisection.  The bracket starts at
[0, 1e5]; at the midpoint the volume sum is compared with volfrac * N: if
it is larger, the lower end moves up, else the upper end moves down.  The
paper stops at an absolute width of 1e-4; this oracle instead bisects until
the midpoint is no longer strictly inside the bracket in FP64, so that the
volume constraint holds to rounding.  If the volume at the upper end still
exceeds the target, the upper end is multiplied by 10 until it does not.
The returned design is the one evaluated at the last midpoint, and the
change is the max-norm of rho_new - rho (Section 4.4 / Appendix loop).

Passive cells (Section 5.4): cells marked void are set to the lower density
bound (the paper writes 0.001, its rho_min) and cells marked solid to 1.
The setting is done inside every bisection evaluation, before the volume
sum, so the constraint counts them (the paper adds the assignment to the
OC loop without saying where; this is the reading taken).
"""

from __future__ import annotations

import numpy as np


VOID, SOLID = 1, 2


def _design(rho, neg_s, lam, move, eta, rho_min, passive=None, dv=None):
    lo = np.maximum(rho_min, rho - move)
    hi = np.minimum(1.0, rho + move)
    B = neg_s / lam if dv is None else neg_s / (dv * lam)
    out = np.maximum(lo, np.minimum(hi, rho * B ** eta))
    if passive is not None:
        out[passive == VOID] = rho_min
        out[passive == SOLID] = 1.0
    return out


def update(rho, s_filtered, volfrac, move=0.2, eta=0.5, rho_min=1e-3,
           l1=0.0, l2=1e5, max_expand=60, passive=None, dv=None, phys=None):
    """Returns (rho_new, lam, volume_sum, change, n_passes).  ``passive`` is
    None or one code per cell: 0 free, 1 void, 2 solid.

    Density-filter mode: ``dv`` is the volume gradient of the design (the
    ratio becomes -s / (lambda dv)) and ``phys`` maps a design to the
    filtered field whose sum is the volume compared with the target, as the
    filtered design is evaluated at every bisection step."""
    vol_of = (lambda x: x.sum()) if phys is None else (lambda x: phys(x).sum())
    rho = np.asarray(rho, dtype=np.float64)
    neg_s = np.maximum(0.0, -np.asarray(s_filtered, dtype=np.float64))
    target = volfrac * rho.size
    passes = 0
    for _ in range(max_expand):
        passes += 1
        if vol_of(_design(rho, neg_s, l2, move, eta, rho_min, passive, dv)) - target > 0:
            l1, l2 = l2, l2 * 10.0
        else:
            break
    rho_new = None
    lam = None
    while True:
        mid = 0.5 * (l1 + l2)
        if not (l1 < mid < l2):
            break
        passes += 1
        lam = mid
        rho_new = _design(rho, neg_s, mid, move, eta, rho_min, passive, dv)
        if vol_of(rho_new) - target > 0:
            l1 = mid
        else:
            l2 = mid
    vol = float(vol_of(rho_new))
    change = float(np.max(np.abs(rho_new - rho)))
    return rho_new, lam, vol, change, passes


def exact_root(rho, s_filtered, volfrac, move=0.2, rho_min=1e-3, passive=None):
    """Independent exact solution for eta = 1/2, used as a pin.

    With mu = lambda^(-1/2) each cell is clamp(a_e mu, lo_e, hi_e) with
    a_e = rho_e sqrt(-s~_e); the volume is piecewise linear and
    non-decreasing in mu.  Sorting the breakpoints and solving the linear
    piece that brackets the target gives the root exactly (up to rounding).
    Passive cells enter as a zero coefficient with both bounds at their fixed
    value (a constant term of the volume).  Returns (rho_new, lam)."""
    rho = np.asarray(rho, dtype=np.float64)
    a = rho * np.sqrt(np.maximum(0.0, -np.asarray(s_filtered, dtype=np.float64)))
    lo = np.maximum(rho_min, rho - move)
    hi = np.minimum(1.0, rho + move)
    if passive is not None:
        fixed = np.where(passive == SOLID, 1.0, rho_min)
        pas = passive != 0
        a = np.where(pas, 0.0, a)
        lo = np.where(pas, fixed, lo)
        hi = np.where(pas, fixed, hi)
    target = volfrac * rho.size
    pos = a > 0
    bps = np.unique(np.concatenate([lo[pos] / a[pos], hi[pos] / a[pos]]))

    def vol(mu):
        return np.clip(a * mu, lo, hi).sum()
    # find the segment [b_k, b_{k+1}] with vol(b_k) <= target <= vol(b_{k+1})
    vals = np.array([vol(b) for b in bps])
    k = int(np.searchsorted(vals, target))
    k = min(max(k, 1), len(bps) - 1)
    mid = 0.5 * (bps[k - 1] + bps[k])
    free = (a * mid > lo) & (a * mid < hi)
    at_lo = a * mid <= lo
    at_hi = a * mid >= hi
    mu = (target - lo[at_lo].sum() - hi[at_hi].sum()) / a[free].sum()
    rho_new = np.clip(a * mu, lo, hi)
    return rho_new, 1.0 / (mu * mu)
