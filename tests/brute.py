"""Brute-force numpy references used to pin the oracle (tests only).

They enumerate all pairs, so they are independent of any cell list, schedule
or stencil.  The minimum image is taken as d - L*rint(d/L); for |d| < L this
equals the per-axis conditional form exactly (d -/+ L is exact there by
Sterbenz's lemma, and rint(+-0.5) == 0 leaves d = +-L/2 unchanged as the
conditional form does).
"""
import numpy as np


def minimg(d, L):
    return d - L * np.rint(d / L)


def q_to_all(rows, y, box, dim):
    """Squared minimum-image distances from point y to every row, summed in
    the order (d0*d0 + d1*d1) + d2*d2."""
    d0 = minimg(y[0] - rows[:, 0], box[0])
    d1 = minimg(y[1] - rows[:, 1], box[1])
    q = d0 * d0 + d1 * d1
    if dim == 3:
        d2 = minimg(y[2] - rows[:, 2], box[2])
        q = q + d2 * d2
    return q


def overlapping_pairs(rows, radii, box, dim, gap=0.0):
    """All i<j with q_ij <= ((R_i + R_j) + gap)^2, sorted by (i, j)."""
    n = rows.shape[0]
    out = []
    for i in range(n - 1):
        q = q_to_all(rows[i + 1:], rows[i], box, dim)
        sig = (radii[i] + radii[i + 1:]) + gap
        js = np.nonzero(q <= sig * sig)[0] + i + 1
        out.extend((i, int(j)) for j in js)
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def any_overlap(rows, radii, box, dim):
    return len(overlapping_pairs(rows, radii, box, dim)) > 0


def colliding(rows, radii, i, y, box, dim):
    """Does particle i placed at y overlap any other particle (all pairs)?"""
    q = q_to_all(rows, y, box, dim)
    sig = radii[i] + radii
    hit = q <= sig * sig
    hit[i] = False
    return bool(hit.any())
