"""An independent thin-disk intersection test (tests only).

Two zero-thickness disks meet exactly when the chords that their planes'
common line cuts from each disk overlap.  This module finds a point of that
line with a general 3x3 linear solve (numpy, float64) and then works in
long double: the chord of disk 1 is |t| <= sqrt(A/uu) around the foot of
centre 1, the chord of disk 2 is |t - t1| <= sqrt(B/uu) around the foot of
centre 2.  The oracle instead writes the foot in closed form and compares
squared chord lengths without a square root, so the two share no formula.
Each answer comes with the distance of its deciding quantity from the
decision boundary, so callers can skip rounding-level ties.
"""
import numpy as np


def chords_meet(d, n1, a1, n2, a2):
    """Disk 1 at the origin (normal n1, radius a1), disk 2 at d.
    Returns (meet, margin)."""
    d = np.asarray(d, dtype=np.longdouble)
    n1l = np.asarray(n1, dtype=np.longdouble)
    n2l = np.asarray(n2, dtype=np.longdouble)
    u = np.cross(n1l, n2l)
    M = np.array([n1l, n2l, u], dtype=np.float64)
    rhs = np.array([0.0, float(np.dot(n2l, d)), 0.0])
    p = np.linalg.solve(M, rhs).astype(np.longdouble)  # on both planes, closest to disk 1
    uu = np.dot(u, u)
    A = np.longdouble(a1) * np.longdouble(a1) - np.dot(p, p)
    t1 = np.dot(d - p, u) / uu
    e2 = d - (p + t1 * u)
    B = np.longdouble(a2) * np.longdouble(a2) - np.dot(e2, e2)
    if A < 0 or B < 0:
        return False, float(min(abs(A), abs(B)))
    reach = np.sqrt(A / uu) + np.sqrt(B / uu)
    return bool(abs(t1) <= reach), float(abs(abs(t1) - reach))


def chords_overlap_ref(c1, n1, a1, c2, n2, a2):
    """The same test for centres c1, c2 (no periodic image)."""
    d = np.asarray(c2, dtype=np.longdouble) - np.asarray(c1, dtype=np.longdouble)
    return chords_meet(d, n1, a1, n2, a2)
