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


def _disk_point_dist(P, c, n, A):
    """Long-double distances of points P (k, 3) to the disk (centre c, unit
    normal n, radius A): the foot on the plane, pulled back to the rim when
    it falls outside."""
    x = P - c
    h = x @ n
    foot = x - np.outer(h, n)
    r = np.sqrt(np.sum(foot * foot, axis=1))
    out = np.maximum(r - A, 0)
    return np.sqrt(h * h + out * out)


def _rim(c, n, A, th):
    e1 = np.cross(n, np.array([1, 0, 0], dtype=np.longdouble) if abs(n[0]) < 0.9
                  else np.array([0, 1, 0], dtype=np.longdouble))
    e1 = e1 / np.sqrt(np.dot(e1, e1))
    e2 = np.cross(n, e1)
    th = np.asarray(th, dtype=np.longdouble)
    return c + A * (np.outer(np.cos(th), e1) + np.outer(np.sin(th), e2))


def core_distance(d, n1, A1, n2, A2, samples=720):
    """Minimum distance between two flat disks: disk 1 at the origin
    (normal n1, radius A1), disk 2 at d (n2, A2).  0 when the chords test
    says they meet; otherwise a closest pair has a point on a rim, so the
    distance is the smaller of min over rim 1 of the distance to disk 2 and
    the same with the roles swapped -- each found by sampling the rim
    angle densely, then golden-section search (long double) around the six
    best samples."""
    meet, _ = chords_meet(d, n1, A1, n2, A2)
    if meet:
        return 0.0
    d = np.asarray(d, dtype=np.longdouble)
    n1 = np.asarray(n1, dtype=np.longdouble)
    n2 = np.asarray(n2, dtype=np.longdouble)
    z = np.zeros(3, dtype=np.longdouble)
    best = np.longdouble(np.inf)
    step = 2 * np.pi / samples
    for (c, n, A, cc, nn, AA) in ((z, n1, A1, d, n2, A2), (d, n2, A2, z, n1, A1)):
        A, AA = np.longdouble(A), np.longdouble(AA)
        th = np.arange(samples, dtype=np.longdouble) * np.longdouble(step)
        f = _disk_point_dist(_rim(c, n, A, th), cc, nn, AA)

        # golden-section search, six brackets at once
        idx = np.argsort(f)[:6]
        lo = th[idx] - np.longdouble(step)
        hi = th[idx] + np.longdouble(step)
        r = (np.sqrt(np.longdouble(5)) - 1) / 2
        x1, x2 = hi - r * (hi - lo), lo + r * (hi - lo)
        f1 = _disk_point_dist(_rim(c, n, A, x1), cc, nn, AA)
        f2 = _disk_point_dist(_rim(c, n, A, x2), cc, nn, AA)
        for _ in range(64):
            left = f1 <= f2  # the minimum lies in [lo, x2]
            hi = np.where(left, x2, hi)
            lo = np.where(left, lo, x1)
            x1n = np.where(left, hi - r * (hi - lo), x2)
            x2n = np.where(left, x1, lo + r * (hi - lo))
            fk = np.where(left, f1, f2)  # the kept interior value
            fnew = _disk_point_dist(_rim(c, n, A, np.where(left, x1n, x2n)), cc, nn, AA)
            f1 = np.where(left, fnew, fk)
            f2 = np.where(left, fk, fnew)
            x1, x2 = x1n, x2n
        best = min(best, f1.min(), f2.min(), f[idx].min())
    return float(best)
