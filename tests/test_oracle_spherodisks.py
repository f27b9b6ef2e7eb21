"""Pins of the oracle's spherodisk platelets (Sec. 3.3 models its thin
platelets as spherodisks) against facts fixed outside it.

A spherodisk of outer radius a and thickness t = 2h is every point within h
of a flat core disk of radius A = a - h; two overlap iff their core disks
come within h_i + h_j.  The oracle decides that with certificates (a pair of
points closer than the bound, or a direction along which the disks'
projections are further apart), so its answers are checked here against:

* an independent core-disk distance (tests/disk_ref.py: the chords test for
  meeting disks, else dense sampling of each rim's distance to the other
  disk refined by golden-section search in long double), at 1e-9 of the
  distance on either side, for random pairs;
* closed forms: coplanar disks (|d| - A1 - A2), parallel stacked disks
  (the plane gap, or its hypotenuse with the lateral gap), a rim above a
  face (perpendicular disks), a rim facing a rim (T junction);
* the zero-thickness limit (the exact disk-disk intersection test) and the
  symmetry of the distance under swapping the disks;
* the volume 2 pi A^2 h + pi^2 A h^2 + 4/3 pi h^3 against Monte Carlo;
* a whole migration pass replayed particle by particle with all-pairs
  decisions from the independent distance (trials from rocRAND's words), an
  oracle run checked overlap-free, and the soft-shell pair list.
"""
import math

import numpy as np
import pytest

import srm_inputs
from tests import disk_ref
from tests.test_oracle_platelets import _minimg_ld, _trial_ld


def _unit(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def test_decisions_match_independent_distance(oracle_lib):
    rng = np.random.default_rng(21)
    near = 0
    for _ in range(500):
        d = rng.uniform(-2.1, 2.1, 3)
        n1, n2 = _unit(rng), _unit(rng)
        A1, A2 = rng.uniform(0.6, 1.0, 2)
        dist = disk_ref.core_distance(d, n1, A1, n2, A2)
        if dist == 0.0:
            assert oracle_lib.sd_within(d, n1, A1, n2, A2, 1e-3)
            continue
        if dist > 0.6:
            continue
        near += 1
        # the oracle counts a distance within 1e-12 (A1 + A2) of the bound as
        # overlap; step outside that band
        eps = max(1e-9 * dist, 1e-11 * (A1 + A2))
        assert not oracle_lib.sd_within(d, n1, A1, n2, A2, dist - eps), (d, dist)
        assert oracle_lib.sd_within(d, n1, A1, n2, A2, dist + eps), (d, dist)
    assert near > 80


def _check_closed_form(oracle_lib, d, n1, A1, n2, A2, dist):
    assert oracle_lib.sd_within(d, n1, A1, n2, A2, dist * (1 + 1e-9))
    assert not oracle_lib.sd_within(d, n1, A1, n2, A2, dist * (1 - 1e-9))


def test_closed_form_configurations(oracle_lib):
    rng = np.random.default_rng(22)
    for _ in range(40):
        n = _unit(rng)
        e = np.cross(n, _unit(rng))
        e /= np.linalg.norm(e)
        A1, A2 = rng.uniform(0.3, 1.0, 2)
        # coplanar, apart: the gap between the circles along the centre line
        r = (A1 + A2) * rng.uniform(1.01, 1.5)
        _check_closed_form(oracle_lib, r * e, n, A1, n, A2, r - A1 - A2)
        # stacked parallel, projections overlapping: the plane gap
        h = rng.uniform(0.01, 0.5) * rng.choice([-1.0, 1.0])
        lat = (A1 + A2) * rng.uniform(0.0, 0.95)
        _check_closed_form(oracle_lib, h * n + lat * e, n, A1, -n, A2, abs(h))
        # parallel, projections apart: plane gap and lateral gap
        lat = (A1 + A2) * rng.uniform(1.05, 1.4)
        _check_closed_form(oracle_lib, h * n + lat * e, n, A1, n, A2,
                           math.hypot(h, lat - A1 - A2))
    z = np.array([0.0, 0.0, 1.0])
    for A1, A2, z0 in ((1.0, 0.5, 0.62), (0.7, 0.7, 0.75), (0.4, 0.9, 1.3)):
        # disk 2 stands upright above the centre of disk 1: its lowest rim
        # point faces disk 1's face
        _check_closed_form(oracle_lib, np.array([0.0, 0.0, z0]), z, A1,
                           np.array([1.0, 0.0, 0.0]), A2, z0 - A2)
        # T junction in one plane: rim against rim along x
        x0 = A1 + A2 + 0.3 * z0
        _check_closed_form(oracle_lib, np.array([x0, 0.0, 0.0]), z, A1,
                           np.array([0.0, 1.0, 0.0]), A2, x0 - A1 - A2)


def test_zero_thickness_limit_and_symmetry(oracle_lib):
    rng = np.random.default_rng(23)
    asym = 0
    for _ in range(2000):
        d = rng.uniform(-2.0, 2.0, 3)
        n1, n2 = _unit(rng), _unit(rng)
        meet, margin = disk_ref.chords_meet(d, n1, 1.0, n2, 1.0)
        if margin < 1e-9:
            continue
        assert oracle_lib.sd_within(d, n1, 1.0, n2, 1.0, 1e-14) == meet
    for _ in range(300):
        d = rng.uniform(-2.0, 2.0, 3)
        n1, n2 = _unit(rng), _unit(rng)
        T = rng.uniform(0.0, 0.3)
        ab = oracle_lib.sd_within(d, n1, 0.9, n2, 0.8, T)
        ba = oracle_lib.sd_within(-d, n2, 0.8, n1, 0.9, T)
        if ab != ba:
            dist = disk_ref.core_distance(d, n1, 0.9, n2, 0.8)
            assert abs(dist - T) < 1e-11  # only rounding-level ties may differ
            asym += 1
    assert asym == 0


@pytest.mark.parametrize("thick", [0.005, 0.05, 0.3])
def test_spherodisk_volume_against_monte_carlo(oracle_lib, thick):
    a = 1.0
    h = thick * a
    A = a - h
    v = srm_inputs.spherodisk_volume_coeff(thick) * a ** 3
    assert v == pytest.approx(2 * math.pi * A * A * h + math.pi ** 2 * A * h * h
                              + 4 / 3 * math.pi * h ** 3, rel=1e-15)
    rng = np.random.default_rng(24)
    m = 2_000_000
    pts = rng.uniform([-a, -a, -h], [a, a, h], (m, 3))  # the bounding box
    foot = np.hypot(pts[:, 0], pts[:, 1])
    out = np.maximum(foot - A, 0.0)
    inside = pts[:, 2] ** 2 + out ** 2 <= h * h
    box = (2 * a) ** 2 * 2 * h
    p = inside.mean()
    assert abs(p * box - v) < 5 * math.sqrt(p * (1 - p) / m) * box
    # the oracle's fraction at scale s uses the same volume
    w = srm_inputs.make("spherodisks", n=50, seed=3, aspect_ratio=1.0 / thick,
                        f_target=0.01)
    o = oracle_lib.Oracle.from_workload(w)
    assert o.fraction(0.2) == pytest.approx(50 * srm_inputs.spherodisk_volume_coeff(thick)
                                            * 0.2 ** 3, rel=1e-13)


def _spherodisks(oracle_lib, n, seed, ar, f, cap_deg=None, c_w=0.01):
    w = srm_inputs.make("spherodisks", n=n, seed=seed, aspect_ratio=ar, f_target=f,
                        cap_deg=cap_deg, c_w=c_w)
    return w, oracle_lib.Oracle.from_workload(w)


def _hits_ref(d, n1, n2, a, tau):
    """Independent overlap decision of two equal spherodisks (outer radius
    a) and the distance of the deciding quantity from its boundary."""
    h = tau * a
    A = a - h
    T = 2 * h
    if float(np.dot(d, d)) > (2 * a) ** 2 * (1 + 1e-9):
        return False, math.inf
    meet, mg = disk_ref.chords_meet(d, n1, A, n2, A)
    if meet:
        return True, mg
    _hits_ref.distance_calls += 1
    # a separating plane normal to either disk: cheap and exact
    for n, m in ((n1, n2), (n2, n1)):
        lb = abs(float(np.dot(d, n))) - A * float(np.linalg.norm(np.cross(n, m)))
        if lb > T * (1 + 1e-6):
            return False, lb - T
    dist = disk_ref.core_distance(d, n1, A, n2, A)
    _hits_ref.shell_hits += dist <= T  # cores apart, shells in contact
    return dist <= T, abs(dist - T)


_hits_ref.distance_calls = 0
_hits_ref.shell_hits = 0


def _replay_pass(o, na, inv, s, kind, k, tau):
    p = o.params
    rows = o.pos.astype(np.longdouble)
    nrm = o.nrm.astype(np.longdouble)
    cell = o.bin(na, inv)
    ci = np.stack([cell % na[0], (cell // na[0]) % na[1], cell // (na[0] * na[1])], 1)
    colour = np.zeros(o.n, dtype=np.int64)
    for a in range(3):
        if na[a] >= 4:
            colour |= (ci[:, a] & 1) << a
    order = np.lexsort((np.arange(o.n), cell, colour))
    acc = np.zeros(o.n, dtype=np.uint8)
    margin = math.inf
    for i in order:
        old, nold = rows[i].copy(), nrm[i].copy()
        for l in range(1, p.n_l + 1):
            y, ny = _trial_ld(o, i, kind, k, l, old, nold)
            d = np.stack([_minimg_ld(rows[:, a] - y[a], p.box[a]) for a in range(3)], 1)
            dd = np.sum(d * d, axis=1).astype(np.float64)
            hit = False
            for j in np.nonzero(dd <= (2 * s) ** 2 * (1 + 1e-9))[0]:
                if j == i:
                    continue
                # lower id as disk 1: d points from disk 1 to disk 2
                if i < j:
                    h_, mg = _hits_ref(d[j].astype(np.float64), ny.astype(np.float64),
                                       nrm[j].astype(np.float64), s, tau)
                else:
                    h_, mg = _hits_ref(-d[j].astype(np.float64), nrm[j].astype(np.float64),
                                       ny.astype(np.float64), s, tau)
                margin = min(margin, mg)
                if h_:
                    hit = True
                    break
            if not hit:
                rows[i], nrm[i] = y, ny
                acc[i] = l
                break
    return rows, nrm, acc, margin


@pytest.mark.parametrize("ar,seed,swell", [(10.0, 31, 0.0), (10.0, 32, 0.03), (100.0, 33, 0.03)])
def test_spherodisk_pass_equals_allpairs_replay(oracle_lib, ar, seed, swell):
    """Thick (aspect ratio 10) and thin (100) spherodisks at number density
    about 2.5, at their target scale or swollen as in a sweep's first pass."""
    tau = 1.0 / ar  # h / a = t / D
    v = srm_inputs.spherodisk_volume_coeff(tau)
    n = 120
    f = n * v * (2.5 / n) / 8.0  # number density N D^3 = 2.5 in the unit box
    w, o = _spherodisks(oracle_lib, n, seed, ar, f)
    rc, _, _ = o.run(2000)
    assert rc == 0
    o.t = 555
    s = o.s * (1.0 + swell)
    na, inv = o.grid(s)
    _hits_ref.shell_hits = 0
    rows, nrm, ref_acc, margin = _replay_pass(o, na, inv, s, 0, 3, tau)
    if ar <= 10.0:
        assert _hits_ref.shell_hits > 0  # the thickness decided some trials
    acc, _ = o.pass_(na, inv, s, 0, 3)
    assert margin > 1e-9 * s  # no decision near a tie
    assert np.array_equal(acc, ref_acc)
    assert (acc > 1).sum() > 3 or (acc == 0).sum() > 0  # rejections happened
    assert np.allclose(o.pos, rows.astype(np.float64), rtol=0, atol=8e-16)
    assert np.allclose(o.nrm, nrm.astype(np.float64), rtol=0, atol=2e-15)


def test_spherodisk_run_is_overlap_free_and_pairs_match(oracle_lib):
    ar = 8.0
    tau = 1.0 / ar
    n = 250
    f = n * srm_inputs.spherodisk_volume_coeff(tau) * (2.0 / n) / 8.0  # N D^3 = 2
    w, o = _spherodisks(oracle_lib, n, 41, ar, f, c_w=0.02)
    rc, _, _ = o.run(2000)
    assert rc == 0 and o.s == w.s_target
    a = o.s
    gap = 0.3 * a
    ref_pairs, checked = set(), 0
    for i in range(o.n - 1):
        d = o.pos[i + 1:] - o.pos[i]
        d -= np.rint(d)
        for j in np.nonzero(np.sum(d * d, axis=1) <= (2 * a + gap) ** 2)[0]:
            dist = disk_ref.core_distance(d[j], o.nrm[i], a - tau * a, o.nrm[i + 1 + j],
                                          a - tau * a)
            assert dist > 2 * tau * a * (1 - 1e-9), (i, i + 1 + j)  # no overlap
            checked += 1
            if dist <= 2 * tau * a + gap:
                assert abs(dist - (2 * tau * a + gap)) > 1e-10
                ref_pairs.add((i, i + 1 + j))
    assert checked > 100
    got = {tuple(map(int, p)) for p in o.pairs_brute(gap)}
    assert got == ref_pairs and len(got) > 20
