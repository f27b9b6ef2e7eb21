"""Pins of the oracle's thin-platelet migration (Sec. 3.3 platelets moved by
Algorithm 3, tested by the exact disk-disk predicate in Algorithm 5's place)
against facts fixed outside it.

* A platelet's trial: the centre moves by c_m times a random unit vector
  (stream 0) and the normal becomes (n + c_n w) / |n + c_n w| with w a
  second random unit vector (stream 1).  Both are rebuilt in long double
  from rocRAND's Philox words and compared with the oracle's trials.
* The angle between n and the trial normal: with w uniform on the sphere,
  u = n.w is uniform on [-1, 1] and x = n.n' = (1 + c u)/sqrt(1 + c^2 + 2cu).
  For c < 1 that gives P(x <= X) = X sqrt(X^2 - 1 + c^2) / c on
  [sqrt(1 - c^2), 1] and E[x] = 1 - c^2/3 (derived here, not taken from the
  oracle); the oracle's trial normals follow it (Kolmogorov-Smirnov).
* A whole migration pass replayed particle by particle in the schedule
  order, every trial built from rocRAND's words in long double, and every
  collision decided against all other platelets with the independent
  chord formulation of tests/disk_ref.py (no cell list): the accept codes
  match exactly, the centres and normals to a few ulp.
* The lower-id-first operand order of the disk test: rounding-level ties
  where the predicate's answer depends on operand order are searched out,
  and the oracle's global check (Algorithm 6) on two platelets must give
  the answer with the lower id as disk 1, for both id assignments.
* An oracle platelet run ends with no intersecting pair under the
  independent predicate (all pairs).
"""
import math

import numpy as np
import pytest

import srm_inputs
from tests import disk_ref
from tests.test_oracle_pins import _ref_direction


def _platelets(oracle_lib, n, seed, cap_deg=None, c_w=0.01, f=0.02):
    w = srm_inputs.make("platelets", n=n, seed=seed, cap_deg=cap_deg, c_w=c_w, f_target=f)
    return w, oracle_lib.Oracle.from_workload(w)


def _set_c_n(o, c):
    o.params.c_n = c
    o.st.p.c_n = c  # the state holds its own copy of the parameters


def _trial_ld(o, i, kind, k, l, old, nold):
    """Centre and normal of trial l of particle i from rocRAND words, long
    double: y = wrap(old + c_m u0), n' = (n + c_n u1) / |n + c_n u1|."""
    p = o.params
    u0, _ = _ref_direction(3, p.seed, int(i), o.t, kind, k, l, 0)
    u1, _ = _ref_direction(3, p.seed, int(i), o.t, kind, k, l, 1)
    y = old + np.longdouble(p.c_m) * u0
    for a in range(3):
        L = np.longdouble(p.box[a])
        if y[a] < 0:
            y[a] += L
        if y[a] >= L:
            y[a] -= L
    m = nold + np.longdouble(p.c_n) * u1
    return y, m / np.sqrt(np.dot(m, m))


def test_platelet_trial_from_rocrand_words(oracle_lib):
    """Platelets too small to meet accept their first trial: the oracle's
    new centres and normals equal the long-double trials."""
    n = 400
    w, o = _platelets(oracle_lib, n, 7)
    _set_c_n(o, 0.37)  # any step works; not the workload's 0.1
    s = 1e-7
    o.t = 4321
    old, nold = o.pos.copy(), o.nrm.copy()
    na, inv = o.grid(s)
    acc, ov = o.pass_(na, inv, s, 0, 2)
    assert (acc == 1).all() and not ov
    for i in range(n):
        y, ny = _trial_ld(o, i, 0, 2, 1, old[i].astype(np.longdouble),
                          nold[i].astype(np.longdouble))
        assert np.allclose(o.pos[i], y.astype(np.float64), rtol=0, atol=4e-16), i
        assert np.allclose(o.nrm[i], ny.astype(np.float64), rtol=0, atol=8e-16), i
        assert abs(float(np.dot(o.nrm[i], o.nrm[i])) - 1.0) < 8e-16


def _trial_normal_cdf(x, c):
    x = np.asarray(x, dtype=np.float64)
    lo = math.sqrt(1.0 - c * c)
    inside = np.clip(x, lo, 1.0)
    return np.where(x < lo, 0.0, inside * np.sqrt(np.maximum(inside * inside - lo * lo, 0.0)) / c)


@pytest.mark.parametrize("c", [0.1, 0.6])
def test_platelet_trial_normal_angle_distribution(oracle_lib, c):
    n = 20000
    w, o = _platelets(oracle_lib, n, 12)
    _set_c_n(o, c)
    s = 1e-9
    nold = o.nrm.copy()
    na, inv = o.grid(s)
    acc, _ = o.pass_(na, inv, s, 0, 1)
    assert (acc == 1).all()
    x = np.sum(nold * o.nrm, axis=1)
    assert x.min() >= math.sqrt(1 - c * c) - 1e-12 and x.max() <= 1 + 1e-15
    xs = np.sort(x)
    cdf = _trial_normal_cdf(xs, c)
    emp_hi = np.arange(1, n + 1) / n
    emp_lo = np.arange(0, n) / n
    ks = max(np.max(emp_hi - cdf), np.max(cdf - emp_lo))
    assert ks < 1.63 / math.sqrt(n)  # 1% level
    # mean over the sample against 1 - c^2/3, 5 sigma
    var = np.var(x)
    assert abs(x.mean() - (1 - c * c / 3)) < 5 * math.sqrt(var / n)


def _minimg_ld(d, L):
    L = np.longdouble(L)
    return d - L * np.rint(d / L)


def _replay_platelet_pass(o, na, inv, s, kind, k):
    """Sequential replay of one platelet pass with all-pairs tests by the
    independent chord formulation.  Returns (centres, normals, acc, the
    smallest decision margin met)."""
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
    a_r = np.longdouble(s)  # monodisperse: every disk radius is s
    acc = np.zeros(o.n, dtype=np.uint8)
    margin = math.inf
    for i in order:
        old, nold = rows[i].copy(), nrm[i].copy()
        for l in range(1, p.n_l + 1):
            y, ny = _trial_ld(o, i, kind, k, l, old, nold)
            d = np.stack([_minimg_ld(rows[:, a] - y[a], p.box[a]) for a in range(3)], 1)
            dd = np.sum(d * d, axis=1)
            near = np.nonzero(dd <= (2 * a_r) ** 2)[0]
            hit = False
            for j in near:
                if j == i:
                    continue
                meet, mg = disk_ref.chords_meet(d[j], ny, a_r, nrm[j], a_r)
                margin = min(margin, mg)
                if meet:
                    hit = True
                    break
            if not hit:
                rows[i], nrm[i] = y, ny
                acc[i] = l
                break
    return rows, nrm, acc, margin


@pytest.mark.parametrize("seed,cap,swell", [(3, None, 0.0), (4, 15.0, 0.0), (5, None, 0.04)])
def test_platelet_pass_equals_allpairs_replay(oracle_lib, seed, cap, swell):
    """A dense platelet box (number density 2.55, about 11 centres within a
    diameter), at its target radius or swollen beyond it as in a sweep's
    first pass."""
    w, o = _platelets(oracle_lib, 300, seed, cap_deg=cap)
    rc, _, _ = o.run(2000)
    assert rc == 0
    o.t = 777
    s = o.s * (1.0 + swell)
    na, inv = o.grid(s)
    rows, nrm, ref_acc, margin = _replay_platelet_pass(o, na, inv, s, 0, 2)
    acc, _ = o.pass_(na, inv, s, 0, 2)
    assert margin > 1e-12  # no decision is a rounding-level tie
    assert np.array_equal(acc, ref_acc)
    assert (acc == 0).sum() > 0 or swell == 0.0
    assert (acc > 1).sum() > 5  # rejections happened
    assert np.allclose(o.pos, rows.astype(np.float64), rtol=0, atol=8e-16)
    assert np.allclose(o.nrm, nrm.astype(np.float64), rtol=0, atol=2e-15)


def _find_ties(oracle_lib, count, seed):
    """Pairs of equal disks where the predicate's answer depends on the
    operand order: bisect a shift of disk 2 onto the decision boundary, then
    walk its x coordinate ulp by ulp."""
    f = oracle_lib.disks_intersect
    rng = np.random.default_rng(seed)
    want = {False: [], True: []}  # keyed by the answer with (c1, n1) as disk 1
    a = 0.05
    while min(len(v) for v in want.values()) < count:
        c1 = rng.uniform(0.4, 0.6, 3)
        n1 = rng.standard_normal(3)
        n1 /= np.linalg.norm(n1)
        n2 = rng.standard_normal(3)
        n2 /= np.linalg.norm(n2)
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        lo, hi = 0.0, 2 * a
        if not f(c1, n1, a, c1, n2, a) or f(c1, n1, a, c1 + hi * e, n2, a):
            continue
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            if f(c1, n1, a, c1 + mid * e, n2, a):
                lo = mid
            else:
                hi = mid
        base = c1 + lo * e
        for step in range(-40, 41):
            c2 = base.copy()
            c2[0] = base[0] + step * np.spacing(base[0])
            ab, ba = f(c1, n1, a, c2, n2, a), f(c2, n2, a, c1, n1, a)
            if ab != ba:
                want[ab].append((c1, n1, c2, n2, a))
                break
    return want[False][:count] + want[True][:count]


def test_platelet_disk_order_is_lower_id_first(oracle_lib):
    ties = _find_ties(oracle_lib, 4, 3)
    f = oracle_lib.disks_intersect
    for c1, n1, c2, n2, a in ties:
        for first, second in (((c1, n1), (c2, n2)), ((c2, n2), (c1, n1))):
            pos = np.stack([first[0], second[0]], 1)
            nrm = np.stack([first[1], second[1]], 1)
            o = oracle_lib.Oracle(dim=3, n=2, s_target=a, c_w=0.0, c_m=0.0, n_k=1, n_l=1,
                                  seed=0, pos=pos, normals=nrm, shape=1, c_n=0.0,
                                  thick_ratio=0.01, s0=a)
            expect = f(first[0], first[1], a, second[0], second[1], a)
            assert o.overlap() == expect


def test_platelet_run_has_no_intersecting_pair(oracle_lib):
    w, o = _platelets(oracle_lib, 400, 9, c_w=0.02)
    rc, _, _ = o.run(2000)
    assert rc == 0 and o.s == w.s_target
    a = o.s
    checked = 0
    for i in range(o.n - 1):
        d = o.pos[i + 1:] - o.pos[i]
        d -= np.rint(d)  # unit box
        near = np.nonzero(np.sum(d * d, axis=1) <= (2 * a) ** 2)[0]
        for j in near:
            meet, margin = disk_ref.chords_meet(d[j], o.nrm[i], a, o.nrm[i + 1 + j], a)
            assert not meet or margin < 1e-12, (i, i + 1 + j)
            checked += 1
    assert checked > 200
