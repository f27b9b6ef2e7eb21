"""Pins of the CPU oracle against facts fixed outside it.

* Philox4x32-10 against rocRAND's independent implementation (bitwise).
* Unit vectors: norm, isotropy, acceptance rate, and the direction computed
  in long double from rocRAND's words at the first accepted attempt.
* Cell size and binning against their definitions and the completeness
  requirement (every overlapping pair lies in neighbouring cells).
* A migration pass replayed particle by particle with all-pairs brute-force
  collision tests (no cell list) must give the same positions and accept
  codes bit for bit.
* Special cases: c_m = 0 and N_l = 0 make a pass the identity; N = 1 always
  accepts the first trial; shakes keep admissible states admissible.
* A full 2D run (N=2000, f=0.5) ends at the closed-form volume fraction with
  no overlapping pair under all-pairs enumeration.
"""
import math

import numpy as np
import pytest

import srm_inputs
from tests import brute, rocrand_ref



def test_philox4x32_matches_rocrand(oracle_lib):
    rng = np.random.default_rng(7)
    n = 300
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0], key[0] = 0, 0
    ctr[1], key[1] = 0xFFFFFFFF, 0xFFFFFFFF
    ref = rocrand_ref.philox4x32(ctr, key)
    for i in range(n):
        assert np.array_equal(oracle_lib.philox4x32(ctr[i], key[i]), ref[i]), i


def _ref_direction(dim, seed, pid, t, kind, k, l, stream):
    """First accepted attempt from rocRAND words, in long double: the unit
    vector (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1-2s) or (v1, v2)/sqrt(s)."""
    for r in range(64):
        ctr = np.array([[pid, t, (kind << 31) | (k << 16) | (l << 8) | r, stream]],
                       dtype=np.uint64).astype(np.uint32)
        key = np.array([[seed & 0xFFFFFFFF, seed >> 32]], dtype=np.uint64).astype(np.uint32)
        W = rocrand_ref.philox4x32(ctr, key)[0].astype(np.longdouble)
        for a in range(2):
            v1 = (W[2 * a] - np.longdouble(2147483647.5)) / np.longdouble(2**31)
            v2 = (W[2 * a + 1] - np.longdouble(2147483647.5)) / np.longdouble(2**31)
            s = v1 * v1 + v2 * v2
            if s < 1:
                if dim == 3:
                    h = 2 * np.sqrt(1 - s)
                    return np.array([v1 * h, v2 * h, 1 - 2 * s]), r + 1
                return np.array([v1, v2]) / np.sqrt(s), r + 1
    return None, 65


@pytest.mark.parametrize("dim", [2, 3])
def test_unitvec_direction_and_norm(oracle_lib, dim):
    c_m = 3.7e-4
    for pid in range(300):
        v, rounds = oracle_lib.unitvec(dim, 11, pid, 5, 0, 2, 3, 0, c_m)
        u, r_ref = _ref_direction(dim, 11, pid, 5, 0, 2, 3, 0)
        assert rounds == r_ref
        norm = math.sqrt(float(np.sum(v[:dim].astype(np.longdouble) ** 2)))
        assert abs(norm / c_m - 1.0) < 4e-16 * 4
        assert np.allclose(v[:dim] / c_m, u.astype(np.float64), rtol=0, atol=4e-16 * 4)
        if dim == 2:
            assert v[2] == 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_unitvec_isotropic(oracle_lib, dim):
    n = 20000
    vs = np.array([oracle_lib.unitvec(dim, 3, i, 0, 1, 1, 1, 0, 1.0)[0][:dim] for i in range(n)])
    # mean 0, second moments I/d: 5-sigma bounds
    assert np.all(np.abs(vs.mean(axis=0)) < 5 * math.sqrt(1.0 / dim / n))
    cov = vs.T @ vs / n
    assert np.allclose(np.diag(cov), 1.0 / dim, atol=5 * math.sqrt(2.0 / n) / dim)
    off = cov[~np.eye(dim, dtype=bool)]
    assert np.all(np.abs(off) < 5 * math.sqrt(1.0 / n) / dim)
    # acceptance: two attempts per Philox call, each kept with probability
    # pi/4, so a call succeeds with p = 1 - (1 - pi/4)^2
    rounds = np.array([oracle_lib.unitvec(dim, 3, i, 0, 1, 1, 1, 0, 1.0)[1] for i in range(n)])
    p = 1.0 - (1.0 - math.pi / 4) ** 2
    assert abs(rounds.mean() - 1.0 / p) < 5 * math.sqrt((1 - p) / p**2 / n)


def test_unitvec_streams_and_counters_distinct(oracle_lib):
    seen = set()
    for kind in (0, 1):
        for k in (1, 2):
            for l in (1, 2):
                for stream in (0, 1):
                    v, _ = oracle_lib.unitvec(3, 1, 9, 4, kind, k, l, stream, 1.0)
                    seen.add(tuple(v))
    assert len(seen) == 16


def _mk(dim, n, seed, f=0.3, **kw):
    return srm_inputs.make("disks2d" if dim == 2 else "spheres3d", n=n, seed=seed, f_target=f,
                           **kw)


def test_grid_definition(oracle_lib):
    w = _mk(2, 2000, 0, 0.5)
    o = oracle_lib.Oracle.from_workload(w)
    for s in [0.0, 1e-5, w.s_target * 0.37, w.s_target]:
        na, inv = o.grid(s)
        cs = 2.5 * s + 2.5 * w.c_m
        for a in range(2):
            assert na[a] == 1 or (na[a] >= 4 and na[a] % 2 == 0)
            assert na[a] ** 2 <= w.n
            if na[a] > 1:
                assert 1.0 / na[a] >= cs
            assert inv[a] == na[a] / 1.0
        assert na[2] == 1
    na, _ = o.grid(w.s_target)
    # 2.5 * (s_t + c_m) = 0.02453...: floor(1/cs) = 40
    assert tuple(na[:2]) == (40, 40)
    # tiny radius: capped at the largest even m with m^2 <= 2000
    na, _ = o.grid(0.0)
    assert tuple(na[:2]) == (44, 44)


@pytest.mark.parametrize("dim", [2, 3])
def test_binning_definition(oracle_lib, dim):
    w = _mk(dim, 5000, 4)
    o = oracle_lib.Oracle.from_workload(w)
    na, inv = o.grid(w.s_target)
    cell = o.bin(na, inv)
    rows = o.pos
    c = np.empty((w.n, 3), dtype=np.int64)
    c[:, 0] = cell % na[0]
    c[:, 1] = (cell // na[0]) % na[1]
    c[:, 2] = cell // (na[0] * na[1])
    for a in range(dim):
        lo = c[:, a] / na[a]
        hi = (c[:, a] + 1) / na[a]
        x = rows[:, a]
        ok = ((x >= lo - 1e-15) & (x < hi + 1e-15)) | ((c[:, a] == 0) & (x >= 1 - 1e-15))
        assert ok.all()


@pytest.mark.parametrize("dim", [2, 3])
def test_cells_complete_for_overlaps(oracle_lib, dim):
    """Particles within R_i + R_j + 2 c_m of each other are binned into
    neighbouring cells (the slack the migration pass needs)."""
    w = _mk(dim, 4000, 5, f=0.5 if dim == 2 else 0.35)
    o = oracle_lib.Oracle.from_workload(w)
    s = w.s_target
    na, inv = o.grid(s)
    cell = o.bin(na, inv)
    radii = np.full(w.n, s)
    pairs = brute.overlapping_pairs(o.pos, radii, w.box, dim, gap=2.0 * w.c_m)
    assert len(pairs) > 100
    ci = np.stack([cell % na[0], (cell // na[0]) % na[1], cell // (na[0] * na[1])], 1)
    for i, j in pairs:
        for a in range(dim):
            d = abs(int(ci[i, a]) - int(ci[j, a]))
            assert min(d, na[a] - d) <= 1


def _replay_pass(o, na, inv, s, kind, k):
    """Sequential replay of one pass with all-pairs collision tests."""
    p = o.params
    dim = p.dim
    rows = o.pos.copy()
    cell = o.bin(na, inv)
    ci = np.stack([cell % na[0], (cell // na[0]) % na[1], cell // (na[0] * na[1])], 1)
    colour = np.zeros(o.n, dtype=np.int64)
    for a in range(dim):
        if na[a] >= 4:
            colour |= (ci[:, a] & 1) << a
    order = np.lexsort((np.arange(o.n), cell, colour))
    radii = np.full(o.n, s) if o.rho is None else s * o.rho
    acc = np.zeros(o.n, dtype=np.uint8)
    for i in order:
        old = rows[i].copy()
        for l in range(1, p.n_l + 1):
            v, _ = _unit(o, i, kind, k, l)
            y = old.copy()
            for a in range(dim):
                y[a] = old[a] + v[a]
                if y[a] < 0.0:
                    y[a] += p.box[a]
                if y[a] >= p.box[a]:
                    y[a] -= p.box[a]
            if not brute.colliding(rows, radii, i, y, p.box, dim):
                rows[i] = y
                acc[i] = l
                break
    return rows, acc


def _unit(o, i, kind, k, l):
    import oracle
    return oracle.unitvec(o.dim, o.params.seed, int(i), o.t, kind, k, l, 0, o.params.c_m)


@pytest.mark.parametrize("dim,n,f,cw_mult,box", [(2, 300, 0.45, 1.0, (1.0, 1.0)),
                                                 (3, 300, 0.3, 1.0, (1.0, 1.0, 1.0)),
                                                 (2, 12, 0.3, 1.0, (1.0, 1.0)),
                                                 (3, 700, 0.4, 3.0, (1.0, 1.0, 1.0)),
                                                 (2, 400, 0.45, 1.0, (1.0, 0.55)),
                                                 (3, 600, 0.35, 1.0, (0.8, 1.0, 1.4))])
def test_pass_equals_bruteforce_replay(oracle_lib, dim, n, f, cw_mult, box):
    """One pass replayed particle by particle in the schedule order with
    all-pairs tests, in square and in stretched boxes."""
    w = _mk(dim, n, 21 + dim, f=f, c_w=0.01 * cw_mult, box=box)
    o = oracle_lib.Oracle.from_workload(w)
    # bring it to a dense, admissible state first
    rc, _, _ = o.run(2000)
    assert rc == 0
    o.t = 12345
    s = o.s
    na, inv = o.grid(s)
    ref_rows, ref_acc = _replay_pass(o, na, inv, s, 0, 3)
    acc, ov = o.pass_(na, inv, s, 0, 3)
    assert np.array_equal(acc, ref_acc)
    assert np.array_equal(o.pos, ref_rows)
    assert (acc == 0).sum() < n  # something moved
    radii = np.full(n, s)
    assert ov == brute.any_overlap(o.pos, radii, w.box, dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_pass_after_swell_replay(oracle_lib, dim):
    """The same replay on a swollen (overlapping) start, as in a sweep's
    first pass."""
    w = _mk(dim, 400, 31, f=0.4)
    o = oracle_lib.Oracle.from_workload(w, c_w=0.05)
    for _ in range(12):
        o.sweep()
    s1 = min(o.s + 0.2 * w.s_target, w.s_target)
    na, inv = o.grid(s1)
    ref_rows, ref_acc = _replay_pass(o, na, inv, s1, 0, 1)
    acc, ov = o.pass_(na, inv, s1, 0, 1)
    assert np.array_equal(acc, ref_acc) and np.array_equal(o.pos, ref_rows)


def test_fused_check_equals_full_check(oracle_lib):
    """After a pass, some pair overlaps iff some particle that rejected all
    its trials overlaps another particle (the GPU's reduced global check)."""
    hits = 0
    for seed in range(40):
        w = _mk(2, 250, 100 + seed, f=0.5, c_w=0.2, n_l=3)
        o = oracle_lib.Oracle.from_workload(w)
        o.run(3)
        s1 = min(o.s + 0.1 * w.s_target, w.s_target)
        na, inv = o.grid(s1)
        acc, ov = o.pass_(na, inv, s1, 0, 1)
        radii = np.full(w.n, s1)
        full = brute.any_overlap(o.pos, radii, w.box, 2)
        failed = np.nonzero(acc == 0)[0]
        reduced = any(brute.colliding(o.pos, radii, i, o.pos[i], w.box, 2) for i in failed)
        assert full == reduced == ov
        hits += full
    assert 0 < hits < 40


@pytest.mark.parametrize("dim", [2, 3])
def test_pass_special_cases(oracle_lib, dim):
    w = _mk(dim, 500, 8, f=0.3)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(1000)
    s = o.s
    na, inv = o.grid(s)
    before = o.pos.copy()
    # N_l = 0: no trial at all
    o.params.n_l = 0
    o.st.p = o.params
    acc, ov = o.pass_(na, inv, s, 0, 1)
    assert np.array_equal(o.pos, before) and not acc.any() and not ov
    # c_m = 0: every trial is the old position, accepted at l = 1
    o.params.n_l = 8
    o.params.c_m = 0.0
    o.st.p = o.params
    acc, ov = o.pass_(na, inv, s, 0, 1)
    assert np.array_equal(o.pos, before) and (acc == 1).all() and not ov


def test_single_particle_moves_by_first_trial(oracle_lib):
    for dim in (2, 3):
        pos = np.full((dim, 1), 0.999) if dim == 2 else np.array([[0.0005], [0.5], [0.999]])
        o = oracle_lib.Oracle(dim=dim, n=1, s_target=0.1, c_w=0.01, c_m=0.003, n_k=8, n_l=8,
                              seed=77, pos=pos, sweep0=9)
        u, _ = _ref_direction(dim, 77, 0, 9, 0, 1, 1, 0)
        u = u.astype(np.float64)
        info, acc = o.sweep()
        assert info["committed"] and info["passes_main"] == 1 and acc[0] == 1
        for a in range(dim):
            y = pos[a, 0] + 0.003 * u[a]
            y = y + 1.0 if y < 0 else (y - 1.0 if y >= 1.0 else y)
            assert abs(o.pos[0, a] - y) < 1e-15
        assert o.t == 10 and o.s == 0.001


def test_shake_branch_and_counters(oracle_lib):
    """N_l = 0 cannot resolve the overlaps a big swelling step makes: the
    sweep shakes (with zero trials), keeps P and s, and advances t."""
    w = _mk(2, 400, 9, f=0.5)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(50)
    assert o.s == pytest.approx(0.5 * w.s_target)
    s_half = o.s
    o.params.c_w = 0.5
    o.params.n_l = 0
    o.st.p = o.params
    before = o.pos.copy()
    t0 = o.t
    info, _ = o.sweep()
    assert not info["committed"] and info["passes_main"] == 8 and info["passes_shake"] == 8
    assert np.array_equal(o.pos, before) and o.s == s_half and o.t == t0 + 1


def test_shake_keeps_admissible(oracle_lib):
    w = _mk(3, 600, 10, f=0.35)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(1000)
    radii = np.full(w.n, o.s)
    na, inv = o.grid(o.s)
    for j in range(1, 4):
        o.pass_(na, inv, o.s, 1, j)
        assert not brute.any_overlap(o.pos, radii, w.box, 3)


def test_swell_closed_form(oracle_lib):
    w = _mk(2, 100, 1, f=0.5)
    o = oracle_lib.Oracle.from_workload(w)
    s = 0.0
    for _ in range(150):
        s1 = o.swell(s)
        assert s1 == min(s + w.c_w * w.s_target, w.s_target)
        s = s1
    assert s == w.s_target


def test_config1_full_run(oracle_lib):
    """2D, N=2000, f=0.5, seed 0: converges, zero overlaps (all pairs), and
    the volume fraction at s_target is the target to a few ulps."""
    w = srm_inputs.make("disks2d")
    o = oracle_lib.Oracle.from_workload(w)
    rc, sweeps, passes = o.run(1000)
    assert rc == 0 and o.s == w.s_target and sweeps >= 100
    radii = np.full(w.n, o.s)
    assert not brute.any_overlap(o.pos, radii, w.box, 2)
    f = math.pi * w.n * o.s * o.s
    assert abs(f - 0.5) <= 4 * np.spacing(0.5)
    assert np.all((o.pos[:, :2] >= 0) & (o.pos[:, :2] < 1))


def test_max_sweeps_not_converged(oracle_lib):
    w = _mk(2, 300, 12, f=0.5)
    o = oracle_lib.Oracle.from_workload(w)
    rc, sweeps, _ = o.run(5)
    assert rc == oracle_lib.ENOTCONV and sweeps == 5


def test_sweep_deterministic_and_resumable(oracle_lib):
    w = _mk(3, 800, 13, f=0.3)
    a = oracle_lib.Oracle.from_workload(w)
    for _ in range(30):
        a.sweep()
    b = oracle_lib.Oracle.from_workload(w)
    for _ in range(17):
        b.sweep()
    # resume from a saved state: positions, s and t are the whole state
    c = oracle_lib.Oracle.from_workload(w, pos=b.soa(), s0=b.s, sweep0=b.t)
    for _ in range(13):
        c.sweep()
    assert np.array_equal(a.pos, c.pos) and a.s == c.s and a.t == c.t


def test_polydisperse_run_admissible(oracle_lib):
    w = _mk(3, 1500, 14, f=0.4, polydisperse_sigma=0.2)
    o = oracle_lib.Oracle.from_workload(w)
    rc, _, _ = o.run(2000)
    assert rc == 0
    radii = o.s * o.rho
    assert not brute.any_overlap(o.pos, radii, w.box, 3)
    f = 4.0 / 3.0 * math.pi * float(np.sum(radii ** 3))
    assert abs(f - 0.4) < 1e-14


def test_staged_run_stops_at_the_given_scale(oracle_lib):
    """A run with an intermediate stop scale ends exactly there with no
    overlapping pair (all pairs), having swollen by c_w s_target per
    committed sweep; continuing runs on to s_target."""
    w = _mk(2, 600, 41, f=0.5)
    o = oracle_lib.Oracle.from_workload(w, c_w=0.03)
    stop = 0.62 * w.s_target
    rc, sweeps, passes = o.run(2000, s_stop=stop)
    assert rc == 0 and o.s == stop and sweeps >= math.ceil(0.62 / 0.03)
    assert not brute.any_overlap(o.pos, np.full(o.n, o.s), w.box, 2)
    rc, _, _ = o.run(2000)
    assert rc == 0 and o.s == w.s_target
    assert not brute.any_overlap(o.pos, np.full(o.n, o.s), w.box, 2)
