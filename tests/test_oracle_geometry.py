"""Pins of the oracle's pair enumeration, distance histogram and the thin
platelet (zero-thickness disk) intersection test."""
import math

import numpy as np
import pytest

import srm_inputs
from tests import brute, disk_ref


def _state(oracle_lib, dim, n, seed, f):
    w = srm_inputs.make("disks2d" if dim == 2 else "spheres3d", n=n, seed=seed, f_target=f)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(2000)
    return w, o


@pytest.mark.parametrize("dim", [2, 3])
def test_pairs_match_numpy_enumeration(oracle_lib, dim):
    w, o = _state(oracle_lib, dim, 1500, 40 + dim, 0.35)
    for gap in (0.0, 0.3 * o.s, 2.0 * o.s):
        got = o.pairs_brute(gap)
        ref = brute.overlapping_pairs(o.pos, np.full(w.n, o.s), w.box, dim, gap)
        assert np.array_equal(got, ref)
    assert len(o.pairs_brute(0.0)) == 0  # admissible end state


@pytest.mark.parametrize("dim", [2, 3])
def test_rdf_counts_match_numpy(oracle_lib, dim):
    w, o = _state(oracle_lib, dim, 1200, 50 + dim, 0.3)
    nbins, r_max = 64, 5.0 * o.s
    got = o.rdf_brute(nbins, r_max)
    n = w.n
    ref = np.zeros(nbins, dtype=np.int64)
    inv = nbins / r_max
    for i in range(n - 1):
        q = brute.q_to_all(o.pos[i + 1:], o.pos[i], w.box, dim)
        x = np.sqrt(q) * inv
        b = x[x < nbins].astype(np.int64)
        ref += np.bincount(b, minlength=nbins)
    assert np.array_equal(got.astype(np.int64), ref)
    # no pair closer than a diameter in an admissible hard-sphere state
    assert got[: int(2.0 * o.s * inv) - 1].sum() == 0


def test_rdf_and_pairs_translation_invariant_on_dyadic_grid(oracle_lib):
    """Positions on a 2^-30 grid, shifted by a multiple of 2^-30 with wrap:
    differences and squared sums are exact, so counts and pair sets agree
    bit for bit."""
    rng = np.random.default_rng(3)
    n, dim = 800, 3
    pos = rng.integers(0, 2**30, size=(dim, n)).astype(np.float64) * 2.0**-30
    s = 0.02
    base = oracle_lib.Oracle(dim=dim, n=n, s_target=s, c_w=0.0, c_m=0.0, n_k=1, n_l=1, seed=0,
                             pos=pos, s0=s)
    shift = rng.integers(0, 2**30, size=(dim, 1)).astype(np.float64) * 2.0**-30
    moved = pos + shift
    moved[moved >= 1.0] -= 1.0
    other = oracle_lib.Oracle(dim=dim, n=n, s_target=s, c_w=0.0, c_m=0.0, n_k=1, n_l=1, seed=0,
                              pos=moved, s0=s)
    assert np.array_equal(base.pairs_brute(0.01), other.pairs_brute(0.01))
    assert np.array_equal(base.rdf_brute(32, 0.2), other.rdf_brute(32, 0.2))
    assert len(base.pairs_brute(0.01)) > 0


# ---------------------------------------------------------------- platelets

def _rand_unit(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def test_disks_coplanar_reduce_to_circle_test(oracle_lib):
    """Both normals +z, centres in one plane: intersect iff |d| <= a1 + a2."""
    for d in [0.0, 0.5, 0.999, 1.0, 1.001, 1.5]:
        c1 = np.array([0.5, 0.5, 0.5])
        c2 = c1 + np.array([d * 0.6, d * 0.8, 0.0]) * 0.25
        nz = np.array([0.0, 0.0, 1.0])
        got = oracle_lib.disks_intersect(c1, nz, 0.1, c2, nz, 0.15)
        dist = math.hypot((c2 - c1)[0], (c2 - c1)[1])
        assert got == (dist <= 0.25)
    # parallel but not coplanar: never
    c2 = np.array([0.5, 0.5, 0.5 + 1e-6])
    assert not oracle_lib.disks_intersect(c1, nz, 0.1, c2, nz, 0.1)


def test_disks_perpendicular_analytic(oracle_lib):
    """Disk 1 in the plane z=0 (normal z), disk 2 in the plane x=0 (normal x)
    through the point (0, 0, h): disk 2 meets z=0 in the chord |y - y2| <=
    sqrt(a2^2 - h^2) on x=0; disk 1 covers |y| <= a1 there."""
    a1, a2 = 0.1, 0.08
    base = np.array([0.5, 0.5, 0.5])
    for h in [0.0, 0.03, 0.079, 0.081]:
        for y2 in [0.0, 0.1, 0.15, 0.16, 0.2]:
            c2 = base + np.array([0.0, y2, h])
            got = oracle_lib.disks_intersect(base, np.array([0, 0, 1.0]), a1, c2,
                                             np.array([1.0, 0, 0]), a2)
            if h > a2:
                expect = False
            else:
                half = math.sqrt(a2 * a2 - h * h)
                expect = abs(y2) <= a1 + half
            margin = abs(abs(y2) - (a1 + math.sqrt(max(a2 * a2 - h * h, 0.0))))
            if margin > 1e-9 and abs(h - a2) > 1e-9:
                assert got == expect, (h, y2)


def test_disks_random_against_independent_formulation(oracle_lib):
    rng = np.random.default_rng(11)
    checked = hits = 0
    for _ in range(20000):
        c1 = rng.uniform(0.3, 0.7, 3)
        c2 = c1 + rng.uniform(-0.2, 0.2, 3)
        n1, n2 = _rand_unit(rng), _rand_unit(rng)
        a1, a2 = rng.uniform(0.02, 0.15, 2)
        got = oracle_lib.disks_intersect(c1, n1, a1, c2, n2, a2)
        if np.linalg.norm(c2 - c1) > a1 + a2:
            assert not got
            continue
        ref, margin = disk_ref.chords_overlap_ref(c1, n1, a1, c2, n2, a2)
        if margin < 1e-9:
            continue
        assert got == ref
        checked += 1
        hits += ref
    assert checked > 3000 and 0.1 * checked < hits < 0.9 * checked


def test_disks_dense_sampling(oracle_lib):
    """Tiny cases: sample disk 1 densely; a sample point lying (within a
    tolerance) in plane 2 inside disk 2 proves intersection."""
    rng = np.random.default_rng(5)
    agree = 0
    for _ in range(300):
        c1 = np.array([0.5, 0.5, 0.5])
        c2 = c1 + rng.uniform(-0.1, 0.1, 3)
        n1, n2 = _rand_unit(rng), _rand_unit(rng)
        a1, a2 = 0.08, 0.07
        got = oracle_lib.disks_intersect(c1, n1, a1, c2, n2, a2)
        e1 = np.cross(n1, [1.0, 0, 0] if abs(n1[0]) < 0.9 else [0, 1.0, 0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(n1, e1)
        r = np.linspace(0, a1, 200)[:, None]
        th = np.linspace(0, 2 * np.pi, 800)[None, :]
        pts = c1[None, None, :] + (r * np.cos(th))[..., None] * e1 + (r * np.sin(th))[..., None] * e2
        h = (pts - c2) @ n2
        rad = np.linalg.norm((pts - c2) - h[..., None] * n2, axis=-1)
        sampled = bool(np.any((np.abs(h) < 2e-4) & (rad <= a2)))
        clear = bool(np.all((np.abs(h) > 2e-3) | (rad > a2 + 2e-3)))
        if sampled:
            assert got
            agree += 1
        elif clear:
            assert not got
            agree += 1
    assert agree > 200


# ------------------------------------------------------ nearest neighbours

def test_nearest_on_a_lattice_and_across_the_boundary(oracle_lib):
    """A simple cubic lattice of spacing 1/8 in the unit cube: every nearest
    distance is the spacing (to rounding); two particles 0.02 apart across
    the periodic face find each other; a lone particle gets +inf."""
    m = 8
    g = (np.arange(m) + 0.5) / m
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    o = oracle_lib.Oracle(dim=3, n=pos.shape[1], s_target=0.01, c_w=0.01, c_m=0.001,
                          n_k=8, n_l=8, seed=1, pos=pos)
    d = o.nearest_brute(0.3)
    assert np.all(np.abs(d - 1.0 / m) <= 4e-16)
    pos2 = np.array([[0.99, 0.01], [0.5, 0.5], [0.5, 0.5]])
    o2 = oracle_lib.Oracle(dim=3, n=2, s_target=0.001, c_w=0.01, c_m=0.0001, n_k=8, n_l=8,
                           seed=1, pos=pos2)
    assert np.allclose(o2.nearest_brute(0.3), 0.02, rtol=0, atol=1e-15)
    assert np.all(np.isinf(o2.nearest_brute(0.01)))


@pytest.mark.parametrize("dim", [2, 3])
def test_nearest_matches_a_kd_tree(oracle_lib, dim):
    """Random points: the all-pairs nearest distances equal scipy's periodic
    k-d tree query (another algorithm and another rounding order) to 1e-14
    relative, and the cutoff turns exactly the far ones into +inf."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(11 + dim)
    n = 1500
    pos = rng.random((dim, n))
    o = oracle_lib.Oracle(dim=dim, n=n, s_target=1e-4, c_w=0.01, c_m=1e-5, n_k=8, n_l=8,
                          seed=1, pos=pos)
    r_max = 0.2
    d = o.nearest_brute(r_max)
    ref, _ = cKDTree(pos.T, boxsize=1.0).query(pos.T, k=2)
    ref = ref[:, 1]
    fin = ref < r_max * (1 - 1e-12)
    assert np.allclose(d[fin], ref[fin], rtol=1e-14, atol=0)
    assert np.all(np.isinf(d[ref > r_max * (1 + 1e-12)]))
    med = float(np.median(ref))
    d_small = o.nearest_brute(med)
    clear = np.abs(ref - med) > 1e-12 * med
    assert np.array_equal(np.isinf(d_small)[clear], (ref >= med)[clear])
    assert np.array_equal(d_small[~np.isinf(d_small)], d[~np.isinf(d_small)])


# ------------------------------------------------------------ percolation

def _balls(oracle_lib, pos, s):
    dim, n = pos.shape
    return oracle_lib.Oracle(dim=dim, n=n, s_target=s, c_w=0.01, c_m=0.1 * s, n_k=8, n_l=8,
                             seed=1, pos=pos, s0=s)


def test_percolation_of_chains_and_rings(oracle_lib):
    """A chain of balls 0.1 apart along x wraps along x once the gap closes
    the 0.02 surface gaps (0.1 - 2 * 0.04), and only along x; a lattice of
    such chains in 2D wraps along both axes; a closed ring inside the box
    never percolates."""
    x = (np.arange(10) + 0.5) / 10
    chain = np.stack([x, np.full(10, 0.3), np.full(10, 0.6)])
    o = _balls(oracle_lib, chain, 0.04)
    assert o.percolation(0.0) == 0
    assert o.percolation(0.019) == 0
    assert o.percolation(0.021) == 1
    gc = o.critical_gap(0.0, 0.05, iters=40)
    assert abs(gc - 0.02) < 1e-10
    X, Y = np.meshgrid(x, x, indexing="ij")
    grid = np.stack([X.ravel(), Y.ravel()])
    o2 = _balls(oracle_lib, grid, 0.04)
    assert o2.percolation(0.019) == 0 and o2.percolation(0.021) == 3
    t = np.linspace(0, 2 * np.pi, 24, endpoint=False)
    ring = np.stack([0.5 + 0.2 * np.cos(t), 0.5 + 0.2 * np.sin(t)])
    o3 = _balls(oracle_lib, ring, 0.02)
    assert o3.percolation(0.03) == 0  # neighbours bonded: a ring, no winding
    assert len(o3.pairs_brute(0.03)) >= 24


@pytest.mark.parametrize("dim", [2, 3])
def test_percolation_matches_a_doubled_box(oracle_lib, dim):
    """Random balls: a cluster wraps along axis a exactly when, in the box
    doubled along every axis (2^dim copies, minimum image in the doubled
    box), some particle is connected to its own copy shifted by L along a
    (scipy k-d tree bonds and connected components: another algorithm)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(21 + dim)
    n = 700 if dim == 2 else 900
    pos = rng.random((dim, n))
    r = 0.012 if dim == 2 else 0.03
    o = _balls(oracle_lib, pos, r)
    shifts = np.array(np.meshgrid(*[[0, 1]] * dim, indexing="ij")).reshape(dim, -1).T
    big = np.concatenate([pos.T + sh for sh in shifts])          # (2^dim n, dim) in [0, 2)
    tree = cKDTree(big, boxsize=2.0)
    seen = set()
    for gap in np.linspace(0.0, 3.0 * r, 13):
        pairs = tree.query_pairs(2 * r + gap, output_type="ndarray")
        m = len(big)
        adj = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(m, m))
        _, lab = connected_components(adj, directed=False)
        ref = 0
        for a in range(dim):
            img = np.nonzero(np.all(shifts == np.eye(dim, dtype=int)[a], axis=1))[0][0]
            if np.any(lab[:n] == lab[img * n: img * n + n]):
                ref |= 1 << a
        got = o.percolation(gap)
        assert got == ref, (gap, got, ref)
        seen.add(got)
    assert 0 in seen and (2 ** dim - 1) in seen   # both regimes covered


@pytest.mark.parametrize("dim,axes,eta_ref", [
    (2, 1, 1.12808737),   # disks (Mertens and Moore 2012)
    (3, 7, 0.3418174),    # spheres (Lorenz and Ziff 2001)
])
def test_soft_shells_of_points_percolate_at_the_continuum_threshold(oracle_lib, dim, axes, eta_ref):
    """With vanishing hard cores the soft shells are fully penetrable disks
    (spheres) of radius gap/2 around Poisson points, whose wrapping threshold
    is the continuum percolation threshold: reduced density
    eta = N pi r^2 (N 4/3 pi r^3) of 1.128 in 2D and 0.342 in 3D.  Bisection
    on the gap over 12 boxes of 2000 points lands within 6% (the mean sits
    ~1.7% above, two standard errors of the sampling; wrapping along x in 2D,
    along any axis in 3D, whose finite-size shifts are small)."""
    import math
    etas = []
    for seed in range(12):
        rng = np.random.default_rng(seed)
        n = 2000
        o = _balls(oracle_lib, rng.random((dim, n)), 1e-9)
        lo, hi = 0.0, (0.1 if dim == 2 else 0.3)
        assert not (o.percolation(lo) & axes) and (o.percolation(hi) & axes)
        for _ in range(24):
            mid = 0.5 * (lo + hi)
            if o.percolation(mid) & axes:
                hi = mid
            else:
                lo = mid
        r = 0.5 * (hi + 2e-9)
        etas.append(n * (math.pi * r * r if dim == 2 else 4.0 / 3.0 * math.pi * r ** 3))
    assert abs(np.mean(etas) / eta_ref - 1.0) < 0.06, (np.mean(etas), etas)


@pytest.mark.parametrize("dim", [2, 3])
def test_nearest_distances_of_poisson_points_follow_hertz(oracle_lib, dim):
    """Uniform points in the periodic unit box: the distance from a point to
    its nearest neighbour exceeds r with probability (1 - V(r))^(N-1), V the
    disk (ball) area (volume) of radius r (Hertz's distribution, exact in a
    periodic box for r below half the edge).  The empirical distribution of
    the oracle's nearest distances stays within 0.04 of it in the sup norm,
    and its mean within 3% of the distribution's."""
    import math
    n = 3000
    rng = np.random.default_rng(40 + dim)
    o = _balls(oracle_lib, rng.random((dim, n)), 1e-9)
    d = np.sort(o.nearest_brute(0.45))
    assert np.all(np.isfinite(d))
    vol = (lambda r: math.pi * r * r) if dim == 2 else (lambda r: 4.0 / 3.0 * math.pi * r ** 3)
    cdf = np.array([1.0 - (1.0 - vol(r)) ** (n - 1) for r in d])
    emp_hi = np.arange(1, n + 1) / n
    emp_lo = np.arange(0, n) / n
    assert max(np.max(np.abs(emp_hi - cdf)), np.max(np.abs(emp_lo - cdf))) < 0.04
    rs = np.linspace(0.0, 0.45, 200001)
    surv = (1.0 - np.array([vol(r) for r in rs])) ** (n - 1)
    mean = float(np.sum(0.5 * (surv[1:] + surv[:-1])) * (rs[1] - rs[0]))
    assert abs(d.mean() / mean - 1.0) < 0.03, (d.mean(), mean)


@pytest.mark.parametrize("dim", [2, 3])
def test_distance_histogram_of_poisson_points(oracle_lib, dim):
    """Uniform points in the periodic unit box: the expected number of pairs
    in the distance bin [r_b, r_b+1) is N (N - 1) / 2 times the shell area
    (volume) for r below half the edge; every bin of the oracle's histogram
    lies within 5 standard deviations of it (pair counts ~ Poisson here)."""
    import math
    n, nbins, r_max = 3000, 40, 0.2
    rng = np.random.default_rng(60 + dim)
    o = _balls(oracle_lib, rng.random((dim, n)), 1e-9)
    got = o.rdf_brute(nbins, r_max).astype(np.float64)
    edges = np.arange(nbins + 1) * (r_max / nbins)
    if dim == 2:
        shell = math.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    else:
        shell = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    expect = 0.5 * n * (n - 1) * shell
    z = (got - expect) / np.sqrt(expect)
    assert np.all(np.abs(z[2:]) < 5.0), z
    assert abs(got.sum() / expect.sum() - 1.0) < 0.01
