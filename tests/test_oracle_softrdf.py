"""Pins of the oracle's soft-binned g(r), overlap energy and their gradient."""
import math

import numpy as np
import pytest

import srm_inputs


def _state(oracle_lib, dim, n, f, seed):
    w = srm_inputs.make("disks2d" if dim == 2 else "softrdf", n=n, seed=seed, f_target=f)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(3000)
    return o


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_central_differences(oracle_lib, dim):
    o = _state(oracle_lib, dim, 300, 0.3, 11 + dim)
    s = o.s
    pos = o.soa()
    radii = np.full(o.n, s) * 1.08  # some overlaps so the penalty is active
    rc = 5.0 * s
    kw = dict(dim=dim, nbins=64, r_c=rc)
    rng = np.random.default_rng(dim)
    dg = rng.standard_normal(64)
    dE = 0.37
    gp, gr = oracle_lib.softrdf_gradient(pos, radii, dg, dE, **kw)

    def L(p, r):
        g, e = oracle_lib.softrdf_forward(p, r, **kw)
        return float(dg @ g + dE * e)

    h = 1e-6 * s
    for a, i in [(0, 3), (1, 17), (dim - 1, 101), (0, 250)]:
        p1, p2 = pos.copy(), pos.copy()
        p1[a, i] += h
        p2[a, i] -= h
        fd = (L(p1, radii) - L(p2, radii)) / (2 * h)
        assert abs(fd - gp[a, i]) <= 1e-6 * max(1.0, abs(gp[a, i])), (a, i, fd, gp[a, i])
    for i in (5, 60):
        r1, r2 = radii.copy(), radii.copy()
        r1[i] += h
        r2[i] -= h
        fd = (L(pos, r1) - L(pos, r2)) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1.0, abs(gr[i]))
    assert np.any(gr != 0.0)


def test_poisson_points_give_unit_g(oracle_lib):
    """Uniform points: g ~ 1 away from the origin (kernel smoothing aside)."""
    rng = np.random.default_rng(4)
    n = 1500
    pos = rng.random((3, n))
    rc = 0.2
    g, e = oracle_lib.softrdf_forward(pos, np.zeros(n), dim=3, nbins=32, r_c=rc)
    assert e == 0.0
    mean = g[8:].mean()
    pairs = n * (n - 1) / 2 * (4 / 3 * math.pi * (rc**3 - (rc / 4) ** 3))
    assert abs(mean - 1.0) < 4.0 / math.sqrt(pairs) * 5, mean


def test_energy_of_one_overlapping_pair(oracle_lib):
    pos = np.array([[0.1, 0.13], [0.5, 0.5], [0.5, 0.5]])
    radii = np.array([0.02, 0.025])
    _, e = oracle_lib.softrdf_forward(pos, radii, dim=3, nbins=8, r_c=0.1, kappa=2.0)
    assert e == pytest.approx(0.5 * 2.0 * (0.045 - 0.03) ** 2, rel=1e-14)
    # across the periodic boundary
    pos = np.array([[0.005, 0.985], [0.5, 0.5], [0.5, 0.5]])
    _, e = oracle_lib.softrdf_forward(pos, radii, dim=3, nbins=8, r_c=0.1, kappa=2.0)
    assert e == pytest.approx(0.5 * 2.0 * (0.045 - 0.02) ** 2, rel=1e-12)


def test_translation_and_permutation_invariance(oracle_lib):
    o = _state(oracle_lib, 3, 400, 0.3, 21)
    pos = o.soa()
    radii = np.full(o.n, o.s)
    kw = dict(dim=3, nbins=64, r_c=5 * o.s)
    g0, e0 = oracle_lib.softrdf_forward(pos, radii, **kw)
    moved = pos + np.array([[0.31], [0.77], [0.05]])
    moved[moved >= 1.0] -= 1.0
    g1, e1 = oracle_lib.softrdf_forward(moved, radii, **kw)
    perm = np.random.default_rng(1).permutation(o.n)
    g2, e2 = oracle_lib.softrdf_forward(pos[:, perm], radii[perm], **kw)
    assert np.allclose(g0, g1, rtol=1e-12, atol=1e-12)
    assert np.allclose(g0, g2, rtol=1e-12, atol=1e-12)
    assert e0 == e1 == e2 == 0.0


def test_thomas_process_matches_its_pair_correlation(oracle_lib):
    """Points of a Thomas cluster process (Poisson parents, Poisson
    offspring displaced by N(0, sigma^2) per axis, periodic unit box).
    Given the realised cluster sizes m_c, a pair lies in one cluster with
    probability W = sum m_c (m_c - 1) / (N (N - 1)), its separation then
    having density exp(-r^2/(4 sigma^2)) / (4 pi sigma^2)^(3/2) (the
    difference of two offspring offsets), and otherwise is uniform; so the
    estimator's expectation is 1 - W + W exp(...) / (4 pi sigma^2)^(3/2)
    (the intensity form 1 + exp(...) / (lambda_p (4 pi sigma^2)^(3/2)) on
    average).  The soft estimator follows it from g ~ 14 near the origin
    down to ~2, to the smoothing of a kernel much narrower than sigma."""
    rng = np.random.default_rng(12)
    lam_p, mu, sigma = 200.0, 20.0, 0.02
    parents = rng.random((rng.poisson(lam_p), 3))
    pts = [p + rng.normal(0.0, sigma, (rng.poisson(mu), 3)) for p in parents]
    m = np.array([len(q) for q in pts], dtype=np.float64)
    pos = np.ascontiguousarray((np.concatenate(pts) % 1.0).T)
    n = pos.shape[1]
    rc, nbins = 0.1, 32
    g, e = oracle_lib.softrdf_forward(pos, np.zeros(n), dim=3, nbins=nbins, r_c=rc)
    w_in = float(np.sum(m * (m - 1.0))) / (n * (n - 1.0))
    c = (np.arange(nbins) + 0.5) * rc / nbins
    dens = np.exp(-c * c / (4 * sigma * sigma)) / (4 * math.pi * sigma * sigma) ** 1.5
    want = 1.0 - w_in + w_in * dens
    # beyond ~3 sigma the cross-cluster pairs dominate, and with only ~200
    # parents their count in a shell carries ~10% Poisson noise: compare the
    # bins up to r = 0.06, where g falls from ~14 to ~2
    ratio = g[3:20] / want[3:20]
    assert np.all(np.abs(ratio - 1.0) < 0.06), np.round(ratio, 3)
    assert abs(np.mean(ratio) - 1.0) < 0.03, np.round(ratio, 3)
    assert want[3] > 12.0 and want[19] < 2.5  # the range the test spans
