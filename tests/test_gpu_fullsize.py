"""Full-size checks on the benchmark workload: 3D periodic unit cube, N = 1e7
spheres (seed 1, target fraction 0.35), in the launch configuration bench.py
times (the 178^3 grid at the target radius, the LDS-tiled colour phases).

The oracle cannot run the whole box, so:
  * one dense migration pass is compared bit for bit on sample blocks of
    cells: the oracle runs the pass only on the cells within 9 cells of a
    block (a cell's outcome depends on its 3^3 neighbours at the time of its
    colour phase, so a wrong value travels at most one cell per phase, and a
    pass has 8 phases), and the block's particles must match;
  * a whole run to the target is checked by properties that hold at any
    size: the target radius is reached exactly, the volume fraction equals
    its closed form, and no sampled particle overlaps another.
"""
import math
import sys

import numpy as np
import pytest

import srm_inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def srm():
    import paper_2605_18254_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def workload():
    return srm_inputs.make("spheres3d")


def _cone(na, lo, size, margin):
    """Cells of the periodic grid within Chebyshev distance `margin` of the
    block [lo, lo + size)^3, and the block itself, as flat masks."""
    axes_mask, axes_block = [], []
    for a in range(3):
        c = np.arange(int(na[a]))
        # periodic distance from c to the block along axis a
        d = np.minimum.reduce([np.abs(((c - (lo[a] + j)) + na[a] // 2) % na[a] - na[a] // 2)
                               for j in range(size)])
        axes_mask.append(d <= margin)
        axes_block.append(d == 0)
    m = (axes_mask[2][:, None, None] & axes_mask[1][None, :, None] & axes_mask[0][None, None, :])
    b = (axes_block[2][:, None, None] & axes_block[1][None, :, None] & axes_block[0][None, None, :])
    return m.ravel().astype(np.uint8), b.ravel()


@pytest.mark.parametrize("scale,k", [(1.0, 1), (0.7, 3)])
def test_fullsize_dense_pass_matches_oracle_on_sample_blocks(srm, oracle_lib, workload, scale, k):
    """A migration pass on the uniform start with radii at `scale` times the
    target (at 1.0 heavily overlapping, so most trials are rejected and the
    failure path runs; at 0.7 about half the particles move) at N = 1e7:
    accept codes and coordinates of every particle of two 8^3-cell sample
    blocks -- one inside the box, one across the periodic corner -- equal
    the oracle's."""
    w = workload
    s = w.s_target * scale
    g = srm.SRM.from_workload(w, device=True)
    _say(f"fullsize pass: N={w.n}, s={s}, k={k}")
    acc_g, _ = g.pass_(s, s, 0, k)
    pos_g = g.state()[0]
    grid_g = g.grid(s)
    g.close()
    _say(f"GPU pass done, grid {grid_g}, rejected {int(np.sum(acc_g == 0))}")
    for lo in [(60, 90, 100), (172, 174, 170)]:
        o = oracle_lib.Oracle.from_workload(w)
        na, inv = o.grid_for_scale(s)
        assert tuple(int(x) for x in na) == tuple(grid_g)
        cell = o.bin(na, inv)
        mask, block = _cone(na, lo, 8, 9)
        acc_o, _ = o.pass_(na, inv, s, 0, k, mask=mask)
        sel = block[cell]
        n_sel = int(sel.sum())
        assert n_sel > 300
        assert np.array_equal(acc_g[sel], acc_o[sel]), lo
        assert np.array_equal(pos_g[:, sel], o.soa()[:, sel]), lo
        _say(f"block {lo}: {n_sel} particles, {int(np.sum(acc_o[sel] == 0))} rejected, "
             f"{int(np.sum(acc_o[sel] > 1))} moved on a later trial, equal")
        del o


@pytest.mark.parametrize("na,bits", [(170, 32), (160, 16)])
def test_fullsize_larger_tiles_pass_matches_oracle_on_sample_blocks(srm, oracle_lib, workload,
                                                                    na, bits):
    """The same comparison on coarser grids: 170^3 (about 2.04 particles a
    cell, the density of the Fig. 2 protocol's late sweeps) runs the middle
    LDS region, 160^3 (2.44) the wide one; sample blocks inside the box and
    across the periodic corner equal the oracle."""
    w = workload
    grid_s = (1.0 / (na + 0.5) - 2.5 * w.c_m) / 2.5
    s = 0.7 * w.s_target
    g = srm.SRM.from_workload(w, device=True)
    assert tuple(g.grid(grid_s)) == (na, na, na)
    g.profile(True)
    acc_g, _ = g.pass_(grid_s, s, 0, 2)
    assert g.profile()["main_kernels"] == bits
    pos_g = g.state()[0]
    g.close()
    for lo in [(40, 120, 70), (na - 4, na - 3, na - 5)]:
        o = oracle_lib.Oracle.from_workload(w)
        nao, inv = o.grid(grid_s * o.rho_max())
        assert tuple(int(x) for x in nao) == (na, na, na)
        cell = o.bin(nao, inv)
        mask, block = _cone(nao, lo, 8, 9)
        acc_o, _ = o.pass_(nao, inv, s, 0, 2, mask=mask)
        sel = block[cell]
        assert int(sel.sum()) > 500
        assert np.array_equal(acc_g[sel], acc_o[sel]), lo
        assert np.array_equal(pos_g[:, sel], o.soa()[:, sel]), lo
        _say(f"{na}^3 block {lo}: {int(sel.sum())} particles, "
             f"{int(np.sum(acc_o[sel] == 0))} rejected, equal")
        del o


def test_fullsize_run_reaches_target_without_overlap(srm, workload):
    """The benchmark run itself (srm_run_to_fraction) ends at s == s_target
    with the closed-form fraction N (4/3) pi s^3 / |box| = 0.35, and none of
    200 000 sampled particles overlaps its nearest neighbour."""
    from scipy.spatial import cKDTree

    w = workload
    g = srm.SRM.from_workload(w, device=True)
    st, info = g.run(1000)
    assert st == 0 and info["s"] == w.s_target
    frac = w.n * (4.0 / 3.0) * math.pi * w.s_target ** 3
    assert abs(info["fraction"] - frac) <= 1e-12 * frac
    assert abs(frac - 0.35) <= 1e-12
    pos = g.state()[0]
    g.close()
    _say(f"run: {info['sweeps']} sweeps, {info['passes']} passes")
    tree = cKDTree(pos.T, boxsize=1.0)
    rng = np.random.default_rng(7)
    ids = rng.choice(w.n, size=200_000, replace=False)
    dist, _ = tree.query(pos.T[ids], k=2)
    nearest = dist[:, 1]
    assert nearest.min() > 2.0 * w.s_target * (1.0 - 1e-12), nearest.min() / (2 * w.s_target)
    _say(f"closest sampled pair at {nearest.min() / (2 * w.s_target):.6f} diameters")


@pytest.mark.parametrize("cap", [None, 15.0])
def test_fullsize_platelet_pass_matches_oracle(srm, oracle_lib, cap):
    """The platelet workload at its full size (N = 2e5, f = 0.02, 30^3 grid,
    about 7 platelets a cell, so the wavefront-per-cell kernel runs): one
    pass at the target radius from each start, every accept code, centre and
    normal equal to the oracle's (isotropic: ~90% rejected; 15-degree cap:
    ~30% rejected, ~25% accepted on a later trial)."""
    w = srm_inputs.make("platelets", cap_deg=cap)
    s = w.s_target
    g = srm.SRM.from_workload(w, device=True)
    acc_g, _ = g.pass_(s, s, 0, 1)
    pos_g, nrm_g, _, _ = g.state()
    g.close()
    o = oracle_lib.Oracle.from_workload(w)
    na, inv = o.grid_for_scale(s)
    acc_o, _ = o.pass_(na, inv, s, 0, 1)
    assert np.array_equal(acc_g, acc_o)
    assert np.array_equal(pos_g, o.soa())
    assert np.array_equal(nrm_g, np.ascontiguousarray(o.nrm.T))
    _say(f"platelets cap={cap}: {int(np.sum(acc_o == 0))} rejected, "
         f"{int(np.sum(acc_o > 1))} on a later trial, equal")


def test_fullsize_pair_count_beyond_int32_is_refused(srm, workload):
    """10^7 uniform points with a gap of 0.0225 have about
    N^2/2 * (4/3) pi gap^3 = 2.4e9 pairs, more than the int32 row offsets
    hold: srm_pairs reports SRM_ECAPACITY with the exact 64-bit count before
    any offset scan or emit kernel runs, and percolation refuses likewise.
    A gap beyond half the box less the diameters is refused as invalid."""
    import ctypes as C

    w = workload
    g = srm.SRM.from_workload(w, device=True)
    cnt = C.c_int64(-1)
    buf = np.zeros(8, dtype=np.int32)
    _say("pairs at gap 0.0225 on 1e7 points")
    st = srm.lib().srm_pairs(g._ctx, 0.0225, 4, C.c_void_p(buf.ctypes.data), C.byref(cnt), 0)
    expect = 0.5 * w.n * (w.n - 1) * (4.0 / 3.0) * math.pi * 0.0225 ** 3
    assert st == srm.ECAPACITY and cnt.value > 2**31 - 1
    assert abs(cnt.value - expect) < 1e-3 * expect, (cnt.value, expect)
    assert not buf.any()
    m = C.c_int32(-1)
    assert srm.lib().srm_percolation(g._ctx, 0.0225, C.byref(m)) == srm.ECAPACITY
    st = srm.lib().srm_pairs(g._ctx, 0.6, 0, None, C.byref(cnt), 0)
    assert st == srm.EINVAL
    # a moderate gap still enumerates (counted only)
    st = srm.lib().srm_pairs(g._ctx, 0.002, 0, None, C.byref(cnt), 0)
    expect = 0.5 * w.n * (w.n - 1) * (4.0 / 3.0) * math.pi * 0.002 ** 3
    assert st == srm.ECAPACITY and abs(cnt.value - expect) < 0.01 * expect
    g.close()
    _say(f"refused {cnt.value} pairs correctly")
