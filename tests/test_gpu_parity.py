"""GPU parity: the HIP path through the C ABI against the CPU oracle.

The contract is bit-exactness: cell assignment, accept codes, the overlap
flag and every FP64 coordinate must be identical (both sides evaluate the
same IEEE binary64 operation sequence without contraction).
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


def _mk(dim, n, seed, f=0.3, **kw):
    return srm_inputs.make("disks2d" if dim == 2 else "spheres3d", n=n, seed=seed, f_target=f,
                           **kw)


def _gpu_from_oracle(srm, o, w, **over):
    kw = dict(pos=o.soa(), s0=o.s, sweep0=o.t)
    if o.nrm is not None:
        kw["normals"] = np.ascontiguousarray(o.nrm.T)
    kw.update(over)
    return srm.SRM.from_workload(w, **kw)


def _assert_same_state(g, o, where=""):
    pos, nrm, s, t = g.state()
    ref = o.soa()
    if not np.array_equal(pos, ref):
        bad = np.nonzero(np.any(pos != ref, axis=0))[0]
        raise AssertionError(f"{where}: {len(bad)} positions differ, first ids {bad[:8]}")
    if o.nrm is not None:
        assert np.array_equal(nrm, np.ascontiguousarray(o.nrm.T)), where
    assert s == o.s and t == o.t, (where, s, o.s, t, o.t)


# ------------------------------------------------------------ device arithmetic

def test_device_sqrt_and_division_correctly_rounded(srm):
    rng = np.random.default_rng(0)
    n = 1_000_000
    a = np.concatenate([rng.random(n // 2), np.exp(rng.uniform(-700, 700, n // 2)),
                        [0.0, 1.0, 4.0, 2.0, 1e-310, 5e-324, 1.7976931348623157e308]])
    b = np.concatenate([rng.random(n // 2) + 1e-3, np.exp(rng.uniform(-300, 300, n // 2)),
                        [1.0, 3.0, 7.0, 0.1, 3.0, 2.0, 0.5]])
    sq, dv = srm.debug_fp(a, b)
    with np.errstate(over="ignore", under="ignore"):
        assert np.array_equal(sq, np.sqrt(a))
        assert np.array_equal(dv, a / b)
    # the values the unit-vector draw actually sees: q in (0, 1]
    q = rng.random(n) + 2.0**-53
    sq, dv = srm.debug_fp(q, np.sqrt(q))
    assert np.array_equal(sq, np.sqrt(q))
    assert np.array_equal(dv, q / np.sqrt(q))


def test_device_philox_matches_rocrand(srm):
    from tests import rocrand_ref
    rng = np.random.default_rng(1)
    n = 200000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(srm.debug_philox(ctr, key), rocrand_ref.philox4x32(ctr, key))


@pytest.mark.parametrize("dim,stream", [(2, 0), (3, 0), (3, 1)])
def test_device_unitvec_matches_oracle(srm, oracle_lib, dim, stream):
    n = 3000
    dev = srm.debug_unitvec(dim, 99, 17, 1, 5, 3, stream, 2.5e-3, n)
    for i in range(n):
        v, _ = oracle_lib.unitvec(dim, 99, i, 17, 1, 5, 3, stream, 2.5e-3)
        assert np.array_equal(v, dev[i]), i


# ------------------------------------------------------------------- binning

@pytest.mark.parametrize("dim,n,f", [(2, 2000, 0.5), (3, 20000, 0.35), (3, 4097, 0.3),
                                     (2, 7, 0.3), (3, 1, 0.1)])
def test_cell_assignment_parity(srm, oracle_lib, dim, n, f):
    w = _mk(dim, n, 5 + n % 7, f)
    o = oracle_lib.Oracle.from_workload(w)
    g = srm.SRM.from_workload(w)
    for s in (0.0, 0.3 * w.s_target, w.s_target):
        na, inv = o.grid_for_scale(s)
        assert tuple(int(x) for x in na) == g.grid(s)
        assert np.array_equal(g.cells(s).astype(np.int64), o.bin(na, inv))
    g.close()


# -------------------------------------------------------------- single pass

@pytest.mark.parametrize("dim,n,f,kind", [(2, 2000, 0.5, 0), (3, 20000, 0.35, 0),
                                          (3, 5000, 0.45, 1), (2, 333, 0.6, 0),
                                          (3, 600, 0.2, 0)])
def test_single_pass_parity(srm, oracle_lib, dim, n, f, kind):
    w = _mk(dim, n, 60 + n % 11, f)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(5000)
    o.t = 424242
    g = _gpu_from_oracle(srm, o, w)
    for k, grow in [(1, 1.0), (2, 1.02), (3, 1.05)]:
        s = o.s * grow
        na, inv = o.grid_for_scale(s)
        acc_o, ov_o = o.pass_(na, inv, s, kind, k)
        acc_g, ov_g = g.pass_(s, s, kind, k)
        _say(f"pass dim={dim} n={n} k={k}: accepted {int((acc_o > 0).sum())}, overlap {ov_o}")
        assert np.array_equal(acc_g, acc_o), np.nonzero(acc_g != acc_o)[0][:10]
        assert ov_g == ov_o
        _assert_same_state(g, o, f"pass k={k}")
    g.close()


# ------------------------------------------------------------------- sweeps

def _sweep_parity(srm, oracle_lib, w, max_sweeps, every=1, profile=False, **over):
    o = oracle_lib.Oracle.from_workload(w, **over)
    g = srm.SRM.from_workload(w, **over)
    if profile:
        g.profile(True)
    sweeps = 0
    while o.s < w.s_target and sweeps < max_sweeps:
        io, acc_o = o.sweep()
        ig = g.sweep()
        sweeps += 1
        assert ig["committed"] == io["committed"], sweeps
        assert ig["passes_main"] == io["passes_main"], sweeps
        assert ig["passes_shake"] == io["passes_shake"], sweeps
        assert ig["n_failed_last"] == io["n_failed_last"], sweeps
        assert tuple(ig["grid"]) == tuple(int(x) for x in io["na"]), sweeps
        assert ig["s"] == o.s and ig["sweep"] == o.t
        if sweeps % every == 0:
            assert np.array_equal(g.last_acc(), acc_o), sweeps
            _assert_same_state(g, o, f"sweep {sweeps}")
    _assert_same_state(g, o, "final")
    return o, g, sweeps


def test_config1_full_run_bitexact(srm, oracle_lib):
    """2D, N=2000 disks, f=0.5, seed 0: every sweep bit-identical."""
    w = srm_inputs.make("disks2d")
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 1000)
    assert o.s == w.s_target
    _say(f"config 1: {sweeps} sweeps, fraction {o.fraction()}")
    g.close()


def test_3d_run_bitexact(srm, oracle_lib):
    w = _mk(3, 20000, 71, 0.35)
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 1000, every=10)
    assert o.s == w.s_target
    g.close()


def test_polydisperse_run_bitexact(srm, oracle_lib):
    w = _mk(3, 3000, 72, 0.4, polydisperse_sigma=0.2)
    o, g, _ = _sweep_parity(srm, oracle_lib, w, 1000, every=5)
    assert o.s == w.s_target
    g.close()


@pytest.mark.parametrize("dim,n,seed,f,sigma", [(3, 2500, 75, 0.5, 0.2), (2, 3000, 74, 0.5, 0.5)])
def test_crowded_cells_bitexact(srm, oracle_lib, dim, n, seed, f, sigma):
    """Wide radius spreads make cells crowded (tens of particles a cell, a
    4x4x4 grid in 3D at the end), which moves migration to one wavefront per
    cell; every sweep still equals the oracle."""
    w = _mk(dim, n, seed, f, polydisperse_sigma=sigma)
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 1000, every=3)
    assert o.s == w.s_target
    grid = g.grid(w.s_target)[:dim]
    assert n >= 8 * int(np.prod(grid)), grid
    _say(f"crowded {dim}D: {sweeps} sweeps, final grid {grid}")
    g.close()


@pytest.mark.parametrize("dim,n,big,c_m_rel", [(3, 1500, 8.0, 0.3), (2, 2000, 24.0, 0.5)])
def test_cells_beyond_wave_capacity_bitexact(srm, oracle_lib, dim, n, big, c_m_rel):
    """One particle of 8 (3D) or 24 (2D) times the others' radius sets a cell
    edge of many small diameters, so the grid ends as one cell holding every
    particle.  Cells beyond the wavefront kernel's 96 LDS slots split each
    trial's stencil over the wavefront's lanes; every sweep equals the
    oracle, and most sweeps run such cells."""
    import dataclasses
    w = _mk(dim, n, 80 + dim, 0.3)
    rho = np.ones(n)
    rho[n // 2] = big
    s_t = srm_inputs.target_scale(dim, srm_inputs.BALL, 0.3, w.box, rho, n)
    w = dataclasses.replace(w, rho=rho, s_target=s_t, c_m=c_m_rel * s_t)
    o = oracle_lib.Oracle.from_workload(w)
    g = srm.SRM.from_workload(w)
    sweeps = beyond = 0
    while o.s < w.s_target:
        io, acc_o = o.sweep()
        ig = g.sweep()
        sweeps += 1
        assert ig["committed"] == io["committed"] and tuple(ig["grid"]) == tuple(
            int(x) for x in io["na"]), sweeps
        beyond += n > 96 * int(np.prod(ig["grid"][:dim]))
        if sweeps % 5 == 0:
            assert np.array_equal(g.last_acc(), acc_o), sweeps
            _assert_same_state(g, o, f"sweep {sweeps}")
    _assert_same_state(g, o, "final")
    assert beyond >= 40, beyond
    _say(f"{dim}D, one particle {big}x: {sweeps} sweeps, {beyond} with cells beyond 96")
    g.close()


@pytest.mark.parametrize("sigma,seed,f,bits", [(None, 71, 0.35, 1 | 32),
                                               (0.05, 5, 0.25, 1 | 32 | 16 | 2)])
def test_tile_variants_bitexact(srm, oracle_lib, sigma, seed, f, bits):
    """The grid's mean occupancy picks the migration kernel: the standard
    LDS tile (bit 1), then the middle (32) and the wide (16) regions as the
    region load nears each capacity, then one wavefront per cell (2).  Runs
    that pass through them equal the oracle sweep by sweep."""
    kw = {} if sigma is None else dict(polydisperse_sigma=sigma)
    w = _mk(3, 20000, seed, f, **kw)
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 1000, every=4, profile=True)
    assert o.s == w.s_target
    assert g.profile()["main_kernels"] == bits
    g.close()


@pytest.mark.parametrize("n_l", [3, 5, 13])
def test_tile_trial_counts_bitexact(srm, oracle_lib, n_l):
    """Dense packings make many first trials meet the near list; the LDS tile
    then draws a particle's later trials four at a time across its quad (one
    batch for N_l = 5, three for 13, a partial one for 3).  Thirty sweeps
    toward f = 0.45 (f 0.17 to 0.30 at the end, as N_l allows) equal the
    oracle, accept codes included."""
    w = _mk(3, 20000, 76 + n_l, 0.45, c_w=0.03, n_l=n_l)
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 30, every=3, profile=True)
    assert sweeps == 30
    assert g.profile()["main_kernels"] & 1
    _say(f"n_l={n_l}: {sweeps} sweeps")
    g.close()


def _region_loads(counts, nt, span=9):
    """Particles in each tile's (span)^3-cell region, every colour: a tile
    covers 4 colour cells (8 cells) per axis, its region starts one cell
    below its first cell of the colour."""
    na = counts.shape[0]
    loads = []
    for colour in range(8):
        off = [(colour >> a) & 1 for a in range(3)]
        for tz in range(nt):
            for ty in range(nt):
                for tx in range(nt):
                    idx = [(np.arange(span) + 8 * t + o - 1) % na
                           for t, o in zip((tx, ty, tz), off)]
                    loads.append(int(counts[np.ix_(idx[0], idx[1], idx[2])].sum()))
    return np.array(loads)


def test_tile_over_capacity_bitexact(srm, oracle_lib):
    """A dense slab (f = 0.45 in the lower half of the box) and an empty upper
    half: the mean load picks the standard LDS tile, but tens of tiles inside
    the slab hold more particles than its capacity and go to the
    global-memory kernel in the same colour phase.  Six sweeps without
    swelling equal the oracle, accept codes included."""
    slab = srm_inputs.make("spheres3d", n=6700, seed=91, f_target=0.45, box=(1.0, 1.0, 0.5),
                           c_w=0.03)
    o_slab = oracle_lib.Oracle.from_workload(slab)
    o_slab.run(400)
    s = o_slab.s
    assert s == slab.s_target
    w = srm_inputs.make("spheres3d", n=6700, seed=91, f_target=0.225, c_w=0.0)
    over = dict(pos=o_slab.soa(), s0=s, sweep0=o_slab.t, s_target=s, c_m=slab.c_m)
    o = oracle_lib.Oracle.from_workload(w, **over)
    g = srm.SRM.from_workload(w, **over)
    # the case this test is for: over-capacity tiles under the standard tile
    na, inv = o.grid_for_scale(s)
    assert int(na[0]) == int(na[1]) == int(na[2]) >= 9
    cells = o.bin(na, inv)
    counts = np.bincount(cells, minlength=int(np.prod(na))).reshape(
        int(na[2]), int(na[1]), int(na[0])).transpose(2, 1, 0)
    cap = 1456
    assert w.n / np.prod(na) * 729 <= cap - 3 * math.sqrt(cap)
    loads = _region_loads(counts, (int(na[0]) // 2 + 3) // 4)
    _say(f"over-capacity test: grid {na}, region loads max {loads.max()}, "
         f"over {int((loads > cap).sum())}")
    assert (loads > cap).sum() >= 10
    for k in range(6):
        io, acc_o = o.sweep()
        ig = g.sweep()
        assert ig["committed"] == io["committed"], k
        assert ig["passes_main"] == io["passes_main"], k
        assert np.array_equal(g.last_acc(), acc_o), k
        _assert_same_state(g, o, f"sweep {k}")
    g.close()


@pytest.mark.parametrize("dim,n,box,f", [(3, 20000, (1.0, 0.6, 1.5), 0.35),
                                         (2, 4000, (1.0, 2.5), 0.5)])
def test_stretched_box_bitexact(srm, oracle_lib, dim, n, box, f):
    """Boxes with unequal sides (per-axis grids, wraps and minimum images;
    the 3D one runs the tiled kernel): every sweep equals the oracle, and
    pairs, distance histogram and nearest neighbours of the final state
    too."""
    w = _mk(dim, n, 190 + dim, f, box=box)
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 1000, every=7)
    assert o.s == w.s_target
    grid = g.grid(w.s_target)[:dim]
    assert len(set(grid)) == dim, grid
    pairs = g.pairs(0.5 * o.s)
    assert np.array_equal(pairs, o.pairs_brute(0.5 * o.s))
    r_max = 4.0 * o.s
    counts, _ = g.rdf(40, r_max)
    assert np.array_equal(counts, o.rdf_brute(40, r_max))
    dist, _ = g.nearest(r_max)
    assert np.array_equal(dist, o.nearest_brute(r_max))
    _say(f"stretched {dim}D box {box}: {sweeps} sweeps, grid {grid}")
    g.close()


def test_2d_polydisperse_fast_swell_with_shakes(srm, oracle_lib):
    """Large swelling steps and few trials: sweeps shake, and the shake
    branch must match too."""
    w = _mk(2, 1500, 73, 0.62, polydisperse_sigma=0.2, c_w=0.08, n_k=3, n_l=2)
    o = oracle_lib.Oracle.from_workload(w)
    g = srm.SRM.from_workload(w)
    shakes = 0
    for sweep in range(60):
        io, acc_o = o.sweep()
        ig = g.sweep()
        shakes += not io["committed"]
        assert ig["committed"] == io["committed"] and ig["passes_main"] == io["passes_main"]
        assert np.array_equal(g.last_acc(), acc_o)
        _assert_same_state(g, o, f"sweep {sweep}")
    assert shakes > 0
    g.close()


def test_platelets_bitexact(srm, oracle_lib):
    w = srm_inputs.make("platelets", n=3000, f_target=0.02, cap_deg=15.0)
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 40, every=4)
    _say(f"platelets: {sweeps} sweeps, s={o.s}")
    g.close()


def test_platelets_isotropic_passes(srm, oracle_lib):
    w = srm_inputs.make("platelets", n=2500, seed=5, f_target=0.03, c_w=0.05)
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 25, every=1)
    g.close()


def test_platelets_large_steps_long_near_lists(srm, oracle_lib):
    """Migration steps of half a platelet radius at number density 4 put
    ~50 disks within reach of each one: the long near lists (and their
    overflow path) against the oracle, sweep by sweep, then 10 relaxation
    sweeps without swelling."""
    w = srm_inputs.make("platelets", n=1500, seed=9, f_target=math.pi * 4.0 / 400.0, c_w=0.05,
                        c_m_rel=0.5)
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 60, every=3)
    g.close()
    _say(f"platelets, large steps: {sweeps} sweeps, s/s_t={o.s / w.s_target}")
    # no swelling (s stays below the nominal target), large steps
    o2, g2, n2 = _sweep_parity(srm, oracle_lib, w, 10, every=1, pos=o.soa(), s0=o.s, sweep0=o.t,
                               normals=np.ascontiguousarray(o.nrm.T), c_w=0.0,
                               s_target=1.5 * w.s_target)
    assert n2 == 10 and o2.s == o.s
    g2.close()


# --------------------------------------------------------------- edge cases

def test_single_particle_and_tiny_systems(srm, oracle_lib):
    for n in (1, 2, 3, 9):
        w = _mk(3, n, 80 + n, 0.2)
        o, g, _ = _sweep_parity(srm, oracle_lib, w, 300)
        assert o.s == w.s_target
        g.close()


def test_zero_trials_and_zero_step(srm, oracle_lib):
    w = _mk(2, 500, 90, 0.3, n_l=0)
    o, g, _ = _sweep_parity(srm, oracle_lib, w, 20)
    g.close()
    w = _mk(3, 500, 91, 0.3)
    w.c_m = 0.0
    o, g, _ = _sweep_parity(srm, oracle_lib, w, 30)
    g.close()


def test_overlapping_start_rejected(srm):
    w = _mk(2, 100, 92, 0.3)
    w.pos[:, 1] = w.pos[:, 0]
    with pytest.raises(srm.SrmError) as e:
        srm.SRM.from_workload(w, s0=1e-3)
    assert e.value.status == srm.EOVERLAP


def test_out_of_box_rejected(srm):
    w = _mk(3, 100, 93, 0.3)
    w.pos[1, 7] = 1.0
    with pytest.raises(srm.SrmError) as e:
        srm.SRM.from_workload(w)
    assert e.value.status == srm.EINVAL
    w.pos[1, 7] = float("nan")
    with pytest.raises(srm.SrmError):
        srm.SRM.from_workload(w)


def test_not_converged_keeps_admissible_state(srm, oracle_lib):
    w = _mk(2, 800, 94, 0.5)
    g = srm.SRM.from_workload(w)
    st, info = g.run(7)
    assert st == srm.ENOTCONV and info["sweeps"] == 7
    o = oracle_lib.Oracle.from_workload(w)
    rc, sw, _ = o.run(7)
    assert rc == oracle_lib.ENOTCONV
    _assert_same_state(g, o, "after ENOTCONV")
    assert not o.overlap()
    g.close()


@pytest.mark.parametrize("dim,n,f_mid", [(2, 1500, 0.3), (3, 3000, 0.2)])
def test_staged_run_to_intermediate_fraction(srm, oracle_lib, dim, n, f_mid):
    """srm_run_to_fraction with an intermediate target stops exactly at the
    scale whose fraction is f_mid, bit-identical to the oracle run with the
    same stop scale; the next call continues to the context's target, again
    bit-identical; a target above the context's stops at s_target."""
    w = _mk(dim, n, 97 + dim, 0.5 if dim == 2 else 0.35, c_w=0.03)
    g = srm.SRM.from_workload(w)
    st, info = g.run(2000, f_target=f_mid)
    assert st == 0 and info["s"] < w.s_target
    assert abs(info["fraction"] - f_mid) <= 4e-16 * 8
    o = oracle_lib.Oracle.from_workload(w)
    rc, sweeps, passes = o.run(2000, s_stop=info["s"])
    assert rc == 0 and sweeps == info["sweeps"] and passes == info["passes"]
    _assert_same_state(g, o, "at the intermediate target")
    assert g.run(10, f_target=f_mid)[1]["sweeps"] == 0  # already there
    st, info2 = g.run(2000, f_target=0.99)
    rc, sweeps, passes = o.run(2000)
    assert st == 0 and rc == 0 and info2["s"] == w.s_target
    assert sweeps == info2["sweeps"] and passes == info2["passes"]
    _assert_same_state(g, o, "at the final target")
    import ctypes as C
    ri = srm.RunInfo()
    assert srm.lib().srm_run_to_fraction(g._ctx, float("nan"), 5, C.byref(ri)) == srm.EINVAL
    g.close()


def test_resume_is_bitexact(srm):
    w = _mk(3, 4000, 95, 0.3)
    a = srm.SRM.from_workload(w)
    for _ in range(40):
        a.sweep()
    b = srm.SRM.from_workload(w)
    for _ in range(25):
        b.sweep()
    pos, _, s, t = b.state()
    b.close()
    c = srm.SRM.from_workload(w, pos=pos, s0=s, sweep0=t)
    for _ in range(15):
        c.sweep()
    pa, _, sa, ta = a.state()
    pc, _, sc, tc = c.state()
    assert np.array_equal(pa, pc) and sa == sc and ta == tc
    a.close()
    c.close()


def test_device_memory_inputs_match_host(srm):
    import torch
    w = _mk(3, 5000, 96, 0.3)
    h = srm.SRM.from_workload(w)
    d = srm.SRM.from_workload(w, device=True)
    for _ in range(20):
        h.sweep()
        d.sweep()
    out = torch.empty((3, w.n), dtype=torch.float64, device="cuda")
    d.state_device(out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), h.state()[0])
    h.close()
    d.close()


def test_full_run_fraction_and_no_overlap(srm, oracle_lib):
    """Property at a larger size: the run ends exactly at s_target with the
    closed-form fraction, and the oracle's global check finds no overlap."""
    w = _mk(3, 200000, 97, 0.35)
    g = srm.SRM.from_workload(w)
    st, info = g.run(2000)
    assert st == 0 and info["s"] == w.s_target
    assert abs(info["fraction"] - 0.35) < 1e-12
    pos, _, s, t = g.state()
    o = oracle_lib.Oracle.from_workload(w, pos=pos, s0=s, sweep0=t)
    assert not o.overlap()
    g.close()


# ------------------------------------------------------- pairs and distances

@pytest.mark.parametrize("dim,n,poly", [(2, 3000, False), (3, 12000, False), (3, 4000, True)])
def test_pairs_match_oracle(srm, oracle_lib, dim, n, poly):
    w = _mk(dim, n, 120 + n % 13, 0.35, polydisperse_sigma=0.2 if poly else None)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(3000)
    g = _gpu_from_oracle(srm, o, w)
    for gap in (0.0, 0.2 * o.s, 1.5 * o.s):
        ref = o.pairs_brute(gap)
        got = g.pairs(gap)
        _say(f"pairs dim={dim} n={n} gap={gap:.3g}: {len(ref)}")
        assert np.array_equal(got.astype(np.int64), ref.astype(np.int64))
    g.close()


def test_pairs_capacity_error(srm):
    w = _mk(3, 3000, 125, 0.3)
    g = srm.SRM.from_workload(w)
    import ctypes as C
    cnt = C.c_int64()
    buf = np.zeros(2 * 4, dtype=np.int32)
    st = srm.lib().srm_pairs(g._ctx, 0.05, 4, C.c_void_p(buf.ctypes.data), C.byref(cnt), 0)
    assert st == srm.ECAPACITY and cnt.value > 4 and not buf.any()
    assert len(g.pairs(0.05)) == cnt.value
    g.close()


def test_platelet_pairs_match_oracle(srm, oracle_lib):
    w = srm_inputs.make("platelets", n=2500, seed=7, f_target=0.02)
    o = oracle_lib.Oracle.from_workload(w)
    for _ in range(30):
        o.sweep()
    g = _gpu_from_oracle(srm, o, w)
    for gap in (0.0, 0.3 * o.s, 1.0 * o.s):
        assert np.array_equal(g.pairs(gap).astype(np.int64), o.pairs_brute(gap).astype(np.int64))
    g.close()


@pytest.mark.parametrize("dim,n,nbins", [(2, 3000, 64), (3, 12000, 64), (3, 5000, 10000)])
def test_rdf_counts_match_oracle(srm, oracle_lib, dim, n, nbins):
    w = _mk(dim, n, 130 + n % 7, 0.3)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(3000)
    g = _gpu_from_oracle(srm, o, w)
    r_max = 5.0 * o.s
    counts, gr = g.rdf(nbins, r_max)
    ref = o.rdf_brute(nbins, r_max)
    assert np.array_equal(counts, ref)
    # normalisation: an ideal-gas shell count
    dr = r_max / nbins
    r0 = np.arange(nbins) * dr
    r1 = r0 + dr
    shell = (math.pi * (r1**2 - r0**2)) if dim == 2 else (4 * math.pi / 3 * (r1**3 - r0**3))
    ideal = 0.5 * n * (n - 1) * shell
    assert np.allclose(gr, counts / ideal, rtol=1e-12)
    g.close()


@pytest.mark.parametrize("dim,n,nbins,r_scale", [(2, 3000, 50, 3.0), (3, 8000, 40, 2.4),
                                                 (3, 6000, 20000, 2.2)])
def test_nearest_neighbours_match_oracle(srm, oracle_lib, dim, n, nbins, r_scale):
    """Nearest-neighbour distances of an SRM configuration (every value,
    bit for bit, +inf where none is within r_max; r_max = 2.2 radii leaves
    some particles without a neighbour) and their histogram (LDS counts and,
    for 20000 bins, direct atomics)."""
    w = _mk(dim, n, 150 + n % 11, 0.35)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(3000)
    g = _gpu_from_oracle(srm, o, w)
    r_max = r_scale * o.s
    dist, hist = g.nearest(r_max, nbins)
    ref = o.nearest_brute(r_max)
    assert np.array_equal(dist, ref)
    fin = ref[np.isfinite(ref)]
    b = (fin * (nbins / r_max)).astype(np.int64)
    assert np.array_equal(hist, np.bincount(b[b < nbins], minlength=nbins).astype(np.uint64))
    _say(f"nearest {dim}D: {int(np.isinf(ref).sum())} without a neighbour within r_max")
    g.close()


def test_nearest_edge_cases_and_errors(srm, oracle_lib):
    """One particle has no neighbour (+inf, empty histogram); two particles
    find each other across the periodic face; r_max beyond L/2, a bad bin
    count and a platelet context are rejected with SRM_EINVAL."""
    w1 = _mk(3, 1, 171, 0.2)
    g1 = srm.SRM.from_workload(w1)
    d, h = g1.nearest(0.4, 8)
    assert np.isinf(d).all() and not h.any()
    g1.close()
    pos = np.array([[0.995, 0.005], [0.5, 0.5], [0.25, 0.25]])
    g2 = srm.SRM(dim=3, n=2, s_target=0.001, c_w=0.01, c_m=1e-4, n_k=8, n_l=8, seed=3, pos=pos)
    o2 = oracle_lib.Oracle(dim=3, n=2, s_target=0.001, c_w=0.01, c_m=1e-4, n_k=8, n_l=8, seed=3,
                           pos=pos)
    d, _ = g2.nearest(0.1)
    assert np.array_equal(d, o2.nearest_brute(0.1)) and abs(d[0] - 0.01) < 1e-15
    for bad in (lambda: g2.nearest(0.6), lambda: g2.nearest(0.0), lambda: g2.nearest(0.1, 70000)):
        with pytest.raises(srm.SrmError) as e:
            bad()
        assert e.value.status == srm.EINVAL
    g2.close()
    wp = srm_inputs.make("platelets", n=500, f_target=0.01)
    gp = srm.SRM.from_workload(wp)
    with pytest.raises(srm.SrmError) as e:
        gp.nearest(0.2)
    assert e.value.status == srm.EINVAL
    gp.close()


@pytest.mark.parametrize("kind", ["disks", "spheres", "platelets"])
def test_percolation_matches_oracle(srm, oracle_lib, kind):
    """Wrapping axes of the gap-grown clusters at a ladder of gaps, and the
    critical gap found by 30 bisection steps, equal the oracle's union-find
    (same bonds bit for bit, so the same masks and the same bisection)."""
    if kind == "platelets":
        w = srm_inputs.make("platelets", n=1500, seed=7, f_target=0.02)
        steps = 40
    else:
        w = _mk(2 if kind == "disks" else 3, 2500, 161, 0.45 if kind == "disks" else 0.3)
        steps = 3000
    o = oracle_lib.Oracle.from_workload(w)
    o.run(steps)
    g = _gpu_from_oracle(srm, o, w)
    r = o.s
    lo, hi = 0.0, 3.0 * r
    masks = []
    for gap in np.linspace(lo, hi, 9):
        mg, mo = g.percolation(gap), o.percolation(gap)
        assert mg == mo, (gap, mg, mo)
        masks.append(mo)
    _say(f"percolation {kind}: masks {masks}")
    if masks[0] == 0 and masks[-1] != 0:
        gc_g = g.critical_gap(lo, hi, 30)
        gc_o = o.critical_gap(lo, hi, 30)
        assert gc_g == gc_o
        _say(f"percolation {kind}: critical gap {gc_g / r:.6f} r")
    g.close()


@pytest.mark.parametrize("dim,eta_ref", [(2, 1.12808737), (3, 0.3418174)])
def test_percolation_threshold_of_poisson_points_at_scale(srm, dim, eta_ref):
    """2e5 uniform points with vanishing hard cores: the soft shells are
    fully penetrable disks (spheres) of radius gap/2, and the critical gap
    found by the library's bisection gives the continuum percolation
    threshold, reduced density 1.128 (2D) and 0.342 (3D), within 3% (the
    finite-size spread at 2e5 points is about 1%)."""
    import time
    n = 200_000
    rng = np.random.default_rng(70 + dim)
    pos = rng.random((dim, n))
    g = srm.SRM(dim=dim, n=n, s_target=1e-9, c_w=0.01, c_m=1e-10, n_k=8, n_l=8, seed=1,
                pos=pos, s0=1e-9)
    hi = 0.006 if dim == 2 else 0.03
    t0 = time.perf_counter()
    gc = g.critical_gap(0.0, hi, 24)
    dt = time.perf_counter() - t0
    r = 0.5 * (gc + 2e-9)
    eta = n * (math.pi * r * r if dim == 2 else 4.0 / 3.0 * math.pi * r ** 3)
    _say(f"percolation threshold {dim}D n={n}: eta {eta:.5f} (continuum {eta_ref}), {dt:.2f} s")
    assert abs(eta / eta_ref - 1.0) < 0.03
    g.close()


def test_percolation_chain_and_errors(srm):
    """A chain of balls 0.1 apart percolates along x from a gap of 0.02
    (critical gap to 1e-10); a gap beyond half the box is rejected."""
    x = (np.arange(10) + 0.5) / 10
    chain = np.stack([x, np.full(10, 0.3), np.full(10, 0.6)])
    g = srm.SRM(dim=3, n=10, s_target=0.04, c_w=0.01, c_m=0.004, n_k=8, n_l=8, seed=1,
                pos=chain, s0=0.04)
    assert g.percolation(0.019) == 0 and g.percolation(0.021) == 1
    assert abs(g.critical_gap(0.0, 0.05, 40) - 0.02) < 1e-10
    with pytest.raises(srm.SrmError) as e:
        g.percolation(0.45)
    assert e.value.status == srm.EINVAL
    g.close()


# ------------------------------------------------------------ batched RVEs

def test_batch_members_bitidentical_to_solo_runs(srm, oracle_lib):
    """A reduced ensemble (half 2D, half 3D, lognormal radii, uneven N and
    targets) in one batched run: every RVE equals its solo run bit for bit,
    and two of them equal the oracle."""
    from paper_2605_18254_amd.batch import Batch
    metas = srm_inputs.batch_members(count=12, n_scale=0.02)
    ws = [srm_inputs.make_member(m) for m in metas]
    b = Batch(ws)
    b.configure(3, 128)
    st, info = b.run(600)
    _say(f"batch: {info}")
    assert st == 0 and info["converged"] == len(ws)
    for r, w in enumerate(ws):
        pos_b, s_b, t_b, passes_b = b.get(r)
        g = srm.SRM.from_workload(w)
        st_s, inf = g.run(600)
        assert st_s == 0
        pos_s, _, s_s, t_s = g.state()
        assert np.array_equal(pos_b, pos_s), r
        assert s_b == s_s == w.s_target and t_b == t_s and passes_b == inf["passes"]
        g.close()
    for r in (0, len(ws) - 1):
        o = oracle_lib.Oracle.from_workload(ws[r])
        assert o.run(600)[0] == 0
        assert np.array_equal(b.get(r)[0], o.soa())
    b.close()


def test_batch_configure_rejects_bad_shapes(srm):
    """Pass slots 1..64, blocks of 64, 128 or 256 threads (whole wavefronts
    of lane groups, within the kernels' launch bounds) and a crowded
    threshold of 1..64 particles a cell; anything else is refused before a
    graph is built, and the ensemble still runs after."""
    from paper_2605_18254_amd.batch import Batch
    metas = srm_inputs.batch_members(count=2, n_scale=0.01, seed0=2100)
    ws = [srm_inputs.make_member(m) for m in metas]
    b = Batch(ws)
    for bad in [(0, 128, 3), (65, 128, 3), (2, 32, 3), (2, 96, 3), (2, 512, 3),
                (2, 1024, 3), (2, 128, 0), (2, 128, 65)]:
        with pytest.raises(srm.SrmError):
            b.configure(*bad)
    b.configure(2, 64, 3)
    st, info = b.run(600)
    assert st == 0 and info["converged"] == len(ws)
    b.close()


def test_batch_launch_shape_invariance_and_notconv(srm):
    from paper_2605_18254_amd.batch import Batch
    metas = srm_inputs.batch_members(count=6, n_scale=0.03, seed0=2000)
    ws = [srm_inputs.make_member(m) for m in metas]
    res = []
    # schedules: every grid on one wavefront per cell, then (almost) every
    # grid on one thread per cell
    for slots, block, wave in [(1, 64, 1), (5, 256, 64), (3, 128, 3)]:
        b = Batch(ws)
        b.configure(slots, block, wave)
        st, info = b.run(10)           # stops early: not converged yet
        assert st == srm.ENOTCONV and info["not_converged"] == len(ws)
        st, info = b.run(600)          # continues to the target
        assert st == 0
        res.append([b.get(r)[0] for r in range(len(ws))])
        b.close()
    for other in res[1:]:
        for a_, b_ in zip(res[0], other):
            assert np.array_equal(a_, b_)


@pytest.mark.parametrize("dim,n,f,theory", [(3, 100_000, 0.30, (1 - 0.15) / 0.7 ** 3),
                                            (2, 100_000, 0.35, (1 - 7 * 0.35 / 16) / 0.65 ** 2)])
def test_equilibrium_contact_value_at_scale(srm, dim, n, f, theory):
    """Single-trial passes without swelling sample the hard-particle
    equilibrium (Metropolis with symmetric fixed-length moves).  The
    SRM-grown start carries excess near-contacts (g(sigma+) ~2.2 in 2D) that
    relax within ~1500 sweeps; after 1600, the contact value from srm_rdf at
    N = 1e5 matches Carnahan-Starling (3D) or Henderson (2D) within 1.5%."""
    w = _mk(dim, n, 23, f)
    g = srm.SRM.from_workload(w, device=True)
    assert g.run(5000)[0] == 0
    pos, _, s, t = g.state()
    g.close()
    R = w.s_target
    mc = srm.SRM.from_workload(w, pos=pos, s0=R, sweep0=t, n_l=1, c_w=0.0, c_m=0.25 * R)
    nbins, r_max = 130, 2.6 * R  # bins of 0.02 R; contact at bin 100
    acc = np.zeros(nbins)
    for sweep in range(2400):
        mc.sweep()
        if sweep >= 1600 and sweep % 5 == 0:
            acc += mc.rdf(nbins, r_max)[1]
    mc.close()
    gr = acc[100:106] / len(range(1600, 2400, 5))
    width = r_max / nbins
    b, a = np.polyfit((np.arange(6) + 0.5) * width, gr, 1)
    _say(f"equilibrium {dim}D f={f}: g(sigma+) {a:.4f}, theory {theory:.4f}")
    assert abs(a - theory) < 0.015 * theory, (a, theory, gr)
