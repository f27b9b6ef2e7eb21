"""GPU parity for spherodisk platelets (Sec. 3.3's platelet model): the
HIP path through the C ABI against the CPU oracle, bit for bit -- sweep by
sweep for thick and thin platelets, both starts, the soft-shell pair lists
and percolation; plus the argument checks of the new shape."""
import ctypes as C
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


def _workload(n, seed, ar, rho, **kw):
    """Spherodisks of aspect ratio ar at number density rho = N D^3 / V."""
    f = srm_inputs.spherodisk_volume_coeff(1.0 / ar) * rho / 8.0
    return srm_inputs.make("spherodisks", n=n, seed=seed, aspect_ratio=ar, f_target=f, **kw)


def _assert_same_state(g, o, where=""):
    pos, nrm, s, t = g.state()
    assert np.array_equal(pos, o.soa()), where
    assert np.array_equal(nrm, np.ascontiguousarray(o.nrm.T)), where
    assert s == o.s and t == o.t, (where, s, o.s, t, o.t)


def _sweep_parity(srm, oracle_lib, w, max_sweeps, every=1, until_target=True, **over):
    o = oracle_lib.Oracle.from_workload(w, **over)
    g = srm.SRM.from_workload(w, **over)
    sweeps = 0
    while (o.s < w.s_target or not until_target) and sweeps < max_sweeps:
        io, acc_o = o.sweep()
        ig = g.sweep()
        sweeps += 1
        assert ig["committed"] == io["committed"], sweeps
        assert ig["passes_main"] == io["passes_main"], sweeps
        assert ig["passes_shake"] == io["passes_shake"], sweeps
        assert ig["n_failed_last"] == io["n_failed_last"], sweeps
        assert ig["s"] == o.s and ig["sweep"] == o.t
        assert ig["fraction"] == pytest.approx(o.fraction(), rel=1e-13)
        if sweeps % every == 0:
            assert np.array_equal(g.last_acc(), acc_o), sweeps
            _assert_same_state(g, o, f"sweep {sweeps}")
    _assert_same_state(g, o, "final")
    return o, g, sweeps


@pytest.mark.parametrize("ar,n,seed,rho,cap", [(10.0, 1500, 51, 2.5, None),
                                              (100.0, 2000, 52, 2.5, 15.0),
                                              (200.0, 1500, 53, 4.0, None)])
def test_spherodisks_bitexact(srm, oracle_lib, ar, n, seed, rho, cap):
    w = _workload(n, seed, ar, rho, cap_deg=cap, c_w=0.02)
    _say(f"spherodisks ar={ar} n={n} rho={rho} cap={cap}")
    o, g, sweeps = _sweep_parity(srm, oracle_lib, w, 80, every=2)
    _say(f"  {sweeps} sweeps, s/s_t={o.s / w.s_target}")
    assert sweeps >= 10
    g.close()


def test_spherodisks_relaxation_with_large_steps(srm, oracle_lib):
    """Grown without relaxation, then ten sweeps with no swelling and steps
    of half a radius: tens of spherodisks within reach of each one (the
    long near lists)."""
    w = _workload(1200, 54, 20.0, 3.0, c_w=0.05)
    o = oracle_lib.Oracle.from_workload(w)
    rc, _, _ = o.run(200)
    _say(f"relaxation start: rc={rc} s/s_t={o.s / w.s_target}")
    w2 = _workload(1200, 54, 20.0, 3.0, c_w=0.0, c_m_rel=0.5)
    over = dict(pos=o.soa(), s0=o.s, sweep0=o.t, normals=np.ascontiguousarray(o.nrm.T),
                s_target=1.5 * w.s_target)
    o2, g2, sweeps = _sweep_parity(srm, oracle_lib, w2, 10, every=1, until_target=False, **over)
    assert sweeps == 10 and o2.s == o.s
    g2.close()


def test_spherodisk_pairs_and_percolation_match_oracle(srm, oracle_lib):
    w = _workload(1500, 55, 10.0, 2.0, c_w=0.02)
    o = oracle_lib.Oracle.from_workload(w)
    o.run(200)
    g = srm.SRM.from_workload(w, pos=o.soa(), s0=o.s, sweep0=o.t,
                              normals=np.ascontiguousarray(o.nrm.T))
    r = o.s
    for gap in (0.0, 0.05 * r, 0.3 * r, 1.0 * r):
        gp, op = g.pairs(gap).astype(np.int64), o.pairs_brute(gap).astype(np.int64)
        assert np.array_equal(gp, op), gap
    masks = []
    for gap in np.linspace(0.0, 1.5 * r, 7):
        mg, mo = g.percolation(gap), o.percolation(gap)
        assert mg == mo, (gap, mg, mo)
        masks.append(mo)
    _say(f"spherodisk percolation masks {masks}")
    if masks[0] == 0 and masks[-1] != 0:
        assert g.critical_gap(0.0, 1.5 * r, 30) == o.critical_gap(0.0, 1.5 * r, 30)
    g.close()


def test_spherodisk_arguments_checked(srm):
    w = _workload(200, 56, 50.0, 1.0)
    for bad in (0.0, 0.5, -0.1):
        with pytest.raises(srm.SrmError) as e:
            srm.SRM.from_workload(w, thick_ratio=bad)
        assert e.value.status == srm.EINVAL
    with pytest.raises(srm.SrmError) as e:
        srm.SRM.from_workload(w, normals=None)
    assert e.value.status == srm.EINVAL
    # RSA draws zero-thickness platelets only
    box = np.ones(3)
    st = srm.lib().srm_rsa(3, srm.SPHERODISK, 10, box.ctypes.data_as(C.POINTER(C.c_double)),
                           C.c_double(0.01),
                           C.c_uint64(1), C.c_int64(100), C.c_int64(0), None, None, None, 0, None,
                           None)
    assert st == srm.EINVAL
