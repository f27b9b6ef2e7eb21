"""Equilibrium pin of the oracle's sweep.  With one trial per move (N_l = 1)
and no swelling, a pass moves each particle by a fixed-length step of
uniform direction (a symmetric proposal) and keeps it only if it overlaps
nothing: Metropolis for hard spheres, so repeated passes sample the
equilibrium hard-sphere (hard-disk) ensemble whatever the colour order.
Its contact value g(sigma+) must then match the Carnahan-Starling value
(1 - f/2) / (1 - f)^3 for spheres and Henderson's (1 - 7f/16) / (1 - f)^2
for disks (exact to third order in the virial expansion; at area fraction
0.5 it runs ~2% low, so the disks are tested at 0.35) -- a test of the whole
sweep (random vectors, wrap, contact test, minimum image, schedule) against
physics rather than against itself."""
import math

import numpy as np
import pytest

import oracle
import srm_inputs


def _contact_value(dim, n, f, seed, sweeps, every, step):
    from scipy.spatial import cKDTree
    name = "spheres3d" if dim == 3 else "disks2d"
    w = srm_inputs.make(name, n=n, seed=seed, f_target=f)
    grow = oracle.Oracle.from_workload(w)
    assert grow.run(5000)[0] == oracle.OK
    R = w.s_target
    mc = oracle.Oracle.from_workload(w, pos=grow.soa(), s0=R, sweep0=grow.t, n_l=1, c_w=0.0,
                                     c_m=step * R)
    sig, width, nb = 2.0 * R, 0.02 * R, 6
    counts = np.zeros(nb)
    samples = 0
    for t in range(sweeps):
        mc.sweep()
        if t >= sweeps // 2 and t % every == 0:  # the grown start relaxes first
            pts = mc.soa().T
            d = np.asarray(list(cKDTree(pts, boxsize=1.0).sparse_distance_matrix(
                cKDTree(pts, boxsize=1.0), sig + nb * width, output_type="ndarray")["v"]))
            d = d[d > 0]
            k = np.floor((d - sig) / width).astype(int)
            counts += np.bincount(k[(k >= 0) & (k < nb)], minlength=nb)[:nb] / 2.0
            samples += 1
    r0 = sig + np.arange(nb) * width
    r1 = r0 + width
    shell = (4.0 / 3.0 * math.pi * (r1 ** 3 - r0 ** 3)) if dim == 3 else (math.pi * (r1 ** 2 - r0 ** 2))
    g = counts / (samples * 0.5 * n * n * shell)  # unit box: density n
    # straight line through the bin centres, read at contact
    b, a = np.polyfit(r0 + 0.5 * width - sig, g, 1)
    return a, g


@pytest.mark.parametrize("dim,n,f,theory", [
    (3, 800, 0.30, (1 - 0.30 / 2) / (1 - 0.30) ** 3),          # Carnahan-Starling 2.48
    (2, 800, 0.35, (1 - 7 * 0.35 / 16) / (1 - 0.35) ** 2),     # Henderson 2.00
])
def test_contact_value_matches_equation_of_state(dim, n, f, theory):
    g0, g = _contact_value(dim, n, f, seed=17, sweeps=4000, every=5, step=0.25)
    assert abs(g0 - theory) < 0.04 * theory, (g0, theory, g)
