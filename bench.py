"""SRM sweep throughput on one MI355X.

Workload: 3D periodic unit cube, N = 1e7 monodisperse spheres, positions
uniform (Philox seed 1), radii swelling from 0 by c_w = 0.01 s_target per
sweep to the target volume fraction 0.35, migration step c_m = 0.1 s_target,
N_k = N_l = 8.  A step is one SRM sweep (Algorithm 1 iteration: swell, then
bin + migration pass + global check until a pass leaves no overlap, or a
shake).  Inputs are resident in HBM before timing starts.

Timed window: the K = --steps sweeps that END at the target fraction (the
densest sweeps of the run).  An untimed run first finds how many sweeps the
run takes (and counts the trial moves of every sweep); a second, identical
run (results are a pure function of the inputs) then sweeps untimed up to
the window -- at least --warmup sweeps -- and times exactly the K window
sweeps between two device synchronisations.  When the run is shorter than
warmup + K sweeps the window continues past the target with sweeps at the
target fraction.

value = particle updates per second = N * (migration passes in the timed
sweeps) / wall time of the timed sweeps.

Prints one JSON line.  --gpus must be 1 (single-GPU build).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector instruction issue of MI355X: a wavefront's VALU instruction holds
# one 16-lane SIMD for 4 cycles; 256 CUs x 4 SIMDs at 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wavefront instructions per second
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Algorithmic HBM bytes per particle update of the migration kernel (3D
# spheres, FP64 SoA, int32 ids): read the particle's position and id, write
# its new position.
ALG_BYTES_PER_UPDATE = 24 + 4 + 24
# Floor of one colour phase's traffic: the 3^3 stencils of one colour's
# cells cover the whole box, so a phase reads every particle's position and
# id once and every cell range, and writes its own particles' positions and
# accept codes.
PHASE_READ_PER_PARTICLE = 24 + 4
PHASE_READ_PER_CELL = 4
PHASE_WRITE_PER_OWN = 24 + 1
# Algorithmic bytes per particle update of a whole sweep step: a rebin
# (read position and id, write them sorted, cell ranges amortised: about
# 60 B) plus the migration pass (52 B).
ALG_BYTES_PER_UPDATE_SWEEP = 112


# Sources of the migration kernels: HBM traffic recorded from counters is
# reported only while these are unchanged.
KERNEL_SOURCES = ["paper_2605_18254_amd/csrc/k_migrate.hip",
                  "paper_2605_18254_amd/csrc/srm_cellpass.hpp",
                  "paper_2605_18254_amd/csrc/srm_device.hpp",
                  "paper_2605_18254_amd/csrc/srm_internal.hpp"]
TRAFFIC_FILE = "profiles/migrate_tile_spheres3d_n1e7.md"
VALU_FILE = "profiles/migrate_tile_valu_spheres3d_n1e7.md"
PLATELET_VALU_FILE = "profiles/migrate_platelet_valu_n2e5.md"


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _record(relpath, kernel):
    """The "- key: value" lines of a committed counter summary, or None when
    it is missing, covers another kernel, or the kernel sources changed."""
    path = os.path.join(ROOT, relpath)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                rec[k.strip("`")] = v.strip().strip("`")
    if rec.get("kernel") != kernel or rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return rec


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None."""
    rec = _record(TRAFFIC_FILE, kernel)
    try:
        return None if rec is None else {
            "bytes_per_launch": float(rec["fetch_bytes_per_launch"]) +
            float(rec["write_bytes_per_launch"]), "source": TRAFFIC_FILE}
    except (KeyError, ValueError):
        return None


def _valu_figures(rec, launch_s):
    valu = float(rec["sq_insts_valu_per_launch"])
    fp64 = {k: float(rec[f"sq_insts_valu_{k}_f64_per_launch"]) for k in ("add", "mul", "fma", "trans")}
    lane_ops = 64.0 * (fp64["add"] + fp64["mul"] + fp64["trans"] + 2.0 * fp64["fma"])
    return {"insts_per_launch": valu, "issue_rate": valu / launch_s,
            "issue_peak": VALU_ISSUE_PEAK, "issue_frac": valu / launch_s / VALU_ISSUE_PEAK,
            "fp64_insts_per_launch": sum(fp64.values()),
            "fp64_lane_tflops_upper": lane_ops / launch_s / 1e12,
            "fp64_peak_tflops": FP64_VECTOR_PEAK_TFLOPS,
            "fp64_frac_upper": lane_ops / launch_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "lds_insts_per_launch": float(rec["sq_insts_lds_per_launch"]),
            "vmem_rd_insts_per_launch": float(rec["sq_insts_vmem_rd_per_launch"])}


def recorded_valu(kernel, launch_s):
    """The vector-ALU side of `kernel`: wavefront instruction counts per
    launch from the committed counter summary over the live launch time.
    Issued instructions include address, loop and random-number work, so
    this is a ceiling on issue, not algorithmic flops; FP64 lane operations
    count all 64 lanes of each instruction (an upper bound on useful ones)."""
    rec = _record(VALU_FILE, kernel)
    try:
        return None if rec is None else dict(_valu_figures(rec, launch_s), source=VALU_FILE)
    except (KeyError, ValueError):
        return None


def recorded_platelet_valu(launch_s):
    """The same figures for the platelet kernel (one wavefront per cell, both
    near-list sizes together) on the N = 2e5 platelet runs, the FP64 side
    against the vector FP64 peak."""
    rec = _record(PLATELET_VALU_FILE, "k_migrate_platelet_wave")
    try:
        return None if rec is None else dict(_valu_figures(rec, launch_s),
                                             source=PLATELET_VALU_FILE)
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=0,
                    help="particles of the oracle's sub-box (default: the box of edge 32/178 "
                         "at the workload's number density)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-ensemble and gradient measurements")
    ap.add_argument("--extras",
                    default="at_target,n_scaling,platelets,platelet_protocol,spherodisk_protocol,"
                            "batched,gradient",
                    help="comma-separated extras to run")
    ap.add_argument("--batch-sweeps", type=int, default=400,
                    help="sweep budget of every RVE of the batched ensemble")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy this many MiB device to device before the sweeps (a plain copy "
                         "kernel of known size, to calibrate HBM byte counters)")
    ap.add_argument("--save-window", default="",
                    help="write the state at the start of the timed window to this .npz file")
    ap.add_argument("--window-from", default="",
                    help="start from a state written by --save-window and run only the timed "
                         "window (for a profiler run that sees the window's kernels alone)")
    return ap.parse_args()


def host_boundary(srm, w, torch):
    """The boundary with host buffers, outside the timed region: srm_init
    from host positions (the library copies them to the device), and
    srm_get_state back to host memory; srm_init from positions already in
    device memory beside it."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = srm.SRM.from_workload(w)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.state()
    t2 = time.perf_counter()
    g.close()
    pos_d = torch.from_numpy(w.pos).cuda()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    g = srm.SRM.from_workload(w, pos=pos_d)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    g.close()
    del pos_d
    return {"init_from_host_s": t1 - t0, "state_to_host_s": t2 - t1,
            "init_from_device_s": t4 - t3, "position_bytes_each_way": int(w.pos.nbytes)}


def _cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": allowed}


def cpu_baseline(steps, warmup, n_sub):
    """The oracle (single-threaded C) on a bounded sample of the same
    workload: a sub-box of edge L' at the same number density (1e7 per unit
    volume), so the same target radius, migration step, rates and cell
    occupancy, grown by the oracle itself from its own uniform start to
    f = 0.35 with every sweep timed; the sample is the same window as the
    GPU's, the K sweeps ending at the target (whole sweeps: swell, binning,
    passes, global checks)."""
    import oracle
    import srm_inputs

    L = (n_sub / 1e7) ** (1.0 / 3.0)
    w = srm_inputs.make("spheres3d", n=n_sub, seed=1, box=(L, L, L))
    o = oracle.Oracle.from_workload(w)
    rows, reached = [], None
    t_all = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        info, _ = o.sweep()
        rows.append((time.perf_counter() - t0, info["passes_main"] + info["passes_shake"]))
        if reached is None and o.s == w.s_target:
            reached = len(rows)
        if reached is not None and len(rows) >= max(reached, warmup + steps):
            break
        if len(rows) > 5000:
            raise RuntimeError("oracle sub-box did not reach the target")
    start = max(warmup, reached - steps)
    win = rows[start:start + steps]
    dt = sum(r[0] for r in win)
    passes = sum(r[1] for r in win)
    return dict(value=n_sub * passes / dt, unit="particle-updates/s", cores=1, kind="oracle",
                sample=(f"oracle sub-box of the same workload: N={n_sub} in a cube of edge "
                        f"{L:.6f} (number density 1e7 per unit volume, f_target 0.35, same "
                        f"s_target, c_w, c_m, N_k, N_l), grown by the oracle from its own "
                        f"uniform start; timed: sweeps {start + 1}..{start + steps} of "
                        f"{reached} (the {steps} sweeps ending at the target, {passes} passes, "
                        f"{dt:.1f} s), whole sweeps incl. binning; whole growth "
                        f"{time.perf_counter() - t_all:.1f} s"),
                **_cpu_info())


def _say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batched_extra(max_sweeps):
    """The 256-RVE ensemble (half 2D, half 3D, N log-uniform in [1e3, 1e5],
    targets uniform in [0.30, 0.55], lognormal radii, seeds 1000..1255):
    one batched run against the 256 solo runs, same sweep budget.  Both do
    the same passes (the states are compared bit for bit), so the ratio of
    wall times is the batching gain."""
    import numpy as np
    import torch

    import paper_2605_18254_amd as srm
    import srm_inputs
    from paper_2605_18254_amd.batch import Batch, autotune

    ws = [srm_inputs.make_member(m) for m in srm_inputs.batch_members()]
    t0 = time.perf_counter()
    shape = autotune(ws, sweeps=40, slots=(2, 4, 8), blocks=(128,), wave_occupancy=(1, 2, 3))
    tune_s = time.perf_counter() - t0
    _say(f"batch autotune -> slots={shape[0]} block={shape[1]} wave={shape[2]} ({tune_s:.1f} s)")
    b = Batch(ws)
    b.configure(*shape)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = b.run(max_sweeps)
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    _say(f"batched: {dt_b:.2f} s, {info}")
    ctxs = [srm.SRM.from_workload(w, device=True) for w in ws]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    upd_s = 0
    solo = []  # (converged, seconds, updates) per RVE
    for r, g in enumerate(ctxs):
        t1 = time.perf_counter()
        st_r, info_r = g.run(max_sweeps)
        torch.cuda.synchronize()
        solo.append((st_r == 0, time.perf_counter() - t1, info_r["updates"]))
        upd_s += info_r["updates"]
        if r % 32 == 31:
            _say(f"sequential: {r + 1} RVEs, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    _say(f"sequential: {dt_s:.2f} s")
    # the same comparison on the RVEs that reach their target, at the same
    # final fraction: a batch of those alone against their solo runs
    conv = [r for r in range(len(ws)) if solo[r][0]]
    bc = Batch([ws[r] for r in conv])
    bc.configure(*shape)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_c, info_c = bc.run(max_sweeps)
    torch.cuda.synchronize()
    dt_bc = time.perf_counter() - t0
    conv_identical = True
    for k, r in enumerate(conv):
        pos_b, s_b, t_b, _ = bc.get(k)
        pos_s, _, s_s, t_s = ctxs[r].state()
        conv_identical = conv_identical and np.array_equal(pos_b, pos_s) and s_b == s_s and t_b == t_s
    bc.close()
    dt_sc = sum(solo[r][1] for r in conv)
    upd_c = sum(solo[r][2] for r in conv)
    identical, overlaps, fr_b = True, 0, []
    for r, g in enumerate(ctxs):
        pos_b, s_b, t_b, _ = b.get(r)
        pos_s, _, s_s, t_s = g.state()
        identical = identical and np.array_equal(pos_b, pos_s) and s_b == s_s and t_b == t_s
        overlaps += len(g.pairs(0.0))
        fr_b.append(s_b / ws[r].s_target)
        g.close()
    b.close()
    return {
        "workload": "256 RVEs: 128 2D + 128 3D, N log-uniform [1e3,1e5], f uniform "
                    "[0.30,0.55], lognormal radii sigma 0.2, seeds 1000..1255",
        "max_sweeps": max_sweeps, "converged": info["converged"],
        "not_converged": info["not_converged"],
        "min_s_over_s_target": min(fr_b), "overlapping_pairs": overlaps,
        "bitidentical_to_solo": identical, "launch": {"slots": shape[0], "block": shape[1], "wave_occupancy": shape[2],
                   "autotune_s": tune_s},
        "updates": info["updates"],
        "batched": {"s": dt_b, "updates_per_s": info["updates"] / dt_b,
                    "graph_replays": info["replays"]},
        "sequential": {"s": dt_s, "updates_per_s": upd_s / dt_s},
        "speedup": dt_s / dt_b,
        "converged_subset": {
            "rves": len(conv), "all_at_target": st_c == 0 and info_c["converged"] == len(conv),
            "bitidentical_to_solo": conv_identical,
            "batched": {"s": dt_bc, "updates_per_s": upd_c / dt_bc},
            "sequential": {"s": dt_sc, "updates_per_s": upd_c / dt_sc},
            "speedup": dt_sc / dt_bc},
    }


def platelet_extra(max_sweeps):
    """Thin circular platelets (thickness D/100), N = 2e5, target volume
    fraction 0.02, exact disk-disk test, migration of centre and normal:
    one run from isotropic normals, one from normals within 15 degrees of a
    common axis."""
    import torch

    import paper_2605_18254_amd as srm
    import srm_inputs

    out = {}
    plate_launches, plate_ms, plate_kinds = 0, 0.0, 0
    for tag, cap in (("isotropic", None), ("cap15", 15.0)):
        w = srm_inputs.make("platelets", cap_deg=cap)
        g = srm.SRM.from_workload(w, device=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = g.run(max_sweeps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        overlaps = len(g.pairs(0.0))
        # critical percolation distance of the final state (bisection on the
        # tunnelling gap, 30 halvings), in platelet diameters
        diam = 2.0 * w.s_target
        hi = 0.25 * diam
        while not g.percolation(hi) and hi < 8 * diam:
            hi *= 2.0
        t1 = time.perf_counter()
        gap_c = g.critical_gap(0.0, hi, 30) if g.percolation(hi) else None
        dt_perc = time.perf_counter() - t1
        g.close()
        # the same run again with the device-time profile on: the platelet
        # kernel's launches and time (kept out of the timed run above)
        g = srm.SRM.from_workload(w, device=True)
        g.profile(enable=True)
        g.run(max_sweeps)
        prof = g.profile()
        g.close()
        plate_launches += prof["launches_migrate"]
        plate_ms += prof["ms_migrate_main"]
        plate_kinds |= prof["main_kernels"]
        out[tag] = {"converged": st == 0, "sweeps": info["sweeps"], "passes": info["passes"],
                    "s": dt, "updates_per_s": info["updates"] / dt,
                    "fraction": info["fraction"], "overlapping_pairs": overlaps,
                    "number_density": w.n * diam ** 3,
                    "critical_gap_over_d": None if gap_c is None else gap_c / diam,
                    "critical_gap_s": dt_perc}
        _say(f"platelets {tag}: {out[tag]}")
    out["workload"] = ("platelets N=2e5, thickness D/100, f_target=0.02, seed 2, c_w=0.01, "
                       "c_m=0.1*s_target, c_n=c_m/a_t, N_k=N_l=8")
    launch_s = plate_ms / 1e3 / max(plate_launches, 1)
    out["kernel"] = {"main_kernels": plate_kinds, "launches": plate_launches,
                     "avg_launch_ms": launch_s * 1e3,
                     # the platelet kernel (one wavefront per cell) ran alone
                     "valu": recorded_platelet_valu(launch_s) if plate_kinds == 8 | 2 else None}
    return out

def n_scaling_extra(sizes=(1_000, 10_000, 100_000, 1_000_000, 10_000_000)):
    """The paper's efficiency protocol (Sec. 3.1, Fig. 2): an RSA start at
    f0 = 0.1 (srm_rsa), then SRM to f = 0.4 in 3D and 0.5 in 2D with a large
    swelling step (c_w = 0.02, c_m = 0.1 s_t), for N = 1e3 .. 1e7 in the unit
    box; wall times of both stages, and the fitted exponent of the total time
    in N for N >= 1e5 (the paper's optimised CPU code grows as N^1.15)."""
    import math

    import torch

    import paper_2605_18254_amd as srm
    import srm_inputs

    def one(dim, n, f_t):
        name = "spheres3d" if dim == 3 else "disks2d"
        w = srm_inputs.make(name, n=n, seed=1, f_target=f_t, c_w=0.02)
        r0 = srm_inputs.target_scale(dim, srm.BALL, 0.1, w.box, None, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start = srm.rsa(dim, srm.BALL, n, w.box[:dim], r0, 1, device=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = srm.SRM.from_workload(w, pos=start["pos"], s0=r0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st, info = g.run(2000)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g.close()
        return {"n": n, "rsa_s": t1 - t0, "rsa_candidates": start["drawn"],
                "rsa_batches": start["batches"], "rsa_rounds": start["rounds"],
                "init_s": t2 - t1, "srm_s": t3 - t2, "total_s": t3 - t0,
                "converged": st == 0, "sweeps": info["sweeps"], "passes": info["passes"],
                "srm_updates_per_s": info["updates"] / (t3 - t2)}

    def slope(rows):
        big = [r for r in rows if r["n"] >= 100_000]
        if len(big) < 2:
            return None
        xs = [math.log(r["n"]) for r in big]
        ys = [math.log(r["total_s"]) for r in big]
        mx, my = sum(xs) / len(xs), sum(ys) / len(ys)
        return sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sum((x - mx) ** 2 for x in xs)

    out = {"protocol": "RSA f0 0.1, then SRM (c_w 0.02, c_m 0.1 s_t) to f 0.4 (3D) / 0.5 (2D), "
                       "unit box, seed 1"}
    for dim, f_t in ((3, 0.4), (2, 0.5)):
        one(dim, 1_000, f_t)  # first launches load the kernels
        rows = []
        for n in sizes:
            rows.append(one(dim, n, f_t))
            _say(f"n-scaling {dim}D: {rows[-1]}")
        out[f"{dim}d"] = {"runs": rows, "time_exponent_n_ge_1e5": slope(rows)}
    return out


def platelet_protocol_extra(densities=(1.0, 2.0, 5.0), n=20_000, relax_sweeps=100):
    """The paper's platelet application (Sec. 3.3, Figs. 8-9): 20000 platelets
    (aspect ratio 100) at number density rho = N D^3 / L^3, grown with a
    larger swelling rate (c_w = 0.02, twice the default, with c_m = 0.1 a_t;
    smaller migration steps jam the run far below the target), then relaxed
    with zero swelling and a large migration step (c_m = 0.5 a_t) for
    `relax_sweeps` sweeps; the critical percolation distance delta_c / D of
    both states and of an RSA configuration at the same density (30
    bisection steps on the tunnelling gap)."""
    import math

    import torch

    import paper_2605_18254_amd as srm
    import srm_inputs

    def gap_c(g, diam):
        hi = 0.05 * diam
        while not g.percolation(hi) and hi < 8 * diam:
            hi *= 2.0
        return g.critical_gap(0.0, hi, 30) / diam if g.percolation(hi) else None

    rows = []
    for rho in densities:
        f = math.pi * rho / 400.0  # N pi (D/2)^2 (D/100) / L^3
        w = srm_inputs.make("platelets", n=n, seed=11, f_target=f, c_w=0.02, c_m_rel=0.1)
        diam = 2.0 * w.s_target
        g = srm.SRM.from_workload(w, device=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = g.run(2000)
        torch.cuda.synchronize()
        t_hoc = time.perf_counter() - t0
        hoc = gap_c(g, diam)
        pos, nrm, s_fin, t_fin = g.state()
        g.close()
        c_m = 0.5 * w.s_target
        r = srm.SRM(dim=3, n=n, s_target=w.s_target, c_w=0.0, c_m=c_m, n_k=8, n_l=8,
                    seed=w.seed, pos=pos, normals=nrm, shape=srm.PLATELET, c_n=c_m / w.s_target,
                    thick_ratio=w.thick_ratio, s0=s_fin, sweep0=t_fin)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(relax_sweeps):
            r.sweep()
        torch.cuda.synchronize()
        t_rel = time.perf_counter() - t0
        rel = gap_c(r, diam)
        overlaps = len(r.pairs(0.0))
        r.close()
        # the RSA configuration at the same number density (Fig. 9's reference)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start = srm.rsa(3, srm.PLATELET, n, (1.0, 1.0, 1.0), w.s_target, w.seed)
        t_rsa = time.perf_counter() - t0
        q = srm.SRM(dim=3, n=n, s_target=w.s_target, c_w=0.0, c_m=c_m, n_k=8, n_l=8,
                    seed=w.seed, pos=start["pos"], normals=start["normals"], shape=srm.PLATELET,
                    c_n=c_m / w.s_target, thick_ratio=w.thick_ratio, s0=w.s_target)
        rsa = gap_c(q, diam)
        q.close()
        rows.append({"rho": rho, "f": f, "converged": st == 0, "grow_sweeps": info["sweeps"],
                     "grow_s": t_hoc, "relax_s": t_rel, "delta_c_over_d_grown": hoc,
                     "delta_c_over_d_relaxed": rel, "overlapping_pairs": overlaps,
                     "rsa_s": t_rsa, "rsa_candidates": start["drawn"],
                     "delta_c_over_d_rsa": rsa})
        _say(f"platelet protocol: {rows[-1]}")
    return {"workload": f"{n} platelets, aspect ratio 100, seed 11; grown: c_w 0.02, c_m 0.1 a_t; "
                        f"relax: c_w 0, c_m 0.5 a_t, {relax_sweeps} sweeps; RSA at the same "
                        f"density", "runs": rows}

def spherodisk_protocol_extra(densities=(1.0, 2.0, 5.0), aspect_ratios=(100.0, 200.0),
                              n=20_000, relax_sweeps=100, dense_rho=30.0, dense_budget_s=60.0):
    """Sec. 3.3 with the paper's platelet model: 20000 spherodisks of aspect
    ratio 100 and 200 at number density rho = N D^3 / L^3, grown into
    house-of-cards networks (c_w = 0.02, c_m = 0.1 a_t) and relaxed (no
    swelling, c_m = 0.5 a_t, `relax_sweeps` sweeps); the critical
    percolation distance delta_c / D of both (hard core - soft shell: bonded
    when the core disks come within t + delta, 30 bisection steps).  Then
    the densification of Fig. 10: the relaxed aspect-ratio-100 state at the
    highest density swollen toward rho = `dense_rho` (c_w = 0.002,
    c_m = 0.2 a, N_l = 16) for at most `dense_budget_s` seconds."""
    import torch

    import paper_2605_18254_amd as srm
    import srm_inputs

    def gap_c(g, diam):
        hi = 0.05 * diam
        while not g.percolation(hi) and hi < 8 * diam:
            hi *= 2.0
        return g.critical_gap(0.0, hi, 30) / diam if g.percolation(hi) else None

    def make(ar, rho, **kw):
        tau = 1.0 / ar
        f = srm_inputs.spherodisk_volume_coeff(tau) * rho / 8.0  # N v (D/2)^3 / L^3
        return srm_inputs.make("spherodisks", n=n, seed=11, aspect_ratio=ar, f_target=f, **kw)

    rows, dense = [], None
    for ar in aspect_ratios:
        for rho in densities:
            w = make(ar, rho, c_w=0.02, c_m_rel=0.1)
            diam = 2.0 * w.s_target
            g = srm.SRM.from_workload(w, device=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, info = g.run(2000)
            torch.cuda.synchronize()
            t_hoc = time.perf_counter() - t0
            hoc = gap_c(g, diam)
            pos, nrm, s_fin, t_fin = g.state()
            g.close()
            c_m = 0.5 * w.s_target
            r = srm.SRM(dim=3, n=n, s_target=w.s_target, c_w=0.0, c_m=c_m, n_k=8, n_l=8,
                        seed=w.seed, pos=pos, normals=nrm, shape=srm.SPHERODISK,
                        c_n=c_m / w.s_target, thick_ratio=w.thick_ratio, s0=s_fin, sweep0=t_fin)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(relax_sweeps):
                r.sweep()
            torch.cuda.synchronize()
            t_rel = time.perf_counter() - t0
            rel = gap_c(r, diam)
            overlaps = len(r.pairs(0.0))
            rows.append({"aspect_ratio": ar, "rho": rho, "f": w.f_target, "converged": st == 0,
                         "grow_sweeps": info["sweeps"], "grow_s": t_hoc, "relax_s": t_rel,
                         "delta_c_over_d_grown": hoc, "delta_c_over_d_relaxed": rel,
                         "ratio_relaxed_to_grown": (rel / hoc) if (hoc and rel) else None,
                         "overlapping_pairs": overlaps})
            _say(f"spherodisk protocol: {rows[-1]}")
            if ar == aspect_ratios[0] and rho == max(densities) and dense_rho > rho:
                # densification: swell the relaxed state toward dense_rho
                pos, nrm, s_rel, t_rel_sw = r.state()
                s_dense = s_rel * (dense_rho / rho) ** (1.0 / 3.0)
                c_m = 0.2 * s_rel
                d = srm.SRM(dim=3, n=n, s_target=s_dense, c_w=0.002, c_m=c_m, n_k=8, n_l=16,
                            seed=w.seed, pos=pos, normals=nrm, shape=srm.SPHERODISK,
                            c_n=c_m / s_rel, thick_ratio=w.thick_ratio, s0=s_rel,
                            sweep0=t_rel_sw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sweeps = 0
                info_d = None
                while time.perf_counter() - t0 < dense_budget_s:
                    info_d = d.sweep()
                    sweeps += 1
                    if info_d["s"] == s_dense:
                        break
                torch.cuda.synchronize()
                s_now = info_d["s"] if info_d else s_rel
                dense = {"from_rho": rho, "target_rho": dense_rho,
                         "reached_rho": n * (2.0 * s_now) ** 3, "sweeps": sweeps,
                         "s": time.perf_counter() - t0, "fraction": info_d["fraction"] if info_d else None,
                         "overlapping_pairs": len(d.pairs(0.0)),
                         "delta_c_over_d": gap_c(d, 2.0 * s_now)}
                d.close()
                _say(f"spherodisk densification: {dense}")
            r.close()
    return {"workload": f"{n} spherodisks (outer diameter D, thickness D / aspect ratio), seed "
                        f"11; grown: c_w 0.02, c_m 0.1 a_t; relax: c_w 0, c_m 0.5 a_t, "
                        f"{relax_sweeps} sweeps", "runs": rows, "densification": dense}


def grad_extra(steps, steer_steps):
    """Soft g(r) (64 Gaussian bins up to 5r) + overlap energy, forward and
    hand-written backward, on N = 2e5 spheres grown by SRM to f = 0.30; then
    steering toward a Thomas-process target with an SRM sweep after each
    gradient step."""
    import torch

    import paper_2605_18254_amd as srm
    import srm_inputs
    from paper_2605_18254_amd import softrdf

    w = srm_inputs.make("softrdf")
    grow = srm.SRM.from_workload(w, device=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, run = grow.run(3000)
    torch.cuda.synchronize()
    dt_grow = time.perf_counter() - t0
    pos = torch.empty((3, w.n), dtype=torch.float64, device="cuda")
    grow.state_device(pos)
    r = w.s_target
    nb, r_c = 64, 5.0 * r
    counts, _ = grow.rdf(1, r_c + 4.0 * r_c / nb)
    pairs = int(counts.sum())
    grow.close()
    ws = softrdf.SoftRDF(w.n, 3, r_c, nbins=nb)
    radii = torch.full((w.n,), r, dtype=torch.float64, device="cuda")
    centres = (torch.arange(nb, dtype=torch.float64, device="cuda") + 0.5) * (r_c / nb)
    target = softrdf.thomas_g(centres, 1e-3 * w.n, 3.0 * r)
    target = torch.where(centres < 2 * r, torch.zeros_like(target), target)
    p = pos.clone().requires_grad_(True)

    def step():
        g, e = softrdf.soft_rdf(p, radii, ws)
        loss = ((g - target) ** 2).sum() + e
        p.grad = None
        loss.backward()
        return loss

    for _ in range(2):
        step()
    fwd0, fwd1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    fwd0.record()
    for _ in range(steps):
        softrdf.soft_rdf(p.detach(), radii, ws)
    fwd1.record()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(steps):
        loss = step()
    s1.record()
    torch.cuda.synchronize()
    ms_fwd = fwd0.elapsed_time(fwd1) / steps
    ms_step = s0.elapsed_time(s1) / steps
    # steering toward two readings of the clustered target: parents at
    # 1e-3 N per unit volume (literal; g(0) ~ 12.6, far beyond what a hard
    # sphere fluid at f = 0.30 can reach) and N / 50 parents (every point in
    # a cluster of 50; g(0) ~ 1.58)
    steer_out = {}
    for name, parents in (("parents_1e-3N", 1e-3 * w.n), ("parents_N_over_50", w.n / 50.0)):
        tgt = softrdf.thomas_g(centres, parents, 3.0 * r)
        tgt = torch.where(centres < 2 * r, torch.zeros_like(tgt), tgt)
        ctx = srm.SRM(dim=3, n=w.n, s_target=r, c_w=0.0, c_m=0.02 * r, n_k=8, n_l=8,
                      seed=w.seed, pos=pos, s0=r, sweep0=run["sweeps"])
        with torch.no_grad():
            g_first, _ = ws.forward(pos, radii)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = softrdf.steer(ctx, ws, tgt, r, steps=steer_steps, max_step=0.5 * w.c_m)
        torch.cuda.synchronize()
        dt_steer = time.perf_counter() - t0
        fin = torch.empty_like(pos)
        ctx.state_device(fin)
        _, _, s_fin, _ = ctx.state()
        g_last, _ = ws.forward(fin, radii)
        overlaps = len(ctx.pairs(0.0))
        ctx.close()
        losses = [h[0] for h in hist]
        pick = list(range(0, nb, 8))
        steer_out[name] = {
            "steps": steer_steps, "s": dt_steer, "ms_per_step": dt_steer / steer_steps * 1e3,
            "kept": sum(1 for h in hist[1:] if h[1]),
            "loss_first": losses[0], "loss_last": losses[-1],
            "loss_decrease": 1.0 - losses[-1] / losses[0],
            "monotone": all(b <= a for a, b in zip(losses, losses[1:])),
            "bins_r_over_radius": [round(float(centres[b] / r), 3) for b in pick],
            "g_target": [round(float(tgt[b]), 4) for b in pick],
            "g_first": [round(float(g_first[b]), 4) for b in pick],
            "g_last": [round(float(g_last[b]), 4) for b in pick],
            "s_over_s_target": s_fin / r, "overlapping_pairs": overlaps}
        _say(f"steering {name}: {steer_out[name]}")
    ws.close()
    return {
        "workload": "spheres3d N=2e5 f=0.30 seed 3; soft g(r) 64 bins on [0, 5r], h = bin "
                    "width, C2 taper to 5r+4h; target Thomas process (sigma 3r, two parent "
                    "densities), 0 below 2r; loss |g - target|^2 + E; steering: monotone "
                    "line search, largest move <= c_m/2, SRM sweep with c_w 0 and c_m 0.02 r "
                    "after each step",
        "grow_to_fraction": {"s": dt_grow, "sweeps": run["sweeps"],
                             "updates_per_s": run["updates"] / dt_grow,
                             "fraction": run["fraction"]},
        "pairs_within_cutoff": pairs,
        "ms_forward": ms_fwd, "ms_forward_backward": ms_step,
        "pair_evals_per_s": 3 * pairs / (ms_step / 1e3),
        "steer": steer_out,
    }


def plan_window(srm, w, steps, warmup):
    """The whole run, untimed, with trial moves counted per sweep: returns
    the per-sweep records, the sweep that reaches the target, and the first
    sweep (0-based) of the timed window, the `steps` sweeps ending there."""
    g = srm.SRM.from_workload(w, device=True)
    g.profile(enable=False, trials=True)
    rows, reached, prev = [], None, 0
    while True:
        info = g.sweep()
        tr = g.profile()["trials"]
        rows.append({"passes": info["passes_main"] + info["passes_shake"], "trials": tr - prev,
                     "committed": info["committed"], "fraction": info["fraction"],
                     "s": info["s"]})
        prev = tr
        if reached is None and info["s"] == w.s_target:
            reached = len(rows)
        if reached is not None and len(rows) >= max(reached, warmup + steps):
            break
        if len(rows) > 5000:
            raise RuntimeError("the run did not reach its target in 5000 sweeps")
    g.close()
    return rows, reached, max(warmup, reached - steps)


def at_target_extra(g, n, steps, torch):
    """`steps` further sweeps at the target fraction (swelling clamped, so
    every sweep only migrates and checks), timed the same way."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    passes = 0
    for _ in range(steps):
        info = g.sweep()
        passes += info["passes_main"] + info["passes_shake"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"sweeps": steps, "passes": passes, "s": dt, "updates_per_s": n * passes / dt,
            "fraction": info["fraction"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2605_18254_amd as srm
    import srm_inputs

    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        a = torch.empty(args.copy_probe_mib << 17, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    w = srm_inputs.make("spheres3d", n=args.n)
    rows, t_prefix = None, None
    if args.window_from:
        z = np.load(args.window_from)
        start, reached = int(z["start"]), int(z["reached"])
        g = srm.SRM.from_workload(w, device=True, pos=torch.from_numpy(z["pos"]).cuda(),
                                  s0=float(z["s"]), sweep0=int(z["t"]))
        frac_before = float(z["fraction"])
        _say(f"window replay from sweep {start}")
    else:
        rows, reached, start = plan_window(srm, w, args.steps, args.warmup)
        _say(f"target reached at sweep {reached}; window sweeps {start + 1}..{start + args.steps}")
        g = srm.SRM.from_workload(w, device=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(start):
            g.sweep()
        torch.cuda.synchronize()
        t_prefix = time.perf_counter() - t0
        frac_before = rows[start - 1]["fraction"] if start > 0 else 0.0
        if args.save_window:
            pos, _, s_w, t_w = g.state()
            np.savez(args.save_window, pos=pos, s=s_w, t=t_w, start=start, reached=reached,
                     fraction=frac_before)
    g.profile(enable=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    passes = shakes = 0
    phase_bytes = 0  # floor of the timed colour phases' real traffic
    for step in range(args.steps):
        info = g.sweep()
        npass = info["passes_main"] + info["passes_shake"]
        ncell = info["grid"][0] * info["grid"][1] * info["grid"][2]
        phase_bytes += npass * (8 * (PHASE_READ_PER_PARTICLE * w.n + PHASE_READ_PER_CELL * ncell)
                                + PHASE_WRITE_PER_OWN * w.n)
        passes += npass
        shakes += 0 if info["committed"] else 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = g.profile()
    final = info
    trials = None
    if rows is not None:
        win = rows[start:start + args.steps]
        if passes != sum(r["passes"] for r in win) or final["fraction"] != win[-1]["fraction"]:
            raise RuntimeError("the timed run departed from the planning run")
        trials = sum(r["trials"] for r in win)
    names = [] if (args.no_extras or args.window_from) else [x for x in args.extras.split(",") if x]
    at_target = None
    if "at_target" in names:
        g.profile(enable=False)
        at_target = at_target_extra(g, w.n, args.steps, torch)
        _say(f"at target: {at_target}")
    g.close()
    boundary = None if args.window_from else host_boundary(srm, w, torch)

    updates = w.n * passes
    value = updates / dt
    # dominant kernel: the migration colour phases
    mig_ms = prof["ms_migrate"]
    launches = max(prof["launches_migrate"], 1)
    # the colour phases' main kernel alone (the tiled kernel on this workload)
    avg_launch_s = prof["ms_migrate_main"] / 1e3 / launches
    main_name = {1: "k_migrate_tile<3,false>", 2: "k_migrate_wave<3,false>",
                 16: "k_migrate_tile_wide<3,false>",
                 32: "k_migrate_tile_mid<3,false>"}.get(prof["main_kernels"], "mixed")
    traffic = recorded_traffic(main_name)
    upd_per_launch = updates / launches
    bytes_per_launch = ALG_BYTES_PER_UPDATE * upd_per_launch
    achieved_gbs = bytes_per_launch / avg_launch_s / 1e9
    floor_per_launch = phase_bytes / launches
    sweep_bytes = ALG_BYTES_PER_UPDATE_SWEEP * updates
    window = {"first_sweep": start + 1, "last_sweep": start + args.steps,
              "target_reached_at_sweep": reached,
              "sweeps_past_target": max(0, start + args.steps - reached),
              "fraction_before": frac_before, "fraction_after": final["fraction"]}
    out = {
        "metric": "particle-updates/sec per SRM sweep (N=1e7 3D)",
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"spheres3d N={w.n} f_target=0.35 c_w=0.01 c_m=0.1*s_target "
                               "N_k=N_l=8 seed=1; timed: the sweeps ending at the target",
                   "n": w.n, "dim": 3, "passes": passes, "shakes": shakes,
                   "final_fraction": final["fraction"], "final_sweep": final["sweep"],
                   "grid": list(final["grid"]), "window": window},
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "kernel": main_name, "avg_launch_ms": avg_launch_s * 1e3,
                     "launches": launches, "alg_bytes_per_launch": bytes_per_launch,
                     "alg_bytes_per_update": ALG_BYTES_PER_UPDATE,
                     "updates_per_launch": upd_per_launch,
                     "phase_floor_bytes_per_launch": floor_per_launch,
                     "phase_floor_gbs": floor_per_launch / avg_launch_s / 1e9,
                     "traffic_source": traffic["source"] if traffic else None},
        "valu": recorded_valu(main_name, avg_launch_s),
        "trial_moves_per_s": None if trials is None else trials / dt,
        "trials_per_update": None if trials is None else trials / max(updates, 1),
        "kernel_ms": {"bin": prof["ms_bin"], "migrate": mig_ms, "check": prof["ms_check"],
                      "wall": dt * 1e3},
        "hbm_sweep": {"alg_bytes_per_update": ALG_BYTES_PER_UPDATE_SWEEP,
                      "alg_bytes": sweep_bytes, "achieved_gbs": sweep_bytes / dt / 1e9,
                      "frac": sweep_bytes / dt / 1e9 / HBM_PEAK_GBS},
    }
    if t_prefix is not None and start + args.steps == reached:
        run_passes = sum(r["passes"] for r in rows[:reached])
        out["whole_run"] = {"sweeps": reached, "passes": run_passes, "s": t_prefix + dt,
                            "updates_per_s": w.n * run_passes / (t_prefix + dt)}
    if boundary is not None:
        boundary["value_pcie_inclusive"] = updates / (dt + boundary["init_from_host_s"] +
                                                      boundary["state_to_host_s"])
        out["host_boundary"] = boundary
    if names:
        runs = {"n_scaling": n_scaling_extra,
                "platelets": lambda: platelet_extra(3000),
                "platelet_protocol": platelet_protocol_extra,
                "spherodisk_protocol": spherodisk_protocol_extra,
                "batched": lambda: batched_extra(args.batch_sweeps),
                "gradient": lambda: grad_extra(20, 100)}
        unknown = [x for x in names if x not in runs and x != "at_target"]
        if unknown:
            raise SystemExit(f"unknown extras: {unknown}")
        out["extras"] = {x: runs[x]() for x in names if x != "at_target"}
        if at_target is not None:
            out["extras"]["at_target"] = at_target
    if not args.no_cpu_baseline and not args.window_from:
        n_sub = args.cpu_n or int(round(1e7 * (32.0 / 178.0) ** 3))
        out["cpu_baseline"] = cpu_baseline(args.steps, args.warmup, n_sub)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
