"""SRM sweep throughput on one MI355X.

Workload: 3D periodic unit cube, N = 1e7 monodisperse spheres, positions
uniform (Philox seed 1), radii swelling from 0 by c_w = 0.01 s_target per
sweep to the target volume fraction 0.35, migration step c_m = 0.1 s_target,
N_k = N_l = 8.  A step is one SRM sweep (Algorithm 1 iteration: swell, then
bin + migration pass + global check until a pass leaves no overlap, or a
shake).  Inputs are resident in HBM before timing starts.

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
# Vector ALU issue rate of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic HBM bytes per particle update (3D spheres, FP64 SoA, int32 ids).
MIGRATE_BYTES = 24 + 4 + 24 + 1 + 4   # own position, id, new position, accept code, cell range
BIN_BYTES = (24 + 4 + 4 + 4) + (24 + 4 + 4 + 4 + 4 + 24 + 4) + 4  # count pass + scatter + fix-up


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=110)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fraction", type=float, default=0.25,
                    help="fraction of the cell layers the oracle sample covers")
    return ap.parse_args()


def cpu_baseline(w, frac):
    """The oracle (single-threaded C) on a bounded sample of the same
    workload: the first migration pass of sweep 1, restricted to the cells of
    the first `frac` of the z layers."""
    import numpy as np
    import oracle

    o = oracle.Oracle.from_workload(w)
    s1 = o.swell(o.s)
    na, inv = o.grid_for_scale(s1)
    nz = int(na[2])
    layers = max(1, int(nz * frac))
    ncell = int(na[0] * na[1] * na[2])
    mask = np.zeros(ncell, dtype=np.uint8)
    mask[: int(na[0] * na[1] * layers)] = 1
    cell = o.bin(na, inv)
    updates = int(mask[cell].sum())
    t0 = time.perf_counter()
    o.pass_(na, inv, s1, 0, 1, mask=mask)
    dt = time.perf_counter() - t0
    return dict(value=updates / dt, unit="particle-updates/s", cores=1, kind="oracle",
                sample=f"sweep 1, pass 1 of the same N={w.n} workload restricted to "
                       f"{layers}/{nz} cell layers ({updates} particle updates, "
                       f"{dt:.1f} s incl. binning all N), single-threaded C oracle")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note only)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2605_18254_amd as srm
    import srm_inputs

    torch.cuda.set_device(0)
    w = srm_inputs.make("spheres3d", n=args.n)
    g = srm.SRM.from_workload(w, device=True)
    for _ in range(args.warmup):
        g.sweep()
    g.profile(enable=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    passes = shakes = 0
    for _ in range(args.steps):
        info = g.sweep()
        passes += info["passes_main"] + info["passes_shake"]
        shakes += 0 if info["committed"] else 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = g.profile()
    final = info
    g.close()

    updates = w.n * passes
    value = updates / dt
    # dominant kernel: the migration colour phases
    mig_ms = prof["ms_migrate"]
    launches = max(prof["launches_migrate"], 1)
    avg_launch_s = mig_ms / 1e3 / launches
    upd_per_launch = updates / launches
    achieved_gbs = MIGRATE_BYTES * upd_per_launch / avg_launch_s / 1e9
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
                               "N_k=N_l=8 seed=1", "n": w.n, "dim": 3,
                   "passes": passes, "shakes": shakes, "final_fraction": final["fraction"],
                   "final_sweep": final["sweep"], "grid": list(final["grid"])},
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_migrate_ball<3,false> (one colour phase per launch)",
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "bytes_per_update": MIGRATE_BYTES},
        "kernel_ms": {"bin": prof["ms_bin"], "migrate": mig_ms, "check": prof["ms_check"],
                      "wall": dt * 1e3},
        "hbm_sweep": {"bytes_per_update": MIGRATE_BYTES + BIN_BYTES,
                      "achieved_gbs": (MIGRATE_BYTES + BIN_BYTES) * updates / dt / 1e9,
                      "frac": (MIGRATE_BYTES + BIN_BYTES) * updates / dt / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_fraction)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
