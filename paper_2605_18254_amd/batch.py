"""Batched SRM ensembles: many independent RVEs advanced together on one GPU.

``Batch`` wraps the ``srm_batch_*`` entry points: the RVEs' Algorithm 1
state lives on the device and a captured hipGraph of batched kernels moves
every unfinished RVE by a few passes per replay.  ``autotune`` picks the
launch shape (pass slots per replay, migration block size) by timing short
runs; the shape never changes results.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import time
from typing import Optional, Sequence

import numpy as np

from . import ENOTCONV, OK, Params, SrmError, lib

BATCH_SYMBOLS = ["srm_batch_init", "srm_batch_configure", "srm_batch_run", "srm_batch_get",
                 "srm_batch_free", "srm_batch_last_error"]


class BatchInfo(C.Structure):
    _fields_ = [("replays", C.c_int64), ("slots", C.c_int64), ("converged", C.c_int32),
                ("not_converged", C.c_int32), ("passes", C.c_int64), ("updates", C.c_int64)]


def _bind():
    L = lib()
    if getattr(L, "_batch_bound", False):
        return L
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.srm_batch_init.argtypes = [C.c_int32, C.POINTER(Params), dp, dp, C.POINTER(vp)]
    L.srm_batch_configure.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    L.srm_batch_run.argtypes = [vp, C.c_int32, C.POINTER(BatchInfo)]
    L.srm_batch_get.argtypes = [vp, C.c_int32, dp, dp, C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64)]
    L.srm_batch_free.argtypes = [vp]
    L.srm_batch_last_error.restype = C.c_char_p
    for f in BATCH_SYMBOLS[:-1]:
        getattr(L, f).restype = C.c_int32
    L._batch_bound = True
    return L


def _bcheck(st):
    if st not in (OK,):
        raise SrmError(st, _bind().srm_batch_last_error().decode())


class Batch:
    """An ensemble of ball RVEs (``srm_inputs.Workload`` objects, all with or
    all without shape radii)."""

    def __init__(self, workloads: Sequence):
        L = _bind()
        self.members = list(workloads)
        count = len(self.members)
        params = (Params * count)()
        poly = self.members[0].rho is not None
        for r, w in enumerate(self.members):
            if (w.rho is not None) != poly:
                raise ValueError("all RVEs need shape radii, or none")
            p = params[r]
            p.dim, p.shape, p.n = w.dim, 0, w.n
            for a in range(3):
                p.box[a] = float(w.box[a]) if a < len(w.box) else 1.0
            p.s_target, p.c_w, p.c_m, p.c_n = w.s_target, w.c_w, w.c_m, 0.0
            p.thick_ratio = 0.0
            p.n_k, p.n_l, p.seed = w.n_k, w.n_l, w.seed
        pos = np.ascontiguousarray(np.concatenate([np.ascontiguousarray(w.pos).ravel()
                                                   for w in self.members]))
        rho = (np.ascontiguousarray(np.concatenate([w.rho for w in self.members]))
               if poly else None)
        dp = C.POINTER(C.c_double)
        ctx = C.c_void_p()
        _bcheck(L.srm_batch_init(count, params, pos.ctypes.data_as(dp),
                                 rho.ctypes.data_as(dp) if rho is not None else None,
                                 C.byref(ctx)))
        self._ctx = ctx

    def configure(self, slots: int, block: int, wave_occupancy: int = 3):
        """Schedule: pass slots per graph replay, threads per block of the
        sparse-grid kernels (a group of lanes a cell), and the occupancy from
        which a grid is migrated with one wavefront per cell."""
        _bcheck(_bind().srm_batch_configure(self._ctx, int(slots), int(block),
                                            int(wave_occupancy)))

    def run(self, max_sweeps: int):
        info = BatchInfo()
        st = _bind().srm_batch_run(self._ctx, int(max_sweeps), C.byref(info))
        if st not in (OK, ENOTCONV):
            _bcheck(st)
        return st, {name: getattr(info, name) for name, _ in BatchInfo._fields_}

    def get(self, r: int):
        w = self.members[r]
        pos = np.empty((w.dim, w.n), dtype=np.float64)
        s, t, passes = C.c_double(), C.c_int64(), C.c_int64()
        _bcheck(_bind().srm_batch_get(self._ctx, int(r),
                                      pos.ctypes.data_as(C.POINTER(C.c_double)), C.byref(s),
                                      C.byref(t), C.byref(passes)))
        return pos, s.value, t.value, passes.value

    def close(self):
        if getattr(self, "_ctx", None):
            _bind().srm_batch_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(workloads: Sequence, sweeps: int = 6, cache: Optional[str] = None,
             slots=(1, 2, 4, 8), blocks=(64, 128, 256), wave_occupancy=(3,)):
    """Time a few sweeps of the ensemble for each schedule (pass slots per
    replay, block size, wavefront-per-cell occupancy threshold) and return
    the fastest (slots, block, wave_occupancy); results are cached by
    ensemble size in `cache` (JSON).  Every schedule gives bit-identical
    results, so the choice only affects speed."""
    key = f"{len(workloads)}:{sum(w.n for w in workloads)}:" \
          f"{sum(w.n for w in workloads if w.dim == 3)}"
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return tuple(table[key])
    best, best_t = None, None
    for sl in slots:
        for bl in blocks:
            for wo in wave_occupancy:
                b = Batch(workloads)
                b.configure(sl, bl, wo)
                t0 = time.perf_counter()
                b.run(sweeps)
                dt = time.perf_counter() - t0
                b.close()
                if best_t is None or dt < best_t:
                    best, best_t = (sl, bl, wo), dt
    if cache:
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        table[key] = list(best)
        with open(cache, "w") as f:
            json.dump(table, f)
    return best
