"""Python binding of libsrm, the MI355X (gfx950) Swelling and Random Migration
library.

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels behind the C ABI of ``include/srm.h``.  Inputs may be numpy arrays
(host) or torch CUDA tensors (device memory of the current GPU); with torch
tensors the library runs on torch's current stream.  There is no CPU
fallback: loading fails loudly when ``libsrm.so`` is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

__all__ = ["SRM", "SrmError", "rsa", "lib", "LIB_PATH", "BALL", "PLATELET", "SPHERODISK",
           "MAIN", "SHAKE"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libsrm.so")

BALL, PLATELET, SPHERODISK = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
MAIN, SHAKE = 0, 1
OK, EINVAL, ENOMEM, EDEVICE, EOVERLAP, ENOTCONV, ECAPACITY = 0, -1, -2, -3, -4, -5, -6

SYMBOLS = ["srm_init", "srm_sweep", "srm_run_to_fraction", "srm_pairs", "srm_rdf", "srm_nearest",
           "srm_percolation", "srm_critical_gap", "srm_rsa",
           "srm_get_state", "srm_free", "srm_last_error", "srm_grid", "srm_cells", "srm_pass",
           "srm_last_acc", "srm_set_state", "srm_softrdf_create", "srm_softrdf_forward",
           "srm_softrdf_backward", "srm_softrdf_free", "srm_softrdf_forward_static", "srm_profile_enable", "srm_profile_read",
           "srm_batch_init", "srm_batch_configure", "srm_batch_run", "srm_batch_get",
           "srm_batch_free", "srm_batch_last_error", "srm_debug_fp",
           "srm_debug_philox", "srm_debug_unitvec"]


class SrmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"srm status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("shape", C.c_int32), ("n", C.c_int64),
                ("box", C.c_double * 3), ("s_target", C.c_double), ("c_w", C.c_double),
                ("c_m", C.c_double), ("c_n", C.c_double), ("thick_ratio", C.c_double),
                ("n_k", C.c_int32), ("n_l", C.c_int32), ("seed", C.c_uint64)]


class SweepInfo(C.Structure):
    _fields_ = [("committed", C.c_int32), ("passes_main", C.c_int32),
                ("passes_shake", C.c_int32), ("grid", C.c_int32 * 3), ("sweep", C.c_int64),
                ("s", C.c_double), ("fraction", C.c_double), ("n_failed_last", C.c_int64)]


class Profile(C.Structure):
    _fields_ = [("ms_bin", C.c_double), ("ms_migrate", C.c_double), ("ms_check", C.c_double),
                ("bins", C.c_int64), ("launches_migrate", C.c_int64), ("passes", C.c_int64),
                ("checks", C.c_int64), ("ms_migrate_main", C.c_double),
                ("main_kernels", C.c_int64), ("trials", C.c_int64)]


class RsaInfo(C.Structure):
    _fields_ = [("drawn", C.c_int64), ("placed", C.c_int64), ("batches", C.c_int32),
                ("rounds", C.c_int32)]


class RunInfo(C.Structure):
    _fields_ = [("sweeps", C.c_int64), ("passes", C.c_int64), ("shakes", C.c_int64),
                ("updates", C.c_int64), ("s", C.c_double), ("fraction", C.c_double)]


_lib = None


def lib():
    """Load libsrm.so (built by ``paper_2605_18254_amd/build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2605_18254_amd/build.py "
                          "(there is no CPU fallback)")
    # One HIP runtime per process: when torch is installed its bundled
    # libamdhip64 is loaded first, and libsrm's dependency (same soname)
    # resolves to it instead of a second copy from /opt/rocm.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.srm_init.argtypes = [C.POINTER(Params), vp, vp, vp, C.c_double, C.c_int64, C.c_int32, vp,
                           C.POINTER(vp)]
    L.srm_sweep.argtypes = [vp, C.POINTER(SweepInfo)]
    L.srm_run_to_fraction.argtypes = [vp, C.c_double, C.c_int32, C.POINTER(RunInfo)]
    L.srm_pairs.argtypes = [vp, C.c_double, C.c_int64, vp, C.POINTER(C.c_int64), C.c_int32]
    L.srm_rdf.argtypes = [vp, C.c_int32, C.c_double, C.POINTER(C.c_uint64), dp]
    L.srm_nearest.argtypes = [vp, C.c_double, dp, C.c_int32, C.POINTER(C.c_uint64)]
    L.srm_percolation.argtypes = [vp, C.c_double, C.POINTER(C.c_int32)]
    L.srm_critical_gap.argtypes = [vp, C.c_double, C.c_double, C.c_int32, dp]
    L.srm_get_state.argtypes = [vp, vp, vp, dp, C.POINTER(C.c_int64), C.c_int32]
    L.srm_rsa.argtypes = [C.c_int32, C.c_int32, C.c_int64, dp, C.c_double, C.c_uint64, C.c_int64,
                          C.c_int64, vp, vp, vp, C.c_int32, vp, C.POINTER(RsaInfo)]
    L.srm_free.argtypes = [vp]
    L.srm_last_error.argtypes = []
    L.srm_last_error.restype = C.c_char_p
    L.srm_grid.argtypes = [vp, C.c_double, C.POINTER(C.c_int32)]
    L.srm_cells.argtypes = [vp, C.c_double, C.POINTER(C.c_int32)]
    L.srm_pass.argtypes = [vp, C.c_double, C.c_double, C.c_int32, C.c_int32,
                           C.POINTER(C.c_uint8), C.POINTER(C.c_int32)]
    L.srm_last_acc.argtypes = [vp, C.POINTER(C.c_uint8)]
    L.srm_profile_enable.argtypes = [vp, C.c_int32]
    L.srm_profile_read.argtypes = [vp, C.POINTER(Profile)]
    L.srm_debug_fp.argtypes = [dp, dp, C.c_int64, dp, dp]
    L.srm_debug_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.c_int64,
                                   C.POINTER(C.c_uint32)]
    L.srm_debug_unitvec.argtypes = [C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.c_double, C.c_int64, dp]
    for name in SYMBOLS:
        if name != "srm_last_error":
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def _check(st: int):
    if st != OK:
        raise SrmError(st, lib().srm_last_error().decode())


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a, mem_kind, dtype):
    """(pointer, keepalive) for a numpy array or a torch CUDA tensor."""
    if a is None:
        return None, None
    if mem_kind == MEM_DEVICE:
        a = a.contiguous()
        return C.c_void_p(a.data_ptr()), a
    a = np.ascontiguousarray(a, dtype=dtype)
    return C.c_void_p(a.ctypes.data), a


def debug_fp(a: np.ndarray, b: np.ndarray):
    """Device sqrt(a) and a / b (float64), for checking correct rounding."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    sq, dv = np.empty_like(a), np.empty_like(a)
    dp = C.POINTER(C.c_double)
    _check(lib().srm_debug_fp(a.ctypes.data_as(dp), b.ctypes.data_as(dp), a.size,
                              sq.ctypes.data_as(dp), dv.ctypes.data_as(dp)))
    return sq, dv


def debug_philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Device Philox4x32-10 for ctr (n, 4) and key (n, 2) uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty_like(ctr)
    up = C.POINTER(C.c_uint32)
    _check(lib().srm_debug_philox(ctr.ctypes.data_as(up), key.ctypes.data_as(up), ctr.shape[0],
                                  out.ctypes.data_as(up)))
    return out


def debug_unitvec(dim, seed, t, kind, k, l, stream, length, n) -> np.ndarray:
    """Device trial vectors for particle ids 0..n-1, shape (n, 3)."""
    out = np.empty((n, 3), dtype=np.float64)
    word = (int(kind) << 31) | (int(k) << 16) | (int(l) << 8)
    _check(lib().srm_debug_unitvec(int(dim), int(seed), int(t), word, int(stream), float(length),
                                   int(n), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def rsa(dim, shape, n, box, radius, seed, max_candidates=None, batch=0, device=False):
    """Random sequential addition of n equal particles on the GPU (srm_rsa).

    Returns a dict: status (OK or ENOTCONV), pos (dim, n), normals (3, n) or
    None, src (n,) candidate indices, drawn, placed, batches, rounds.  With
    device=True the arrays are torch CUDA tensors written on torch's current
    stream; otherwise numpy arrays.  Other errors raise SrmError."""
    dim, shape, n = int(dim), int(shape), int(n)
    box3 = (C.c_double * 3)(*(list(box) + [1.0] * (3 - len(box))))
    if max_candidates is None:
        max_candidates = 1000 * max(n, 1)
    stream = None
    if device:
        import torch
        pos = torch.zeros((dim, n), dtype=torch.float64, device="cuda")
        nrm = torch.zeros((3, n), dtype=torch.float64, device="cuda") if shape == PLATELET else None
        src = torch.zeros(n, dtype=torch.int64, device="cuda")
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        ptr = lambda a: None if a is None else C.c_void_p(a.data_ptr())  # noqa: E731
        kind = MEM_DEVICE
    else:
        pos = np.zeros((dim, n))
        nrm = np.zeros((3, n)) if shape == PLATELET else None
        src = np.zeros(n, dtype=np.int64)
        ptr = lambda a: None if a is None else C.c_void_p(a.ctypes.data)  # noqa: E731
        kind = MEM_HOST
    info = RsaInfo()
    st = lib().srm_rsa(dim, shape, n, box3, float(radius), int(seed), int(max_candidates),
                       int(batch), ptr(pos), ptr(nrm), ptr(src), kind, stream, C.byref(info))
    if st not in (OK, ENOTCONV):
        _check(st)
    return dict(status=st, pos=pos, normals=nrm, src=src, drawn=info.drawn, placed=info.placed,
                batches=info.batches, rounds=info.rounds)


class SRM:
    """One SRM context (a periodic box of particles on the GPU).

    ``pos`` has shape (dim, n) (structure of arrays, particle-id order);
    ``normals`` (3, n) for platelets; ``rho`` (n,) shape radii or None.
    """

    def __init__(self, *, dim, n, s_target, c_w, c_m, n_k, n_l, seed, pos,
                 box=(1.0, 1.0, 1.0), rho=None, normals=None, shape=BALL, c_n=0.0,
                 thick_ratio=0.0, s0=0.0, sweep0=0, stream=None):
        L = lib()
        p = Params()
        p.dim, p.shape, p.n = int(dim), int(shape), int(n)
        box3 = list(box) + [1.0] * (3 - len(box))
        for a in range(3):
            p.box[a] = float(box3[a])
        p.s_target, p.c_w, p.c_m, p.c_n = float(s_target), float(c_w), float(c_m), float(c_n)
        p.thick_ratio = float(thick_ratio)
        p.n_k, p.n_l, p.seed = int(n_k), int(n_l), int(seed)
        self.params = p
        self.dim, self.n = int(dim), int(n)
        self.plate = int(shape) in (PLATELET, SPHERODISK)
        device = _is_torch(pos)
        self.mem_kind = MEM_DEVICE if device else MEM_HOST
        if device:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
            pos = pos.to(torch.float64)
            rho = None if rho is None else rho.to(torch.float64)
            normals = None if normals is None else normals.to(torch.float64)
        pp, k1 = _ptr(pos, self.mem_kind, np.float64)
        rp, k2 = _ptr(rho, self.mem_kind, np.float64)
        np_, k3 = _ptr(normals, self.mem_kind, np.float64)
        self._stream = C.c_void_p(stream) if stream else None
        ctx = C.c_void_p()
        _check(L.srm_init(C.byref(p), pp, rp, np_, float(s0), int(sweep0), self.mem_kind,
                          self._stream, C.byref(ctx)))
        self._ctx = ctx
        del k1, k2, k3

    @classmethod
    def from_workload(cls, w, device: bool = False, **over):
        pos, rho, nrm = w.pos, w.rho, w.normals
        if device:
            import torch
            pos = torch.from_numpy(pos).cuda()
            rho = None if rho is None else torch.from_numpy(rho).cuda()
            nrm = None if nrm is None else torch.from_numpy(nrm).cuda()
        kw = dict(dim=w.dim, n=w.n, box=w.box, s_target=w.s_target, c_w=w.c_w, c_m=w.c_m,
                  n_k=w.n_k, n_l=w.n_l, seed=w.seed, pos=pos, rho=rho, normals=nrm,
                  shape=w.shape, c_n=w.c_n, thick_ratio=w.thick_ratio, s0=w.s0,
                  sweep0=w.sweep0)
        kw.update(over)
        return cls(**kw)

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            lib().srm_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- Algorithm 1 ---------------------------------------------------------
    def sweep(self) -> dict:
        info = SweepInfo()
        _check(lib().srm_sweep(self._ctx, C.byref(info)))
        return dict(committed=bool(info.committed), passes_main=info.passes_main,
                    passes_shake=info.passes_shake, grid=tuple(info.grid), sweep=info.sweep,
                    s=info.s, fraction=info.fraction, n_failed_last=info.n_failed_last)

    def run(self, max_sweeps: int, f_target: float = 0.0):
        """Sweep until the volume fraction reaches f_target (<= 0: until
        s == s_target); returns (status, info dict)."""
        info = RunInfo()
        st = lib().srm_run_to_fraction(self._ctx, float(f_target), int(max_sweeps),
                                       C.byref(info))
        if st not in (OK, ENOTCONV):
            _check(st)
        return st, dict(sweeps=info.sweeps, passes=info.passes, shakes=info.shakes,
                        updates=info.updates, s=info.s, fraction=info.fraction)

    def state(self):
        """(pos (dim, n), normals (3, n) or None, s, sweep) in id order, host."""
        pos = np.empty((self.dim, self.n), dtype=np.float64)
        nrm = np.empty((3, self.n), dtype=np.float64) if self.plate else None
        s, t = C.c_double(), C.c_int64()
        _check(lib().srm_get_state(self._ctx, C.c_void_p(pos.ctypes.data),
                                   C.c_void_p(nrm.ctypes.data) if nrm is not None else None,
                                   C.byref(s), C.byref(t), MEM_HOST))
        return pos, nrm, s.value, t.value

    def state_device(self, out_pos, out_normals=None):
        """Write the state into torch CUDA tensors (dim, n) [and (3, n)]."""
        s, t = C.c_double(), C.c_int64()
        _check(lib().srm_get_state(self._ctx, C.c_void_p(out_pos.data_ptr()),
                                   C.c_void_p(out_normals.data_ptr()) if out_normals is not None
                                   else None, C.byref(s), C.byref(t), MEM_DEVICE))
        return s.value, t.value

    # -- step level ----------------------------------------------------------
    def grid(self, s: float):
        na = (C.c_int32 * 3)()
        _check(lib().srm_grid(self._ctx, float(s), na))
        return tuple(na)

    def cells(self, grid_s: float) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        _check(lib().srm_cells(self._ctx, float(grid_s),
                               out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def pass_(self, grid_s: float, radius_s: float, kind: int, k: int):
        acc = np.empty(self.n, dtype=np.uint8)
        ov = C.c_int32()
        _check(lib().srm_pass(self._ctx, float(grid_s), float(radius_s), int(kind), int(k),
                              acc.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(ov)))
        return acc, bool(ov.value)

    def last_acc(self) -> np.ndarray:
        acc = np.empty(self.n, dtype=np.uint8)
        _check(lib().srm_last_acc(self._ctx, acc.ctypes.data_as(C.POINTER(C.c_uint8))))
        return acc

    def profile(self, enable: Optional[bool] = None, trials: bool = False) -> dict:
        """Read the device-time profile; enable=True/False (re)starts it
        (trials=True also counts trial moves, which adds a reduction per
        pass)."""
        if enable is not None:
            _check(lib().srm_profile_enable(self._ctx, (1 if enable else 0) | (2 if trials else 0)))
        pr = Profile()
        _check(lib().srm_profile_read(self._ctx, C.byref(pr)))
        return {name: getattr(pr, name) for name, _ in Profile._fields_}

    # -- analysis ------------------------------------------------------------
    def pairs(self, gap: float = 0.0) -> np.ndarray:
        cnt = C.c_int64()
        st = lib().srm_pairs(self._ctx, float(gap), 0, None, C.byref(cnt), MEM_HOST)
        if st not in (OK, ECAPACITY):
            _check(st)
        out = np.empty((max(cnt.value, 1), 2), dtype=np.int32)
        _check(lib().srm_pairs(self._ctx, float(gap), cnt.value, C.c_void_p(out.ctypes.data),
                               C.byref(cnt), MEM_HOST))
        return out[: cnt.value]

    def nearest(self, r_max: float, nbins: int = 0):
        """(distance to the nearest other particle by id, +inf if none within
        r_max; histogram of those distances over nbins bins on [0, r_max),
        or None when nbins is 0)."""
        dist = np.empty(self.n, dtype=np.float64)
        hist = np.zeros(max(nbins, 1), dtype=np.uint64)
        _check(lib().srm_nearest(self._ctx, float(r_max),
                                 dist.ctypes.data_as(C.POINTER(C.c_double)), int(nbins),
                                 hist.ctypes.data_as(C.POINTER(C.c_uint64)) if nbins > 0
                                 else None))
        return dist, (hist if nbins > 0 else None)

    def percolation(self, gap: float) -> int:
        """Bit a set when a cluster of particles grown by `gap` wraps around
        the box along axis a."""
        m = C.c_int32()
        _check(lib().srm_percolation(self._ctx, float(gap), C.byref(m)))
        return m.value

    def critical_gap(self, lo: float, hi: float, iters: int = 40) -> float:
        """Smallest percolating gap found by bisection between lo (not
        percolating) and hi (percolating)."""
        out = C.c_double()
        _check(lib().srm_critical_gap(self._ctx, float(lo), float(hi), int(iters), C.byref(out)))
        return out.value

    def rdf(self, nbins: int, r_max: float):
        counts = np.zeros(nbins, dtype=np.uint64)
        g = np.zeros(nbins, dtype=np.float64)
        _check(lib().srm_rdf(self._ctx, int(nbins), float(r_max),
                             counts.ctypes.data_as(C.POINTER(C.c_uint64)),
                             g.ctypes.data_as(C.POINTER(C.c_double))))
        return counts, g
