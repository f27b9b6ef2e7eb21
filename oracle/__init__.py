"""CPU oracle of the SRM sweep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it.

The arithmetic lives in ``srm_oracle.c`` (plain sequential C, compiled with
``-O2 -ffp-contract=off -fno-fast-math``); this module compiles it with gcc
and marshals numpy arrays through ctypes.  States are held in particle-id
order, positions as (n, 3) float64 rows (z = 0 in 2D).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srm_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

MAIN = 0
SHAKE = 1
OK = 0
ENOTCONV = -5

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wno-unused-function"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc; returns the library path."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("shape", C.c_int32), ("n", C.c_int64),
                ("box", C.c_double * 3), ("s_target", C.c_double), ("c_w", C.c_double),
                ("c_m", C.c_double), ("c_n", C.c_double), ("thick_ratio", C.c_double),
                ("n_k", C.c_int32), ("n_l", C.c_int32), ("seed", C.c_uint64)]


class State(C.Structure):
    _fields_ = [("p", Params), ("pos", C.POINTER(C.c_double)), ("nrm", C.POINTER(C.c_double)),
                ("rho", C.POINTER(C.c_double)), ("s", C.c_double), ("t", C.c_int64)]


class SoftParams(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nbins", C.c_int32), ("box", C.c_double * 3),
                ("r_c", C.c_double), ("kappa", C.c_double)]


class SweepInfo(C.Structure):
    _fields_ = [("committed", C.c_int32), ("passes_main", C.c_int32),
                ("passes_shake", C.c_int32), ("pad", C.c_int32), ("na", C.c_int64 * 3),
                ("s_new", C.c_double), ("n_failed_last", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.o_philox4x32.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.o_unitvec.argtypes = [C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                                C.c_uint32, C.c_uint32, C.c_uint64, C.c_double, dp]
        L.o_unitvec.restype = C.c_int
        L.o_grid.argtypes = [C.POINTER(Params), C.c_double, C.POINTER(C.c_int64), dp]
        L.o_bin.argtypes = [C.POINTER(Params), C.POINTER(C.c_int64), dp, dp,
                            C.POINTER(C.c_int64)]
        L.o_pass.argtypes = [C.POINTER(State), C.POINTER(C.c_int64), dp, C.c_double,
                             C.c_uint32, C.c_uint32, C.POINTER(C.c_uint8),
                             C.POINTER(C.c_uint8), C.POINTER(C.c_int32)]
        L.o_overlap.argtypes = [C.POINTER(State), C.POINTER(C.c_int64), dp, C.c_double,
                                C.POINTER(C.c_int32)]
        L.o_rho_max.argtypes = [C.POINTER(State)]
        L.o_rho_max.restype = C.c_double
        L.o_swell.argtypes = [C.POINTER(Params), C.c_double]
        L.o_swell.restype = C.c_double
        L.o_sweep.argtypes = [C.POINTER(State), C.POINTER(SweepInfo), C.POINTER(C.c_uint8)]
        L.o_run_to.argtypes = [C.POINTER(State), C.c_double, C.c_int32, C.POINTER(C.c_int64),
                               C.POINTER(C.c_int64)]
        L.o_run.argtypes = [C.POINTER(State), C.c_int32, C.POINTER(C.c_int64),
                            C.POINTER(C.c_int64)]
        L.o_pairs_brute.argtypes = [C.POINTER(State), C.c_double, C.c_double, C.c_int64,
                                    C.POINTER(C.c_int32)]
        L.o_pairs_brute.restype = C.c_int64
        L.o_rdf_brute.argtypes = [C.POINTER(State), C.c_int32, C.c_double,
                                  C.POINTER(C.c_uint64)]
        L.o_nearest_brute.argtypes = [C.POINTER(State), C.c_double, dp]
        L.o_percolation.argtypes = [C.POINTER(State), C.c_double, C.c_double,
                                    C.POINTER(C.c_int32)]
        L.o_disks_intersect.argtypes = [dp, dp, C.c_double, dp, dp, C.c_double, dp]
        L.o_softrdf_fwd.argtypes = [C.POINTER(SoftParams), C.c_int64, dp, dp, dp, dp]
        L.o_softrdf_grad.argtypes = [C.POINTER(SoftParams), C.c_int64, dp, dp, dp, C.c_double,
                                     dp, dp]
        L.o_disks_intersect.restype = C.c_int
        L.o_sd_within.argtypes = [dp, dp, C.c_double, dp, C.c_double, C.c_double]
        L.o_sd_within.restype = C.c_int
        L.o_spherodisks_overlap.argtypes = [dp, dp, C.c_double, dp, dp, C.c_double, C.c_double,
                                            C.c_double, dp]
        L.o_spherodisks_overlap.restype = C.c_int
        L.o_rsa_candidate.argtypes = [C.c_int, C.c_int, dp, C.c_uint64, C.c_uint64, dp, dp]
        L.o_rsa.argtypes = [C.c_int, C.c_int, C.c_int64, dp, C.c_double, C.c_uint64,
                            C.c_int64, dp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                            C.POINTER(C.c_int64)]
        L.o_rsa.restype = C.c_int
        for f in ("o_pass", "o_overlap", "o_sweep", "o_run", "o_run_to", "o_rdf_brute", "o_bin",
                  "o_nearest_brute", "o_percolation"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return C.POINTER(C.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox4x32(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    out = (C.c_uint32 * 4)()
    lib().o_philox4x32(c, k, out)
    return np.array(list(out), dtype=np.uint32)


def unitvec(dim, seed, pid, t, kind, k, l, stream, length):
    v = np.zeros(3)
    r = lib().o_unitvec(dim, seed, pid, t, kind, k, l, stream, length, _dp(v))
    return v, r


def rsa_candidates(dim, shape, box, seed, ks):
    """Centres (len(ks), 3) and normals (len(ks), 3; zeros for balls) of the
    RSA stream's candidates ks."""
    box3 = np.array(tuple(box) + (1.0,) * (3 - len(box)), dtype=np.float64)
    ks = np.asarray(ks, dtype=np.int64)
    x = np.zeros((len(ks), 3))
    m = np.zeros((len(ks), 3))
    xi, mi = np.zeros(3), np.zeros(3)
    for r, k in enumerate(ks):
        lib().o_rsa_candidate(dim, shape, _dp(box3), seed, int(k), _dp(xi), _dp(mi))
        x[r], m[r] = xi, mi
    return x, m


def rsa(dim, shape, n, box, radius, seed, max_candidates=None):
    """Classical RSA of n equal particles.  Returns (status, pos (dim, n) SoA,
    normals (n, 3) or None, src (candidate index per particle), drawn,
    placed); on ENOTCONV only the first `placed` particles are valid."""
    box3 = np.array(tuple(box) + (1.0,) * (3 - len(box)), dtype=np.float64)
    if max_candidates is None:
        max_candidates = 1000 * max(n, 1)
    pos = np.zeros((max(n, 1), 3))
    nrm = np.zeros((max(n, 1), 3)) if shape == 1 else None
    src = np.zeros(max(n, 1), dtype=np.int64)
    drawn, placed = C.c_int64(), C.c_int64()
    rc = lib().o_rsa(dim, shape, n, _dp(box3), float(radius), seed, int(max_candidates),
                     _dp(pos), _dp(nrm), src.ctypes.data_as(C.POINTER(C.c_int64)),
                     C.byref(drawn), C.byref(placed))
    if rc not in (OK, ENOTCONV):
        _check(rc)
    soa = np.ascontiguousarray(pos[:n, :dim].T)
    return rc, soa, (nrm[:n] if nrm is not None else None), src[:n], drawn.value, placed.value


def disks_intersect(c1, n1, a1, c2, n2, a2, box=(1.0, 1.0, 1.0)) -> bool:
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (c1, n1, c2, n2, box)]
    return bool(lib().o_disks_intersect(_dp(arrs[0]), _dp(arrs[1]), float(a1), _dp(arrs[2]),
                                        _dp(arrs[3]), float(a2), _dp(arrs[4])))


def sd_within(d, n1, A1, n2, A2, T) -> bool:
    """Core disk 1 (centre 0, unit normal n1, radius A1) and core disk 2
    (centre d, n2, A2): is their minimum distance at most T?"""
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (d, n1, n2)]
    return bool(lib().o_sd_within(_dp(arrs[0]), _dp(arrs[1]), float(A1), _dp(arrs[2]),
                                  float(A2), float(T)))


def spherodisks_overlap(c1, n1, a1, c2, n2, a2, thick_ratio, gap=0.0,
                        box=(1.0, 1.0, 1.0)) -> bool:
    """Spherodisks of outer radii a1, a2 and thickness thick_ratio * 2a
    (lower particle id as disk 1), shells grown by gap."""
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (c1, n1, c2, n2, box)]
    return bool(lib().o_spherodisks_overlap(_dp(arrs[0]), _dp(arrs[1]), float(a1),
                                            _dp(arrs[2]), _dp(arrs[3]), float(a2),
                                            float(thick_ratio), float(gap), _dp(arrs[4])))


def _soft_params(dim, nbins, r_c, box=(1.0, 1.0, 1.0), kappa=1.0):
    sp = SoftParams()
    sp.dim, sp.nbins, sp.r_c, sp.kappa = int(dim), int(nbins), float(r_c), float(kappa)
    box3 = list(box) + [1.0] * (3 - len(box))
    for a in range(3):
        sp.box[a] = float(box3[a])
    return sp


def softrdf_forward(pos, radii, *, dim, nbins, r_c, box=(1.0, 1.0, 1.0), kappa=1.0):
    """Soft g(r) (nbins) and overlap energy of a configuration; pos is SoA
    (dim, n), radii (n,).  All pairs, FP64."""
    n = np.asarray(radii).shape[0]
    rows = _rows(pos, n)
    r = np.ascontiguousarray(radii, dtype=np.float64)
    g = np.zeros(nbins)
    e = np.zeros(1)
    sp = _soft_params(dim, nbins, r_c, box, kappa)
    lib().o_softrdf_fwd(C.byref(sp), n, _dp(rows), _dp(r), _dp(g), _dp(e))
    return g, float(e[0])


def softrdf_gradient(pos, radii, dg, dE, *, dim, nbins, r_c, box=(1.0, 1.0, 1.0), kappa=1.0):
    """Gradient (SoA (dim, n), (n,)) of sum_b dg_b g_b + dE * E."""
    n = np.asarray(radii).shape[0]
    rows = _rows(pos, n)
    r = np.ascontiguousarray(radii, dtype=np.float64)
    dgv = np.ascontiguousarray(dg, dtype=np.float64)
    gp = np.zeros((n, 3))
    gr = np.zeros(n)
    sp = _soft_params(dim, nbins, r_c, box, kappa)
    lib().o_softrdf_grad(C.byref(sp), n, _dp(rows), _dp(r), _dp(dgv), float(dE), _dp(gp),
                         _dp(gr))
    return np.ascontiguousarray(gp[:, :dim].T), gr


class Oracle:
    """A sequential SRM state in particle-id order.

    ``pos`` (and ``normals``) are SoA arrays of shape (dim, n); they are copied.
    """

    def __init__(self, *, dim, n, box=(1.0, 1.0, 1.0), s_target, c_w, c_m, n_k, n_l, seed,
                 pos, rho=None, normals=None, shape=0, c_n=0.0, thick_ratio=0.0,
                 s0=0.0, sweep0=0):
        self.params = Params()
        p = self.params
        p.dim, p.shape, p.n = int(dim), int(shape), int(n)
        box3 = list(box) + [1.0] * (3 - len(box))
        for a in range(3):
            p.box[a] = float(box3[a])
        p.s_target, p.c_w, p.c_m, p.c_n = float(s_target), float(c_w), float(c_m), float(c_n)
        p.thick_ratio = float(thick_ratio)
        p.n_k, p.n_l, p.seed = int(n_k), int(n_l), int(seed)
        self.pos = _rows(pos, n)
        self.nrm = None if normals is None else _rows(normals, n)
        self.rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).copy()
        self.st = State()
        self.st.p = p
        self.st.pos = _dp(self.pos)
        self.st.nrm = _dp(self.nrm)
        self.st.rho = _dp(self.rho)
        self.st.s = float(s0)
        self.st.t = int(sweep0)

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(dim=w.dim, n=w.n, box=w.box, s_target=w.s_target, c_w=w.c_w, c_m=w.c_m,
                  n_k=w.n_k, n_l=w.n_l, seed=w.seed, pos=w.pos, rho=w.rho, normals=w.normals,
                  shape=w.shape, c_n=w.c_n, thick_ratio=w.thick_ratio, s0=w.s0,
                  sweep0=w.sweep0)
        kw.update(over)
        return cls(**kw)

    # -- scalars ---------------------------------------------------------
    @property
    def s(self) -> float:
        return self.st.s

    @s.setter
    def s(self, v):
        self.st.s = float(v)

    @property
    def t(self) -> int:
        return self.st.t

    @t.setter
    def t(self, v):
        self.st.t = int(v)

    @property
    def n(self) -> int:
        return self.params.n

    @property
    def dim(self) -> int:
        return self.params.dim

    def rho_max(self) -> float:
        return lib().o_rho_max(C.byref(self.st))

    def swell(self, s: float) -> float:
        return lib().o_swell(C.byref(self.params), float(s))

    def grid(self, rmax: float):
        na = (C.c_int64 * 3)()
        inv = np.zeros(3)
        lib().o_grid(C.byref(self.params), float(rmax), na, _dp(inv))
        return np.array(list(na), dtype=np.int64), inv

    def grid_for_scale(self, s: float):
        return self.grid(s * self.rho_max())

    # -- steps -----------------------------------------------------------
    def bin(self, na, inv_w) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        na_c = (C.c_int64 * 3)(*[int(x) for x in na])
        inv = np.ascontiguousarray(inv_w, dtype=np.float64)
        lib().o_bin(C.byref(self.params), na_c, _dp(inv), _dp(self.pos),
                    out.ctypes.data_as(C.POINTER(C.c_int64)))
        return out

    def pass_(self, na, inv_w, s, kind, k, mask=None):
        """Bin, then one migration pass at radius scale s; returns (acc, overlap)."""
        acc = np.zeros(self.n, dtype=np.uint8)
        ov = C.c_int32(0)
        na_c = (C.c_int64 * 3)(*[int(x) for x in na])
        inv = np.ascontiguousarray(inv_w, dtype=np.float64)
        m = (C.POINTER(C.c_uint8)() if mask is None
             else np.ascontiguousarray(mask, dtype=np.uint8).ctypes.data_as(C.POINTER(C.c_uint8)))
        rc = lib().o_pass(C.byref(self.st), na_c, _dp(inv), float(s), int(kind), int(k),
                          acc.ctypes.data_as(C.POINTER(C.c_uint8)), m, C.byref(ov))
        _check(rc)
        return acc, bool(ov.value)

    def overlap(self, na=None, inv_w=None, s=None) -> bool:
        s = self.s if s is None else s
        if na is None:
            na, inv_w = self.grid_for_scale(s)
        ov = C.c_int32(0)
        na_c = (C.c_int64 * 3)(*[int(x) for x in na])
        inv = np.ascontiguousarray(inv_w, dtype=np.float64)
        _check(lib().o_overlap(C.byref(self.st), na_c, _dp(inv), float(s), C.byref(ov)))
        return bool(ov.value)

    def sweep(self):
        """One Alg. 1 iteration; returns (info dict, acc of the last pass)."""
        info = SweepInfo()
        acc = np.zeros(self.n, dtype=np.uint8)
        _check(lib().o_sweep(C.byref(self.st), C.byref(info),
                             acc.ctypes.data_as(C.POINTER(C.c_uint8))))
        d = dict(committed=bool(info.committed), passes_main=info.passes_main,
                 passes_shake=info.passes_shake, na=tuple(info.na), s=info.s_new,
                 n_failed_last=info.n_failed_last)
        return d, acc

    def run(self, max_sweeps: int, s_stop=None):
        """Sweep until s == s_stop (default s_target), swelling clamped at
        s_stop; returns (status, sweeps, passes)."""
        sw, ps = C.c_int64(0), C.c_int64(0)
        stop = self.params.s_target if s_stop is None else float(s_stop)
        rc = lib().o_run_to(C.byref(self.st), stop, int(max_sweeps), C.byref(sw), C.byref(ps))
        return rc, sw.value, ps.value

    # -- analysis ------------------------------------------------------------
    def pairs_brute(self, gap: float = 0.0, s=None) -> np.ndarray:
        s = self.s if s is None else s
        cnt = lib().o_pairs_brute(C.byref(self.st), float(s), float(gap), 0,
                                  C.POINTER(C.c_int32)())
        out = np.zeros((max(cnt, 1), 2), dtype=np.int32)
        lib().o_pairs_brute(C.byref(self.st), float(s), float(gap), cnt,
                            out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out[:cnt]

    def rdf_brute(self, nbins: int, r_max: float) -> np.ndarray:
        counts = np.zeros(nbins, dtype=np.uint64)
        _check(lib().o_rdf_brute(C.byref(self.st), int(nbins), float(r_max),
                                 counts.ctypes.data_as(C.POINTER(C.c_uint64))))
        return counts

    def nearest_brute(self, r_max: float) -> np.ndarray:
        """Distance to the nearest other particle (q < r_max^2), id order;
        +inf where there is none."""
        dist = np.empty(self.n, dtype=np.float64)
        _check(lib().o_nearest_brute(C.byref(self.st), float(r_max), _dp(dist)))
        return dist

    def percolation(self, gap: float, s=None) -> int:
        """Axes (bit mask) along which a cluster of particles grown by `gap`
        wraps around the box, at radius scale s (default: the state's)."""
        m = C.c_int32()
        _check(lib().o_percolation(C.byref(self.st), float(self.s if s is None else s),
                                   float(gap), C.byref(m)))
        return m.value

    def critical_gap(self, lo: float, hi: float, iters: int = 40) -> float:
        """Bisection on the gap, as the library does it: lo must not
        percolate and hi must; returns the final hi."""
        assert not self.percolation(lo) and self.percolation(hi)
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if self.percolation(mid):
                hi = mid
            else:
                lo = mid
        return hi

    def soa(self) -> np.ndarray:
        return np.ascontiguousarray(self.pos[:, : self.dim].T)

    def fraction(self, s=None) -> float:
        """Volume fraction sum v_i / |box| at radius scale s."""
        import math
        s = self.s if s is None else s
        p = self.params
        vbox = 1.0
        for a in range(p.dim):
            vbox *= p.box[a]
        rho = np.ones(self.n) if self.rho is None else self.rho
        if p.shape == 1:
            a = s * rho
            return float(np.sum(math.pi * a * a * (p.thick_ratio * 2.0 * a)) / vbox)
        if p.shape == 2:
            # spherodisk: core radius A = a - h, half-thickness h = thick_ratio * a
            a = s * rho
            h = p.thick_ratio * a
            A = a - h
            v = 2.0 * math.pi * A * A * h + math.pi ** 2 * A * h * h + 4.0 / 3.0 * math.pi * h ** 3
            return float(np.sum(v) / vbox)
        w = math.pi if p.dim == 2 else 4.0 * math.pi / 3.0
        return float(w * np.sum((s * rho) ** p.dim) / vbox)


def _rows(a, n) -> np.ndarray:
    """SoA (k, n) with k in {2, 3} -> (n, 3) rows, z = 0 when k == 2."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != n or a.shape[0] not in (2, 3):
        raise ValueError("expected SoA array of shape (dim, n)")
    out = np.zeros((n, 3), dtype=np.float64)
    out[:, : a.shape[0]] = a.T
    return np.ascontiguousarray(out)


def _check(rc):
    if rc != OK:
        raise RuntimeError(f"oracle returned {rc}")
