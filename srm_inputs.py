"""Seeded synthetic starting configurations for the SRM workloads.

This module is shared by the CPU oracle, the GPU library tests and the
benchmark.  It draws starting configurations and workload parameters only;
it holds no step of the SRM method itself (no swelling, binning, migration,
overlap test or schedule).

Draw conventions (all from ``numpy.random.Philox``, i.e. Philox4x64-10 keyed
by the workload seed):

* positions: raw 64-bit word W -> (W >> 11) * 2**-53 in [0, 1), one word per
  axis, particle ids ascending, then scaled by the box edge;
* isotropic unit normals: three standard normals per particle, normalised;
* cap normals: uniform on the spherical cap of half-angle theta about +z
  (cos(angle) uniform in [cos theta, 1], azimuth uniform);
* lognormal shape radii: ln(rho) ~ N(-sigma**2/2, sigma**2) so E[rho] = 1.

The target radius scale ``s_target`` is the scale at which the particle
volumes fill the requested fraction of the box: ball volume omega_d R**d with
omega_2 = pi, omega_3 = 4 pi / 3 (disks and spheres), pi a**2 t with
t = thick_ratio * 2a for thin circular platelets (cylinder model), and the
volume of a spherodisk of outer radius a and thickness t (a core disk of
radius a - t/2 swept by a ball of radius t/2) for spherodisks.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BALL = 0
PLATELET = 1
SPHERODISK = 2


@dataclasses.dataclass
class Workload:
    """One SRM run: parameters plus the starting configuration.

    ``pos`` is SoA, shape (dim, n), float64, in [0, box) per axis.
    ``rho`` is None for monodisperse particles (all shape radii 1).
    ``normals`` is (3, n) float64 unit vectors for platelets, else None.
    """
    name: str
    dim: int
    shape: int
    n: int
    box: tuple
    f_target: float
    s_target: float
    c_w: float
    c_m: float
    c_n: float
    thick_ratio: float
    n_k: int
    n_l: int
    seed: int
    pos: np.ndarray
    rho: Optional[np.ndarray] = None
    normals: Optional[np.ndarray] = None
    s0: float = 0.0
    sweep0: int = 0

    def params(self) -> dict:
        return dict(dim=self.dim, shape=self.shape, n=self.n, box=tuple(self.box),
                    s_target=self.s_target, c_w=self.c_w, c_m=self.c_m,
                    c_n=self.c_n, thick_ratio=self.thick_ratio,
                    n_k=self.n_k, n_l=self.n_l, seed=self.seed)


def philox_words(seed: int, count: int, stream: int = 0) -> np.ndarray:
    """``count`` raw 64-bit Philox4x64-10 words for key (seed, stream)."""
    bg = np.random.Philox(key=int(seed) | (int(stream) << 64))
    return bg.random_raw(int(count))


def uniform_points(n: int, dim: int, seed: int, box=(1.0, 1.0, 1.0)) -> np.ndarray:
    """SoA (dim, n) positions, uniform in the box, one Philox word per axis."""
    w = philox_words(seed, n * dim).reshape(n, dim)
    u = (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    pos = np.empty((dim, n), dtype=np.float64)
    for a in range(dim):
        pos[a] = u[:, a] * float(box[a])
        # u < 1, but u * L can round up to L itself: keep the box half-open
        pos[a] = np.where(pos[a] >= box[a], np.nextafter(float(box[a]), 0.0), pos[a])
    return pos


def isotropic_normals(n: int, seed: int) -> np.ndarray:
    g = np.random.Generator(np.random.Philox(key=int(seed) | (1 << 64)))
    v = g.standard_normal((3, n))
    v /= np.sqrt((v * v).sum(axis=0))
    return v


def cap_normals(n: int, seed: int, half_angle_deg: float) -> np.ndarray:
    g = np.random.Generator(np.random.Philox(key=int(seed) | (2 << 64)))
    ct = math.cos(math.radians(half_angle_deg))
    cz = g.uniform(ct, 1.0, n)
    phi = g.uniform(0.0, 2.0 * math.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    v = np.stack([sz * np.cos(phi), sz * np.sin(phi), cz])
    v /= np.sqrt((v * v).sum(axis=0))
    return v


def lognormal_rho(n: int, seed: int, sigma: float = 0.2) -> np.ndarray:
    g = np.random.Generator(np.random.Philox(key=int(seed) | (3 << 64)))
    return np.exp(g.normal(-0.5 * sigma * sigma, sigma, n))


def ball_volume_coeff(dim: int) -> float:
    return math.pi if dim == 2 else 4.0 * math.pi / 3.0


def spherodisk_volume_coeff(thick_ratio: float) -> float:
    """Volume of a spherodisk of outer radius 1 and thickness 2 thick_ratio:
    core disk radius A = 1 - h swept by a ball of radius h = thick_ratio
    (Steiner: 2 pi A^2 h + pi^2 A h^2 + 4/3 pi h^3)."""
    h = thick_ratio
    A = 1.0 - h
    return 2.0 * math.pi * A * A * h + math.pi ** 2 * A * h * h + 4.0 / 3.0 * math.pi * h ** 3


def target_scale(dim: int, shape: int, f_target: float, box, rho: Optional[np.ndarray],
                 n: int, thick_ratio: float = 0.01) -> float:
    """Scale s at which sum of particle volumes / box volume == f_target."""
    vbox = float(np.prod(np.asarray(box[:dim], dtype=np.float64)))
    srd = float(n) if rho is None else float(np.sum(rho.astype(np.float64) ** dim))
    if shape == PLATELET:
        coeff = 2.0 * math.pi * thick_ratio  # pi a^2 (thick_ratio * 2 a)
    elif shape == SPHERODISK:
        coeff = spherodisk_volume_coeff(thick_ratio)
    else:
        coeff = ball_volume_coeff(dim)
    return (f_target * vbox / (coeff * srd)) ** (1.0 / dim)


def make(name: str = "disks2d", *, n: Optional[int] = None, dim: Optional[int] = None,
         seed: Optional[int] = None, f_target: Optional[float] = None,
         c_w: float = 0.01, c_m_rel: float = 0.1, n_k: int = 8, n_l: int = 8,
         polydisperse_sigma: Optional[float] = None, box=(1.0, 1.0, 1.0),
         cap_deg: Optional[float] = None, aspect_ratio: Optional[float] = None) -> Workload:
    """Build a named workload, optionally overriding its size and seed.

    Named workloads:
      disks2d    2D unit square, N=2000 disks, seed 0, f_target 0.50
      spheres3d  3D unit cube, N=1e7 spheres, seed 1, f_target 0.35
      platelets  3D unit cube, N=2e5 thin platelets (t = D/100), seed 2,
                 f_target 0.02, isotropic normals (cap_deg=15 for the
                 quasi-nematic start)
      softrdf    3D unit cube, N=2e5 spheres, seed 3, f_target 0.30
      spherodisks 3D unit cube, N=2e4 spherodisks of aspect ratio D/t = 100
                 (``aspect_ratio`` overrides it), seed 4, f_target 0.02,
                 isotropic normals (cap_deg as for platelets)
    c_m = c_m_rel * s_target (migration step of a tenth of the final radius).
    """
    defaults = {
        "disks2d": dict(dim=2, n=2000, seed=0, f_target=0.50, shape=BALL),
        "spheres3d": dict(dim=3, n=10_000_000, seed=1, f_target=0.35, shape=BALL),
        "platelets": dict(dim=3, n=200_000, seed=2, f_target=0.02, shape=PLATELET),
        "softrdf": dict(dim=3, n=200_000, seed=3, f_target=0.30, shape=BALL),
        "spherodisks": dict(dim=3, n=20_000, seed=4, f_target=0.02, shape=SPHERODISK),
    }
    if name not in defaults:
        raise KeyError(f"unknown workload {name!r}")
    d = dict(defaults[name])
    if n is not None:
        d["n"] = int(n)
    if dim is not None:
        d["dim"] = int(dim)
    if seed is not None:
        d["seed"] = int(seed)
    if f_target is not None:
        d["f_target"] = float(f_target)
    dim_, n_, seed_, shape = d["dim"], d["n"], d["seed"], d["shape"]
    box3 = tuple(float(b) for b in box) + (1.0,) * (3 - len(box))
    pos = uniform_points(n_, dim_, seed_, box3)
    rho = None if polydisperse_sigma is None else lognormal_rho(n_, seed_, polydisperse_sigma)
    normals = None
    thick = 0.01 if aspect_ratio is None else 1.0 / float(aspect_ratio)
    disk = shape in (PLATELET, SPHERODISK)
    if disk:
        normals = (cap_normals(n_, seed_, cap_deg) if cap_deg is not None
                   else isotropic_normals(n_, seed_))
    s_t = target_scale(dim_, shape, d["f_target"], box3, rho, n_, thick)
    c_m = c_m_rel * s_t
    c_n = c_m / s_t if disk else 0.0
    return Workload(name=name, dim=dim_, shape=shape, n=n_, box=box3,
                    f_target=d["f_target"], s_target=s_t, c_w=c_w, c_m=c_m, c_n=c_n,
                    thick_ratio=thick if disk else 0.0, n_k=n_k, n_l=n_l,
                    seed=seed_, pos=pos, rho=rho, normals=normals)


def batch_members(count: int = 256, seed0: int = 1000, n_lo: float = 1e3, n_hi: float = 1e5,
                  f_lo: float = 0.30, f_hi: float = 0.55, sigma: float = 0.2,
                  n_scale: float = 1.0):
    """Per-RVE metadata of the batched ensemble: first half 2D, second half 3D.

    N is log-uniform in [n_lo, n_hi] (times ``n_scale`` for reduced test
    ensembles), the target fraction uniform in [f_lo, f_hi], shape radii
    lognormal with mean 1.  Seeds are seed0 .. seed0+count-1.
    """
    out = []
    for r in range(count):
        seed = seed0 + r
        g = np.random.Generator(np.random.Philox(key=seed | (4 << 64)))
        u, up = g.random(2)
        n = max(1, int(round(n_scale * 10.0 ** (math.log10(n_lo) + (math.log10(n_hi) - math.log10(n_lo)) * u))))
        f = f_lo + (f_hi - f_lo) * up
        dim = 2 if r < count // 2 else 3
        out.append(dict(seed=seed, n=n, f_target=float(f), dim=dim, sigma=sigma))
    return out


def make_member(meta: dict, c_w: float = 0.01, c_m_rel: float = 0.1, n_k: int = 8,
                n_l: int = 8) -> Workload:
    dim, n, seed = meta["dim"], meta["n"], meta["seed"]
    box3 = (1.0, 1.0, 1.0)
    pos = uniform_points(n, dim, seed, box3)
    rho = lognormal_rho(n, seed, meta["sigma"])
    s_t = target_scale(dim, BALL, meta["f_target"], box3, rho, n)
    return Workload(name=f"rve{seed}", dim=dim, shape=BALL, n=n, box=box3,
                    f_target=meta["f_target"], s_target=s_t, c_w=c_w, c_m=c_m_rel * s_t,
                    c_n=0.0, thick_ratio=0.0, n_k=n_k, n_l=n_l, seed=seed, pos=pos, rho=rho)
