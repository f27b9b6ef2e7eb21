"""Differentiable soft-binned g(r) + overlap energy on the GPU.

``SoftRDF`` wraps a ``srm_soft`` workspace of the C library; ``soft_rdf``
is the ``torch.autograd.Function`` front end (forward and hand-written
backward both run in the library's HIP kernels on torch's current stream).
``steer`` moves a configuration down the gradient of a loss on g(r) and the
overlap energy, letting an SRM sweep (swelling off) restore admissibility
after every step; a step whose sweep cannot commit is rejected.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import SRM, _check, lib


class SoftParams(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nbins", C.c_int32), ("box", C.c_double * 3),
                ("r_c", C.c_double), ("kappa", C.c_double)]


def _bind():
    L = lib()
    if getattr(L, "_soft_bound", False):
        return L
    vp = C.c_void_p
    L.srm_softrdf_create.argtypes = [C.POINTER(SoftParams), C.c_int64, vp, C.POINTER(vp)]
    L.srm_softrdf_forward.argtypes = [vp, vp, vp, vp, vp]
    L.srm_softrdf_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.srm_softrdf_free.argtypes = [vp]
    L.srm_softrdf_forward_static.argtypes = [C.POINTER(SoftParams), C.c_int64, vp, vp, vp, vp,
                                             vp]
    L.srm_set_state.argtypes = [vp, vp, vp, C.c_int32]
    for f in ("srm_softrdf_create", "srm_softrdf_forward", "srm_softrdf_backward",
              "srm_softrdf_free", "srm_softrdf_forward_static", "srm_set_state"):
        getattr(L, f).restype = C.c_int32
    L._soft_bound = True
    return L


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


class SoftRDF:
    """Workspace for n particles: nbins bins on [0, r_c], penalty kappa."""

    def __init__(self, n: int, dim: int, r_c: float, nbins: int = 64, box=(1.0, 1.0, 1.0),
                 kappa: float = 1.0):
        L = _bind()
        p = SoftParams()
        p.dim, p.nbins, p.r_c, p.kappa = int(dim), int(nbins), float(r_c), float(kappa)
        box3 = list(box) + [1.0] * (3 - len(box))
        for a in range(3):
            p.box[a] = float(box3[a])
        self.p, self.n, self.dim, self.nbins = p, int(n), int(dim), int(nbins)
        self.stream = torch.cuda.current_stream().cuda_stream
        ctx = C.c_void_p()
        _check(L.srm_softrdf_create(C.byref(p), self.n, C.c_void_p(self.stream), C.byref(ctx)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            lib().srm_softrdf_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, pos: torch.Tensor, radii: torch.Tensor):
        """pos (dim, n), radii (n,) float64 CUDA -> (g (nbins,), E ())."""
        g = torch.empty(self.nbins, dtype=torch.float64, device=pos.device)
        e = torch.empty((), dtype=torch.float64, device=pos.device)
        _check(lib().srm_softrdf_forward(self._ctx, _ptr(pos), _ptr(radii), _ptr(g), _ptr(e)))
        return g, e

    def backward(self, pos, radii, dg, de):
        gp = torch.empty_like(pos)
        gr = torch.empty_like(radii)
        _check(lib().srm_softrdf_backward(self._ctx, _ptr(pos), _ptr(radii), _ptr(dg), _ptr(de),
                                          _ptr(gp), _ptr(gr)))
        return gp, gr


# Largest n srm_softrdf_forward_static accepts (its fixed device array).
STATIC_MAX_N = 262144


def soft_params(dim: int, r_c: float, nbins: int = 64, box=(1.0, 1.0, 1.0),
                kappa: float = 1.0) -> SoftParams:
    p = SoftParams()
    p.dim, p.nbins, p.r_c, p.kappa = int(dim), int(nbins), float(r_c), float(kappa)
    box3 = list(box) + [1.0] * (3 - len(box))
    for a in range(3):
        p.box[a] = float(box3[a])
    return p


def forward_static(pos: torch.Tensor, radii: torch.Tensor, g: torch.Tensor, e: torch.Tensor,
                   dim: int, r_c: float, nbins: int = 64, box=(1.0, 1.0, 1.0),
                   kappa: float = 1.0) -> None:
    """The soft g(r) forward into caller-owned g (nbins,) and e (), with no
    workspace and no device allocation (``srm_softrdf_forward_static``);
    runs on torch's current stream."""
    L = _bind()
    p = soft_params(dim, r_c, nbins, box, kappa)
    n = pos.shape[1]
    stream = torch.cuda.current_stream().cuda_stream
    _check(L.srm_softrdf_forward_static(C.byref(p), n, _ptr(pos), _ptr(radii), _ptr(g), _ptr(e),
                                        C.c_void_p(stream)))


class SoftRDFFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, radii, ws: SoftRDF):
        pos = pos.contiguous()
        radii = radii.contiguous()
        g, e = ws.forward(pos, radii)
        ctx.save_for_backward(pos, radii)
        ctx.ws = ws
        return g, e

    @staticmethod
    def backward(ctx, dg, de):
        pos, radii = ctx.saved_tensors
        dg = (torch.zeros(ctx.ws.nbins, dtype=torch.float64, device=pos.device)
              if dg is None else dg.contiguous())
        de = (torch.zeros((), dtype=torch.float64, device=pos.device)
              if de is None else de.contiguous())
        gp, gr = ctx.ws.backward(pos, radii, dg, de)
        return gp, gr, None


def soft_rdf(pos: torch.Tensor, radii: torch.Tensor, ws: SoftRDF):
    """Differentiable (g, E) of a configuration (see ``SoftRDF``)."""
    return SoftRDFFunction.apply(pos, radii, ws)


def thomas_g(r, parent_density: float, sigma: float, dim: int = 3):
    """Pair correlation of a Thomas cluster process (Neyman-Scott with
    Gaussian offspring of standard deviation sigma per axis, parents of
    intensity parent_density): 1 + exp(-r^2/(4 sigma^2)) / (lambda_p
    (4 pi sigma^2)^(dim/2))."""
    return 1.0 + torch.exp(-r * r / (4.0 * sigma * sigma)) / (
        parent_density * (4.0 * math.pi * sigma * sigma) ** (dim / 2.0))


def set_positions(srm: SRM, pos: torch.Tensor):
    """Replace an SRM context's committed positions (device tensor (dim, n))."""
    _check(_bind().srm_set_state(srm._ctx, _ptr(pos.contiguous()), None, 1))


def steer(srm: SRM, ws: SoftRDF, target: torch.Tensor, radius: float, steps: int,
          max_step: float, lam: float = 1.0, tries: int = 6, grow: float = 1.25):
    """Monotone descent of L = |g - target|^2 + lam * E over the positions.

    A step moves every particle along -dL/dx, scaled so that the largest move
    is eta (at most max_step).  An SRM sweep (the context's c_w should be 0
    and its c_m small) then has to commit an overlap-free state -- SRM's exact
    test judges admissibility -- and the loss of that committed state has to
    be below the current loss; otherwise the step is undone and retried with
    eta halved, up to `tries` times.  A kept step lets eta grow by `grow`.
    Returns the history [(loss, kept, eta)] after each step, the first entry
    being the starting loss."""
    dim, n = srm.dim, srm.n
    box = torch.tensor(list(srm.params.box)[:dim], dtype=torch.float64, device="cuda")
    pos = torch.empty((dim, n), dtype=torch.float64, device="cuda")
    cand = torch.empty_like(pos)
    radii = torch.full((n,), float(radius), dtype=torch.float64, device="cuda")

    def loss_and_grad(x):
        p = x.clone().requires_grad_(True)
        g, e = soft_rdf(p, radii, ws)
        loss = ((g - target) ** 2).sum() + lam * e
        loss.backward()
        return float(loss.detach()), p.grad.detach()

    srm.state_device(pos)
    loss0, grad = loss_and_grad(pos)
    eta = float(max_step)
    hist = [(loss0, True, 0.0)]
    for _ in range(steps):
        kept = False
        for _t in range(tries):
            gmax = float(grad.abs().max())
            if gmax == 0.0:
                break
            with torch.no_grad():
                new = pos - (eta / gmax) * grad
                new = torch.remainder(new, box[:, None])
                new = torch.where(new >= box[:, None], new - box[:, None], new)
            set_positions(srm, new)
            info = srm.sweep()
            if info["committed"]:
                srm.state_device(cand)
                loss1, grad1 = loss_and_grad(cand)
                if loss1 < loss0:
                    pos.copy_(cand)
                    loss0, grad = loss1, grad1
                    eta = min(eta * grow, float(max_step))
                    kept = True
                    break
            set_positions(srm, pos)
            eta *= 0.5
        hist.append((loss0, kept, eta))
    return hist
