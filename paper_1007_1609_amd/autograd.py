"""torch.autograd wrappers over the ABI: every forward and backward is a
library call; torch only carries the tensors and the tape.

    mu_ee, mu_he = moments(eps, delta, geom, sites, N, tile)   # d/d eps, d/d Delta
    delta_new    = gap_map(mu_he, delta_in, U, weights, alpha)  # d/d mu_he, d/d delta_in
    ldos         = local_dos(mu_ee, energies, weights)          # d/d mu_ee

The rescaling (a, b) in `geom` is a constant: gradients do not flow through
the spectral bound.  Real operators with on-site pairing only.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import _lib as L
from .api import (REVERSIBLE, Operator, chebyshev_moments, chebyshev_moments_backward, gap_update,
                  gap_update_backward, ldos, ldos_backward, reversible_supported)


@dataclass(frozen=True)
class Geometry:
    Lx: int
    Ly: int
    t: float
    mu_c: float
    a: float
    b: float
    bc_x: int = 0
    bc_y: int = 0

    @classmethod
    def of(cls, w, a, b):
        return cls(w.Lx, w.Ly, w.t, w.mu_c, a, b, w.bc_x, w.bc_y)


class _Moments(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, delta, geom, sites, N, tile, ckpt):
        op = Operator(geom.Lx, geom.Ly, geom.t, geom.mu_c, eps.detach().contiguous(),
                      delta.detach().contiguous(), bc_x=geom.bc_x, bc_y=geom.bc_y,
                      fixed=(geom.a, geom.b))
        mu_ee, mu_he = chebyshev_moments(op, sites, N, tile)
        if ckpt is None:  # the checkpoint-free reverse passes where they apply
            ckpt = REVERSIBLE if reversible_supported(op, min(tile, max(1, sites.numel())), N) else 0
        ctx.op, ctx.sites, ctx.N, ctx.tile, ctx.ckpt = op, sites, N, tile, ckpt
        return mu_ee, mu_he

    @staticmethod
    def backward(ctx, g_ee, g_he):
        g_ee = None if g_ee is None else g_ee.contiguous()
        g_he = None if g_he is None else g_he.contiguous()
        # the operator stays alive with the graph (a retained graph may run
        # backward again); it is released when the graph is freed
        ge, gd = chebyshev_moments_backward(ctx.op, ctx.sites, ctx.N, ctx.tile, g_ee, g_he, ctx.ckpt)
        return ge, gd, None, None, None, None, None


def moments(eps, delta, geom: Geometry, sites, N: int, tile: int, ckpt=None):
    """Moments of eqs. (coeff1)/(coeff2) with a backward through the library's
    adjoint.  ckpt: the reverse pass's checkpoint stride (0: sqrt(N)), -1 for
    the checkpoint-free passes, None for those where they apply (doubling,
    lattices 64 W wide), else 0."""
    return _Moments.apply(eps, delta, geom, sites, N, tile, ckpt)


class _Gap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu_he, delta_in, U, w, alpha):
        out, _ = gap_update(mu_he.contiguous(), w, U, delta_in.detach().contiguous(), alpha)
        ctx.U, ctx.w, ctx.alpha, ctx.N = U, w, alpha, mu_he.shape[1]
        return out

    @staticmethod
    def backward(ctx, g):
        d_mu, d_in = gap_update_backward(g.contiguous(), ctx.N, ctx.w, ctx.U, ctx.alpha)
        return d_mu, d_in, None, None, None


def gap_map(mu_he, delta_in, U: float, w: L.cbdg_weights, alpha: float = 1.0):
    return _Gap.apply(mu_he, delta_in, U, w, alpha)


class _Ldos(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu_ee, energies, w):
        ctx.w, ctx.energies, ctx.N = w, energies, mu_ee.shape[1]
        return ldos(mu_ee.contiguous(), w, energies)

    @staticmethod
    def backward(ctx, g):
        return ldos_backward(g.contiguous(), ctx.N, ctx.w, ctx.energies), None, None


def local_dos(mu_ee, energies, w: L.cbdg_weights):
    return _Ldos.apply(mu_ee, energies, w)
