"""Differentiation through the projector pair and through unrolled ImaSk.

`SketchFn` wraps K_k (or K_k^T) of a level set as a torch.autograd.Function
whose backward is the other half of the exact transpose pair, so gradients
of anything built from the sketched operators are exact up to FP32 rounding.
`unrolled_imask` runs Alg. 1 (Tikhonov regulariser, mu = lam) for a fixed,
seeded draw sequence as a differentiable graph, checkpointed every few
iterations; gradients flow to the data (hence to an image that generated
it) and to lam.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from . import imask as im


class SketchFn(torch.autograd.Function):
    """out = K_k inp (adjoint=False) or K_k^T inp (adjoint=True)."""

    @staticmethod
    def forward(ctx, inp, geom, levels, k, adjoint, work):
        ctx.geom, ctx.levels, ctx.k, ctx.adjoint, ctx.work = geom, levels, k, adjoint, work
        return im.sketch_apply(geom, levels, k, inp.contiguous(), adjoint, work)

    @staticmethod
    def backward(ctx, grad):
        g = im.sketch_apply(ctx.geom, ctx.levels, ctx.k, grad.contiguous(), not ctx.adjoint, ctx.work)
        return g, None, None, None, None, None


class ProjectFn(torch.autograd.Function):
    """sino = R_l T_l x with the exact transpose as backward."""

    @staticmethod
    def forward(ctx, x, geom, log2f, work):
        ctx.geom, ctx.log2f, ctx.work = geom, log2f, work
        return im.project(geom, log2f, x.contiguous(), work)

    @staticmethod
    def backward(ctx, grad):
        return im.backproject(ctx.geom, ctx.log2f, grad.contiguous(), ctx.work), None, None, None


class BackprojectFn(torch.autograd.Function):
    """x = T_l^T R_l^T sino with the forward projector as backward."""

    @staticmethod
    def forward(ctx, sino, geom, log2f, work):
        ctx.geom, ctx.log2f, ctx.work = geom, log2f, work
        return im.backproject(geom, log2f, sino.contiguous(), work)

    @staticmethod
    def backward(ctx, grad):
        return im.project(ctx.geom, ctx.log2f, grad.contiguous(), ctx.work), None, None, None


def _step(k, x, y, phi, psi, b, lam, sigma, geom, levels, work):
    """One iteration of Alg. 1 (parallel update, old tables)."""
    p = levels.p
    gx = SketchFn.apply(y, geom, levels, k, True, work)
    gy = SketchFn.apply(x, geom, levels, k, False, work)
    avg_phi = sum(p[j] * phi[j] for j in range(levels.r))
    avg_psi = sum(p[j] * psi[j] for j in range(levels.r))
    xi = (gx - phi[k]) + avg_phi
    zeta = (gy - psi[k]) + avg_psi
    x_new = (x - (sigma / lam) * xi) / (1.0 + sigma)  # prox of (sigma/lam) * lam/2 |.|^2
    y_new = (y + sigma * zeta - sigma * b) / (1.0 + sigma)
    phi = list(phi)
    psi = list(psi)
    phi[k] = gx
    psi[k] = gy
    return x_new, y_new, phi, psi


def unrolled_imask(b: torch.Tensor, lam: torch.Tensor, geom: im.Geometry, levels: im.Levels, sigma: float,
                   iters: int, seed: int = 42, stream_id: int = 0, work: torch.Tensor | None = None,
                   checkpoint_every: int = 2) -> torch.Tensor:
    """x^iters of Alg. 1 from zero state, differentiable in b and lam.

    Segments of `checkpoint_every` iterations are recomputed in the backward
    pass instead of storing their intermediates."""
    if work is None:
        work = im.workspace(geom, b.device)
    draws = [int(k) for k in im.draws(im.Params(sigma, seed, stream_id), levels, 0, iters)]
    r = levels.r
    x = torch.zeros(geom.image_shape, device=b.device)
    y = torch.zeros(geom.sino_shape, device=b.device)
    phi = [torch.zeros(geom.image_shape, device=b.device) for _ in range(r)]
    psi = [torch.zeros(geom.sino_shape, device=b.device) for _ in range(r)]

    def segment(ks, x, y, b, lam, *tables):
        ph, ps = list(tables[:r]), list(tables[r:])
        for k in ks:
            x, y, ph, ps = _step(k, x, y, ph, ps, b, lam, sigma, geom, levels, work)
        return (x, y, *ph, *ps)

    for s0 in range(0, iters, checkpoint_every):
        ks = draws[s0:s0 + checkpoint_every]
        out = checkpoint(segment, ks, x, y, b, lam, *phi, *psi, use_reentrant=False)
        x, y, phi, psi = out[0], out[1], list(out[2:2 + r]), list(out[2 + r:])
    return x
