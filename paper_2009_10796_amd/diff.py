"""Differentiable update frame and query, as a torch.autograd.Function.

``frame_and_query(ctx, R, pos, nrm, view, emission, atlases)`` runs one
probe update frame of the context from the given input atlases with the
given emitter radiance, then queries irradiance at the points.  Its backward
is the library's hand-written adjoint: the reverse of the query, of the
blend (Eq. U with hysteresis, border texels folded onto their interior
sources) and of the hit shading (emission plus albedo times the previous
frame's irradiance at the hit).  Ray hits, shadow decisions and probe states
are those of the forward frame, held fixed; the derivative of the Chebyshev
visibility is taken as zero where its variance is clamped at zero.

Every step runs in the library's kernels; this module only allocates the
gradient buffers and calls the C entry points.
"""
from __future__ import annotations

from typing import Sequence


def _torch():
    import torch
    return torch


def _make_function():
    torch = _torch()

    class _FrameAndQuery(torch.autograd.Function):
        @staticmethod
        def forward(fctx, ctx, R, pos, nrm, view, emission, *atlases):
            V = ctx.volumes
            if len(atlases) != 2 * len(V):
                raise ValueError("atlases: (irradiance, distance) per volume")
            for v, vol in enumerate(V):
                if vol.irradiance.dtype != torch.float32:
                    raise ValueError("differentiation needs float32 atlases")
                vol.irradiance.copy_(atlases[2 * v])
                vol.distance.copy_(atlases[2 * v + 1])
            ctx.set_emission(emission)
            ctx.set_differentiable(True)
            ctx.update_probes(R)
            E = ctx.query_irradiance(pos, nrm, view)
            fctx.irf = ctx
            fctx.frame = ctx.frames
            fctx.q = (pos, nrm, view)
            fctx.n_materials = emission.shape[0]
            return E

        @staticmethod
        def backward(fctx, gE):
            ctx = fctx.irf
            if ctx.frames != fctx.frame:
                raise RuntimeError("another update frame ran on the context since this forward: "
                                   "its saved frame is gone")
            V = ctx.volumes
            dev = ctx.device
            g1i = [torch.zeros(v.irradiance.shape, dtype=torch.float32, device=dev) for v in V]
            g1d = [torch.zeros(v.distance.shape, dtype=torch.float32, device=dev) for v in V]
            pos, nrm, view = fctx.q
            ctx.query_backward(pos, nrm, view, gE.to(torch.float32).contiguous(), g1i, g1d)
            g0i = [torch.zeros_like(t) for t in g1i]
            g0d = [torch.zeros_like(t) for t in g1d]
            ge = torch.zeros((fctx.n_materials, 3), dtype=torch.float32, device=dev)
            ctx.update_backward(g1i, g1d, g0i, g0d, ge)
            grads = []
            for a, b in zip(g0i, g0d):
                grads += [a, b]
            return (None, None, None, None, None, ge, *grads)

    return _FrameAndQuery


_FN = None


def frame_and_query(ctx, R, pos, nrm, view, emission, atlases: Sequence):
    """E [n, 3] after one update frame; differentiable in `emission`
    [n_materials, 3] and in the input atlases (irradiance, distance per
    volume, float32, the volumes' layouts)."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    return _FN.apply(ctx, R, pos, nrm, view, emission, *atlases)
