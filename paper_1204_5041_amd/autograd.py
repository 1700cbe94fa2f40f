"""torch.autograd face of libcsmap.

The map Theta/GU of Eq. (1)-(2) (Sec. II.A) is a function of the segments of
every box: positions x_rel, velocities Xdot, tangents X' and lengths dsigma.
`render` makes it a differentiable torch operation: its forward pass is the
library's render, its backward pass the library's hand-written adjoint
(csmap_backward), which returns dL/d(x_rel, Xdot, X', dsigma) of every
segment for the map cotangent dL/dTheta.  This module only marshals tensors;
every step of the computation runs in the HIP kernels.

Box geometry (FP64 origin, conformal-time slab, visibility rule) is not
differentiated.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import binding as B

_GEOM_KEYS = ("origin", "eta_lo", "eta_hi", "vis", "ext", "cap_dir", "cap_cos", "snapshot")
_SEG_KEYS = ("x_rel", "xdot", "xprime", "dsigma")


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sky: B.Sky, geoms: tuple, *seg):
        sky.reset()
        for b, geom in enumerate(geoms):
            sky.add_box(*seg[4 * b:4 * b + 4], **geom)
        out = sky.render()
        sky._autograd_epoch = getattr(sky, "_autograd_epoch", 0) + 1
        ctx.sky = sky
        ctx.epoch = sky._autograd_epoch
        ctx.dtypes = [t.dtype for t in seg]
        return out

    @staticmethod
    def backward(ctx, dmap):
        sky = ctx.sky
        if getattr(sky, "_autograd_epoch", None) != ctx.epoch:
            raise RuntimeError("the sky was rendered again after this map was made; its "
                               "boxes no longer match the graph (use one sky per graph)")
        grads = sky.backward(dmap.to(torch.float64).contiguous())
        flat = []
        for g in grads:
            flat.extend(g)
        out = [None, None]
        for i, (g, dt) in enumerate(zip(flat, ctx.dtypes)):
            out.append(g.to(dt) if ctx.needs_input_grad[2 + i] else None)
        return tuple(out)


def render(sky: B.Sky, boxes: Sequence[dict]) -> torch.Tensor:
    """Theta/GU at all 12 Nside^2 RING pixels (float64), differentiable with
    respect to the segment tensors of `boxes`.

    Each box is a dict with the CUDA tensors x_rel (n,3), xdot (n,3),
    xprime (n,3), dsigma (n,) of one dtype, and the keyword arguments of
    `Sky.add_box` (origin, eta_lo, eta_hi, and optionally vis, ext, cap_dir,
    cap_cos).  The sky is reset and refilled on every call, so a sky serves
    one graph at a time: rendering again before the backward pass of an
    earlier map makes that backward pass raise."""
    geoms = tuple({k: bx[k] for k in _GEOM_KEYS if k in bx} for bx in boxes)
    seg = []
    for bx in boxes:
        seg.extend(bx[k] for k in _SEG_KEYS)
    return _Render.apply(sky, geoms, *seg)


class StringMap(torch.nn.Module):
    """A module holding one FP32C sky: forward(boxes) -> Theta/GU map."""

    def __init__(self, nside: int, eta0: float, form: int = B.CSMAP_FORM_FP32C):
        super().__init__()
        if form != B.CSMAP_FORM_FP32C:
            raise ValueError("the adjoint is provided for the FP32C form")
        self.sky = B.Sky(nside, eta0, form)

    def forward(self, boxes: Sequence[dict]) -> torch.Tensor:
        return render(self.sky, boxes)
