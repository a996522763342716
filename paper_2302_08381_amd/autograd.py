"""torch.autograd wrapper with first and second derivatives.

Forward: Y = sph(xyz).  When xyz needs a gradient the forward also stores
dY (one pass, sph_compute_with_gradients) and the backward contracts it with
the upstream gradient (sph_backward), as the paper's PyTorch binding does
with the derivatives of the forward pass (Sec. III).  That backward is itself
a differentiable function of (grad_Y, xyz) whose derivatives come from
sph_double_backward, so forces trained through an energy (double backward)
work.  All arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

import torch

from . import _native


class _SphBackward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grad_Y, xyz, dY, l_max, normalize):
        ctx.save_for_backward(grad_Y, xyz)
        ctx.l_max = l_max
        ctx.normalize = normalize
        return _native.sph_backward(dY, grad_Y.contiguous(), l_max)

    @staticmethod
    def backward(ctx, v):
        grad_Y, xyz = ctx.saved_tensors
        want_gg = ctx.needs_input_grad[0]
        want_x = ctx.needs_input_grad[1]
        if not (want_gg or want_x):
            return None, None, None, None, None
        ggY, g2 = _native.sph_double_backward(xyz, grad_Y.contiguous(), v.contiguous(), ctx.l_max,
                                              ctx.normalize, want_grad_grad_Y=want_gg, want_grad_xyz=want_x)
        return ggY, g2, None, None, None


class _Sph(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, l_max, normalize):
        ctx.l_max = l_max
        ctx.normalize = normalize
        if xyz.requires_grad:
            Y, dY = _native.sph_compute_with_gradients(xyz, l_max, normalize)
            ctx.save_for_backward(xyz, dY)
        else:
            Y = _native.sph_compute(xyz, l_max, normalize)
            ctx.save_for_backward(xyz, None)
        return Y

    @staticmethod
    def backward(ctx, grad_Y):
        xyz, dY = ctx.saved_tensors
        if dY is None:
            _, dY = _native.sph_compute_with_gradients(xyz.detach(), ctx.l_max, ctx.normalize)
        gx = _SphBackward.apply(grad_Y, xyz, dY, ctx.l_max, ctx.normalize)
        return gx, None, None


def spherical_harmonics(xyz: torch.Tensor, l_max: int, normalize: bool = True) -> torch.Tensor:
    """Y[n,(l_max+1)^2] for points xyz[n,3]; differentiable twice w.r.t. xyz.

    ``normalize=False`` gives the scaled (solid) harmonics r^l Y_l^m.
    """
    return _Sph.apply(xyz.contiguous(), int(l_max), bool(normalize))


def spherical_harmonics_with_gradients(xyz: torch.Tensor, l_max: int, normalize: bool = True):
    """(Y, dY) without autograd: dY[n,3,K] = dY/dxyz from the same pass."""
    with torch.no_grad():
        return _native.sph_compute_with_gradients(xyz.contiguous(), l_max, normalize)


class _SphE3nn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, l_max, normalize, normalization):
        ctx.l_max = l_max
        xp = _native.sph_e3nn_coordinates(xyz)
        Y, dY = _native.sph_compute_with_gradients(xp, l_max, normalize)
        _native.sph_e3nn_convert(Y, dY, l_max, normalization)
        ctx.save_for_backward(dY)
        return Y

    @staticmethod
    def backward(ctx, grad_Y):
        (dY,) = ctx.saved_tensors
        return _native.sph_backward(dY, grad_Y.contiguous(), ctx.l_max), None, None, None


def e3nn_spherical_harmonics(xyz: torch.Tensor, l_max: int, normalize: bool = True,
                             normalization: str = "integral") -> torch.Tensor:
    """Y[n,(l_max+1)^2] in e3nn's convention (Sec. III.B): degrees 0..l_max,
    y as the polar axis, ``normalization`` "integral", "component" or
    "norm"; differentiable once w.r.t. xyz.  Permutation, forward and
    conversion all run in the library's kernels (include/sph.h:
    sph_e3nn_coordinates, sph_e3nn_convert)."""
    if normalization not in _native.E3NN_NORMALIZATIONS:
        raise ValueError(f"normalization must be one of {sorted(_native.E3NN_NORMALIZATIONS)}")
    return _SphE3nn.apply(xyz.contiguous(), int(l_max), bool(normalize), normalization)


def e3nn_spherical_harmonics_with_gradients(xyz: torch.Tensor, l_max: int, normalize: bool = True,
                                            normalization: str = "integral"):
    """(Y, dY) in e3nn's convention without autograd; dY[n,3,K] along x, y, z."""
    with torch.no_grad():
        xp = _native.sph_e3nn_coordinates(xyz.contiguous())
        Y, dY = _native.sph_compute_with_gradients(xp, l_max, normalize)
        return _native.sph_e3nn_convert(Y, dY, l_max, normalization)


class SphericalHarmonics(torch.nn.Module):
    """Module form: ``SphericalHarmonics(l_max, normalize)(xyz) -> Y``."""

    def __init__(self, l_max: int, normalize: bool = True):
        super().__init__()
        if not 0 <= int(l_max) <= 32:
            raise ValueError("l_max must be in [0, 32]")
        self.l_max = int(l_max)
        self.normalize = bool(normalize)

    def forward(self, xyz: torch.Tensor) -> torch.Tensor:
        return spherical_harmonics(xyz, self.l_max, self.normalize)

    def compute_with_gradients(self, xyz: torch.Tensor):
        return spherical_harmonics_with_gradients(xyz, self.l_max, self.normalize)

    def extra_repr(self) -> str:
        return f"l_max={self.l_max}, normalize={self.normalize}"
