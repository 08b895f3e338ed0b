"""The codec as a differentiable layer (straight-through quantizer).

SteCoder.apply(attr, pos, params) runs the HIP encoder through gsc_ste_forward and returns, for
the Nv occupied voxels in Morton order, the dequantized coefficients yhat, the decoded
attributes ahat = T^T yhat and the voxel means aref (not differentiable). Its backward runs
gsc_ste_backward: the quantizer passes gradients unchanged, the transform's adjoint (the
inverse RAHT) maps them back to voxels, and each Gaussian receives its voxel's gradient divided
by the voxel's member count.

rd_loss is the rate-distortion objective of the differentiable workload: the mean squared error
of the decoded attributes against the voxel means plus lambda times the rate proxy
sum log2(1 + |yhat| / step).
"""
from __future__ import annotations

import torch

from . import gsc


class SteCoder(torch.autograd.Function):
    @staticmethod
    def forward(ctx, attr, pos, params):
        if not attr.is_cuda:
            raise ValueError("SteCoder runs on the GPU only")
        fwd = gsc.ste_forward(pos.contiguous(), attr.detach().contiguous(), params)
        fwd.encoded.check()                 # synchronizes: Nv sizes the outputs
        nv = fwd.encoded.n_vox()
        ctx.fwd, ctx.nv = fwd, nv
        aref = fwd.aref[:nv]
        ctx.mark_non_differentiable(aref)
        return fwd.yhat[:nv], fwd.ahat[:nv], aref

    @staticmethod
    def backward(ctx, g_yhat, g_ahat, _g_aref):
        fwd, nv = ctx.fwd, ctx.nv
        C = fwd.encoded.C
        dev = fwd.yhat.device
        z = None
        if g_yhat is None or g_ahat is None:
            z = torch.zeros((max(nv, 1), C), dtype=torch.float32, device=dev)
        gy = z if g_yhat is None else g_yhat.float().contiguous()
        ga = z if g_ahat is None else g_ahat.float().contiguous()
        grad, info = gsc.ste_backward(fwd, gy, ga)
        return grad[:fwd.n], None, None


def rd_loss(yhat, ahat, aref, steps, lam):
    """(loss, distortion, rate): mean((ahat - aref)^2) + lam * sum(log2(1 + |yhat| / steps))."""
    dist = ((ahat - aref) ** 2).mean()
    rate = lam * torch.log2(1.0 + yhat.abs() / steps).sum()
    return dist + rate, dist, rate
