"""The codec as a differentiable layer (straight-through quantizer).

SteCoder.apply(attr, pos, params) runs the HIP encoder through gsc_ste_forward and returns, for
the Nv occupied voxels in Morton order, the dequantized coefficients yhat, the decoded
attributes ahat = T^T yhat and the voxel means aref (not differentiable). Its backward runs
gsc_ste_backward: the quantizer passes gradients unchanged, the transform's adjoint (the
inverse RAHT) maps them back to voxels, and each Gaussian receives its voxel's gradient divided
by the voxel's member count. Nv is only known once the encoder has run, so this form waits for
the device to cut the outputs to Nv rows.

SteCoderPadded.apply(attr, pos, params) is the same layer without that wait, for training loops
that must not stall on the device: it returns n rows (its outputs start zeroed and the kernels
write rows below Nv only, so rows past Nv are zero) and Nv as a one-element device tensor.
Nothing in its forward or backward synchronizes the host. A device-detected error (corrupt
input, capacity) leaves Nv = 0, which makes rd_loss's distortion NaN.

rd_loss is the rate-distortion objective of the differentiable workload: the mean squared error
of the decoded attributes against the voxel means plus lambda times the rate proxy
sum log2(1 + |yhat| / step).
"""
from __future__ import annotations

import torch

from . import gsc


def _backward(ctx, g_yhat, g_ahat):
    fwd = ctx.fwd
    C = fwd.encoded.C
    dev = fwd.yhat.device
    z = None
    if g_yhat is None or g_ahat is None:
        z = torch.zeros((max(fwd.n, 1), C), dtype=torch.float32, device=dev)
    gy = z if g_yhat is None else g_yhat.float().contiguous()
    ga = z if g_ahat is None else g_ahat.float().contiguous()
    # the kernels read rows < Nv of the gradients (Nv from the workspace, on the device)
    grad, _info = gsc.ste_backward(fwd, gy, ga)
    return grad[:fwd.n]


class SteCoder(torch.autograd.Function):
    @staticmethod
    def forward(ctx, attr, pos, params):
        if not attr.is_cuda:
            raise ValueError("SteCoder runs on the GPU only")
        fwd = gsc.ste_forward(pos.contiguous(), attr.detach().contiguous(), params)
        fwd.encoded.check()                 # synchronizes: Nv sizes the outputs
        nv = fwd.encoded.n_vox()
        ctx.fwd = fwd
        aref = fwd.aref[:nv]
        ctx.mark_non_differentiable(aref)
        return fwd.yhat[:nv], fwd.ahat[:nv], aref

    @staticmethod
    def backward(ctx, g_yhat, g_ahat, _g_aref):
        return _backward(ctx, g_yhat, g_ahat), None, None


class SteCoderPadded(torch.autograd.Function):
    @staticmethod
    def forward(ctx, attr, pos, params):
        if not attr.is_cuda:
            raise ValueError("SteCoderPadded runs on the GPU only")
        n = int(pos.shape[0])
        rows = (max(n, 1), int(params.C))
        # zeroed outputs: the kernels write rows below Nv only
        z = [torch.zeros(rows, dtype=torch.float32, device=attr.device) for _ in range(3)]
        fwd = gsc.ste_forward(pos.contiguous(), attr.detach().contiguous(), params, yhat=z[0], ahat=z[1], aref=z[2])
        info = fwd.encoded.info
        # Nv on the device (0 after a device-detected error)
        nv = torch.where(info[0:1] == 0, info[1:2], torch.zeros_like(info[1:2])).to(torch.int64)
        ctx.fwd = fwd
        out = [t[:n] for t in z]
        ctx.mark_non_differentiable(out[2], nv)
        return out[0], out[1], out[2], nv

    @staticmethod
    def backward(ctx, g_yhat, g_ahat, _g_aref, _g_nv):
        return _backward(ctx, g_yhat, g_ahat), None, None


def rd_loss(yhat, ahat, aref, steps, lam, nv=None):
    """(loss, distortion, rate): mean((ahat - aref)^2) + lam * sum(log2(1 + |yhat| / steps)).

    With nv (SteCoderPadded's device count) the rows are the padded ones: the mean is taken over
    the nv voxel rows (the zero rows past them add nothing to either term), with no host wait."""
    sq = (ahat - aref) ** 2
    r = torch.log2(1.0 + yhat.abs() / steps)
    if nv is None:
        dist = sq.mean()
    else:
        dist = sq.sum() / (nv.to(sq.dtype) * sq.shape[1]).reshape(())
    rate = lam * r.sum()
    return dist + rate, dist, rate
