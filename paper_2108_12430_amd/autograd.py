"""DeepClean retraining through torch.autograd.

``DeepCleanFn`` wraps the library's batch-statistics forward and its
hand-written backward (deepclean_forward with GW_TRAIN, deepclean_backward)
so a torch optimizer can update the flat parameter vector.  The gradient is
taken with respect to the parameters only (the witness windows are data).
PyTorch is used for tensors and the optimizer; every convolution,
normalisation and reduction of the step runs in the library's kernels.
"""
from __future__ import annotations

import torch

from . import gwstream as gs


class DeepCleanFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, x, model, recompute=True):
        # model.params must alias `params` (the library reads weights through it)
        if model.params.data_ptr() != params.data_ptr():
            raise ValueError("model was created on a different parameter tensor")
        flags = gs.TRAIN | (gs.RECOMPUTE if recompute else 0)
        x = x.contiguous()
        n, W = x.shape[0], x.shape[-1]
        noise = torch.empty((n, W), dtype=torch.float32, device=x.device)
        ws = model.forward(x=x, noise=noise, flags=flags)
        ctx.model = model
        ctx.flags = flags
        ctx.save_for_backward(x, ws)
        return noise

    @staticmethod
    def backward(ctx, dnoise):
        x, ws = ctx.saved_tensors
        dparams = torch.empty_like(ctx.model.params)
        ctx.model.backward(x, dnoise.contiguous(), ws, dparams, flags=ctx.flags)
        return dparams, None, None, None


def bandpass_mse_loss(strain, noise, fs=4096.0, f_lo=55.0, f_hi=65.0):
    """Band-passed MSE as an autograd-aware scalar (gw_bandpass_mse)."""
    return _BandpassMSE.apply(strain, noise, fs, f_lo, f_hi)


class _BandpassMSE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, strain, noise, fs, f_lo, f_hi):
        loss, dn = gs.bandpass_mse(strain.contiguous(), noise.contiguous(), fs, f_lo, f_hi, want_grad=True)
        ctx.save_for_backward(dn)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (dn,) = ctx.saved_tensors
        return None, dn * g, None, None, None


def train_step(model, params, opt, x, strain, fs=4096.0, recompute=True):
    """One retraining step: forward, band-passed loss, backward, optimizer
    update; refreshes the model's packed inference data afterwards."""
    opt.zero_grad(set_to_none=True)
    noise = DeepCleanFn.apply(params, x, model, recompute)
    loss = bandpass_mse_loss(strain, noise, fs)
    loss.backward()
    opt.step()
    model.refresh()
    return loss.detach()
