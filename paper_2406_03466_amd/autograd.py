"""torch.autograd.Functions over a qvpu batch. ExpectationFn: forward returns the energies E_b(theta) of
every circuit, backward returns dL/dtheta from one adjoint reverse sweep (qv_batch_gradient with
QV_ADJOINT) seeded with the upstream gradient dL/dE_b. JSDivergenceFn: forward returns the Jensen-Shannon
divergences JS_b(theta) of Eq. 3 against target distributions, backward one adjoint sweep seeded with
dL/dJS_b times the divergence weights (qv_batch_js_gradient). Tensors stay on the device; torch's current
stream orders the work.

Both keep the parameters of their forward call: if the batch received other parameters in between (the
same batch evaluated at several points before one backward), backward sets the saved ones again, and the
gradient call re-runs the forward sweep at them before its reverse sweep."""
from __future__ import annotations

import torch

from . import qvpu


def _restore_params(ctx, batch, th):
    """Sets the forward call's parameters again if the batch has received others since."""
    if batch.param_version != ctx.version:
        batch.set_params(th)
        ctx.version = batch.param_version


class ExpectationFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, batch: "qvpu.Batch"):
        if theta.dtype != torch.float64 or not theta.is_cuda:
            raise TypeError("theta must be a float64 tensor on the batch's device")
        th = theta.detach().contiguous()
        batch.ctx.set_stream(torch.cuda.current_stream(theta.device).cuda_stream)
        batch.set_params(th)
        energies = torch.empty(batch.B, dtype=torch.float64, device=theta.device)
        batch.expectations(energies, None)
        ctx.batch = batch
        ctx.version = batch.param_version
        ctx.save_for_backward(th.clone())
        return energies

    @staticmethod
    def backward(ctx, grad_energies: torch.Tensor):
        batch = ctx.batch
        (th,) = ctx.saved_tensors
        up = grad_energies.detach().to(torch.float64).contiguous()
        grad = torch.empty(batch.n_grad, dtype=torch.float64, device=up.device)
        batch.ctx.set_stream(torch.cuda.current_stream(up.device).cuda_stream)
        _restore_params(ctx, batch, th)
        batch.gradient(qvpu.QV_ADJOINT, upstream=up, grad=grad)
        return grad, None


def expectation(theta: torch.Tensor, batch: "qvpu.Batch") -> torch.Tensor:
    return ExpectationFn.apply(theta, batch)


class JSDivergenceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, batch: "qvpu.Batch", target: torch.Tensor):
        if theta.dtype != torch.float64 or not theta.is_cuda:
            raise TypeError("theta must be a float64 tensor on the batch's device")
        if target.dtype != torch.float64 or not target.is_cuda or target.numel() != batch.n_amplitudes():
            raise TypeError("target must be a float64 device tensor of batch.n_amplitudes() values")
        th = theta.detach().contiguous()
        tg = target.detach().contiguous()
        batch.ctx.set_stream(torch.cuda.current_stream(theta.device).cuda_stream)
        batch.set_params(th)
        js = torch.empty(batch.B, dtype=torch.float64, device=theta.device)
        batch.js_gradient(tg, qvpu.QV_ADJOINT, None, js, None)
        ctx.batch = batch
        ctx.version = batch.param_version
        ctx.save_for_backward(tg, th.clone())
        return js

    @staticmethod
    def backward(ctx, grad_js: torch.Tensor):
        batch = ctx.batch
        (tg, th) = ctx.saved_tensors
        up = grad_js.detach().to(torch.float64).contiguous()
        grad = torch.empty(batch.n_grad, dtype=torch.float64, device=up.device)
        batch.ctx.set_stream(torch.cuda.current_stream(up.device).cuda_stream)
        _restore_params(ctx, batch, th)
        batch.js_gradient(tg, qvpu.QV_ADJOINT, up, None, grad)
        return grad, None, None


def js_divergence(theta: torch.Tensor, batch: "qvpu.Batch", target: torch.Tensor) -> torch.Tensor:
    return JSDivergenceFn.apply(theta, batch, target)
