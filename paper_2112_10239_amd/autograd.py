"""``torch.autograd.Function`` over the library's forward pass and adjoint backward.

The paper (Sec. 2, Sec. 3) gets gradients of expectation values by PyTorch
Autograd backpropagation through the whole contraction.  Here the forward
keeps only the final state of every batch row on the device, and the backward
calls the library's adjoint sweep, which recomputes earlier states by
applying inverse gates in reverse order (no stored activations).  torch only
provides the parameter tensor, the stream and the chain-rule product with the
incoming gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import qsim


def _stream_handle(t: torch.Tensor):
    if t.is_cuda:
        return torch.cuda.current_stream(t.device).cuda_stream
    return None


def _params(theta: torch.Tensor):
    """Parameters as the library takes them: a float64 device tensor stays on the
    device (the library builds gate coefficients from it there); host tensors go
    as float64 arrays."""
    th = theta.detach().reshape(theta.shape[0], -1)
    if th.is_cuda:
        return th.to(torch.float64).contiguous()
    return th.to(torch.float64).contiguous().numpy()


class Expectation(torch.autograd.Function):
    """E[b] = <psi(theta_b)|H|psi(theta_b)> for theta of shape [B, P]."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, engine: "qsim.Context", circuit, hamiltonian):
        th = _params(theta)
        stream = _stream_handle(theta)
        E, state = engine.expect_circuit(circuit, hamiltonian, th, mode=qsim.MODE_DENSE, dtype=qsim.C64,
                                         stream=stream, keep=True)
        ctx.engine, ctx.circuit, ctx.hamiltonian, ctx.state, ctx.th = engine, circuit, hamiltonian, state, th
        ctx.stream = stream
        return torch.as_tensor(np.asarray(E, dtype=np.float64).reshape(-1), device=theta.device).to(theta.dtype)

    @staticmethod
    def backward(ctx, grad_E: torch.Tensor):
        _, g = ctx.engine.expect_grad(ctx.circuit, ctx.hamiltonian, ctx.th, dtype=qsim.C64, stream=ctx.stream,
                                      saved=ctx.state, want_E=False)
        ctx.state.destroy()
        ctx.state = None
        g = torch.as_tensor(np.asarray(g).reshape(tuple(ctx.th.shape)), device=grad_E.device, dtype=grad_E.dtype)
        ctx.th = None
        return grad_E.reshape(-1, 1) * g, None, None, None


def expectation(theta: torch.Tensor, engine: "qsim.Context", circuit, hamiltonian) -> torch.Tensor:
    """Differentiable <H>; theta [B, P] -> [B]."""
    return Expectation.apply(theta, engine, circuit, hamiltonian)


class ExpectationCones(torch.autograd.Function):
    """E[b] for theta of shape [B, P] with every term on light cones (n in the hundreds).

    When theta needs a gradient, the forward call already runs the adjoint sweep
    inside every cone (it costs little more than the cones' forward pass) and the
    backward only applies the chain rule."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, engine: "qsim.Context", circuit, hamiltonian, mode: int):
        th = _params(theta)
        stream = _stream_handle(theta)
        if theta.requires_grad:
            E, g = engine.expect_grad(circuit, hamiltonian, th, dtype=qsim.C64, stream=stream, mode=mode)
            ctx.grad = np.asarray(g).reshape(tuple(th.shape))
        else:
            E = engine.expect_circuit(circuit, hamiltonian, th, mode=mode, dtype=qsim.C64, stream=stream)
            ctx.grad = None
        return torch.as_tensor(np.asarray(E, dtype=np.float64).reshape(-1), device=theta.device).to(theta.dtype)

    @staticmethod
    def backward(ctx, grad_E: torch.Tensor):
        g = torch.as_tensor(ctx.grad, device=grad_E.device, dtype=grad_E.dtype)
        ctx.grad = None
        return grad_E.reshape(-1, 1) * g, None, None, None, None


def expectation_cones(theta: torch.Tensor, engine: "qsim.Context", circuit, hamiltonian,
                      mode: int = qsim.MODE_LIGHTCONE_FACTORED) -> torch.Tensor:
    """Differentiable <H> evaluated on light cones; theta [B, P] -> [B]."""
    return ExpectationCones.apply(theta, engine, circuit, hamiltonian, mode)
