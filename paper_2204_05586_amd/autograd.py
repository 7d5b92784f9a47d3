"""Final-state populations as differentiable torch functions of field
parameters: ``torch.autograd.Function`` over the adjoint kernel
(``mss_adjoint_*``).

The forward pass runs the adjoint plan once on the current parameters: it
produces loss_i = |psi_final_i[m]|^2 for every simulation of the plan and,
in the same launch sequence, d loss_i / d params (discrete adjoint with
interval checkpoints).  The backward pass only scales those saved
gradients by the incoming gradient of each loss.  There are no
gradients with respect to the initial states.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import native


def _torch():
    import torch
    return torch


class _FinalPopulation:
    """Holder for the autograd Function (built on first use so importing
    this module does not import torch)."""
    fn = None


def _function():
    if _FinalPopulation.fn is not None:
        return _FinalPopulation.fn
    torch = _torch()

    class FinalPopulation(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, plan, bufs, owner):
            if params is not None:
                bufs["params"].copy_(params.detach())
            plan.run(bufs)  # on the current stream, like the copies around it
            grad = bufs["grad"][:plan.n_grad].clone()
            ctx.save_for_backward(grad)
            ctx.owner = owner
            return bufs["loss"].clone()

        @staticmethod
        def backward(ctx, grad_loss):
            (grad,) = ctx.saved_tensors
            if not ctx.needs_input_grad[0]:
                return None, None, None, None
            return grad * grad_loss[ctx.owner], None, None, None

    _FinalPopulation.fn = FinalPopulation
    return FinalPopulation


class PopulationModel:
    """Differentiable populations of a batch of simulations.

    problems: list of ``workloads.Problem`` whose parameter slots hold the
    controls (x / y terms; see ``mss_adjoint_plan_create``); level_m: the
    index m of the population |psi_final[m]|^2.  The packed parameter
    vector concatenates the problems' parameter vectors in order;
    ``initial_params()`` returns it as a device tensor.

    specialize: compile the problems' shared field program into the
    forward pass (same losses and gradients, a faster forward).

    ``model(params)`` returns the [n] losses with gradient flowing to
    ``params`` (float64, on the device, length ``n_params``).  Everything
    runs on torch's current stream.  Calls reuse the model's buffers, so one
    model is not for concurrent use from several threads."""

    def __init__(self, problems, level_m: int, device: str = "cuda", specialize: bool = False):
        torch = _torch()
        self.plan = native.AdjointPlan(problems, level_m, specialize=specialize)
        self.bufs = self.plan.allocate(device)
        self.n_params = int(self.plan.n_grad)
        owner = np.zeros(max(1, self.n_params), dtype=np.int64)
        for i, pk in enumerate(self.plan.packed):
            a = int(self.plan.param_off[i])
            owner[a:a + pk.n_params] = i
        self.owner = torch.from_numpy(owner[:self.n_params]).to(device)
        self.device = device

    def initial_params(self):
        p = self.bufs["params"]
        return p.clone() if p is not None else _torch().zeros(0, dtype=_torch().float64,
                                                              device=self.device)

    def __call__(self, params):
        torch = _torch()
        if self.n_params:
            if params is None or params.dtype != torch.float64 or params.numel() != self.n_params:
                raise ValueError(f"params must be float64 with {self.n_params} entries")
            if params.device != self.bufs["params"].device:
                raise ValueError("params must live on the plan's device")
        return _function().apply(params.contiguous() if self.n_params else None, self.plan,
                                 self.bufs, self.owner)

    def final_states(self):
        """Final states of the last call (packed as mss_batch_layout)."""
        return self.bufs["psi_final"]

    def close(self):
        self.plan.close()


def final_population(problems, level_m: int, params,
                     model: Optional[PopulationModel] = None):
    """One-shot form: losses of ``problems`` at ``params`` (differentiable),
    computed on the current stream."""
    m = model or PopulationModel(problems, level_m, device=str(params.device))
    return m(params)
