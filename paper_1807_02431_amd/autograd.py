"""Differentiable potential energy of a batch of replicas, as a torch.autograd.Function over the
C ABI: gpr_energy_forces_dev for the forward pass, gpr_energy_backward_dev for dU/dx = -F and the
force-field parameter gradient (Lennard-Jones epsilon and sigma, charges, torsion constants).

    model = EnergyModel(spec)                     # the system's topology and parameters
    U = model(x, eps, sigma, charge, torsion_k)   # x: [R, 3, n] CUDA tensor; U: [R] float64
    U.sum().backward()                            # x.grad = -F, eps.grad = sum_r dU_r/d eps, ...

Every step of the computation runs in the HIP library; torch provides the device memory and
the stream.  A forward pass sets the positions of the system's replicas to x.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gpr


class EnergyModel:
    """Energy U_r(x_r; eps, sigma, charge, torsion_k) of the replicas of one molecular system."""

    def __init__(self, spec: dict, stream=None):
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        self.system = gpr.System(spec, path=gpr.PATH_PLAIN, stream=stream)
        self.n, self.R, self.nt = self.system.n, self.system.R, self.system.nt
        self._params = tuple(np.asarray(spec[k], np.float64).copy()
                             for k in ("epsilon", "sigma", "charge", "torsion_k"))
        self._gen = 0          # count of forward evaluations (positions last set by which one)

    def parameters(self, device="cuda"):
        """The current (epsilon, sigma, charge, torsion_k) as float64 tensors."""
        return tuple(torch.tensor(p, dtype=torch.float64, device=device) for p in self._params)

    def _sync_params(self, *tensors):
        new = tuple(t.detach().to("cpu", torch.float64).numpy() for t in tensors)
        if any(a.shape != b.shape for a, b in zip(new, self._params)):
            raise ValueError("parameter shapes must be (n,), (n,), (n,), (n_torsions,)")
        if not all(np.array_equal(a, b) for a, b in zip(new, self._params)):
            self.system.set_params(*new)
            self._params = tuple(a.copy() for a in new)

    def __call__(self, x, epsilon, sigma, charge, torsion_k):
        return _Energy.apply(self, x, epsilon, sigma, charge, torsion_k)


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, x, epsilon, sigma, charge, torsion_k):
        if x.shape != (model.R, 3, model.n) or not x.is_cuda:
            raise ValueError("x must be a CUDA tensor of shape [n_replicas, 3, n_atoms]")
        model._sync_params(epsilon, sigma, charge, torsion_k)
        x32 = x.detach().to(torch.float32).contiguous()
        U = torch.empty(model.R, dtype=torch.float64, device=x.device)
        model.system.energy_forces_dev(x32.data_ptr(), U.data_ptr(), 0)
        model._gen += 1
        ctx.model, ctx.gen, ctx.x_dtype = model, model._gen, x.dtype
        # the parameters this pass used (host copies, owned by the pass): a later pass with
        # other parameters must not change what this pass's backward differentiates
        ctx.params = tuple(a.copy() for a in model._params)
        ctx.save_for_backward(x32)
        return U

    @staticmethod
    def backward(ctx, gU):
        model = ctx.model
        x32, = ctx.saved_tensors
        g = gU.detach().to(torch.float64).contiguous()
        stale_params = not all(np.array_equal(a, b) for a, b in zip(ctx.params, model._params))
        if stale_params:
            # a later forward pass changed the parameters: put this pass's back
            model.system.set_params(*ctx.params)
            model._params = tuple(a.copy() for a in ctx.params)
        if model._gen != ctx.gen or stale_params:
            # a later forward pass moved the replicas: put this pass's positions (and forces) back
            model.system.energy_forces_dev(x32.data_ptr(), 0, 0)
            model._gen += 1
            ctx.gen = model._gen
        dev = x32.device
        gx = torch.empty_like(x32) if ctx.needs_input_grad[1] else None
        want = any(ctx.needs_input_grad[2:6])
        ge = gs = gq = gk = None
        if want:
            ge, gs, gq = (torch.empty(model.n, dtype=torch.float64, device=dev) for _ in range(3))
            gk = torch.empty(max(1, model.nt), dtype=torch.float64, device=dev)
        ptr = lambda t: 0 if t is None else t.data_ptr()
        model.system.energy_backward_dev(g.data_ptr(), ptr(gx), ptr(ge), ptr(gs), ptr(gq), ptr(gk))
        if gx is not None:
            gx = gx.to(ctx.x_dtype)
        if gk is not None:
            gk = gk[: model.nt]
        return None, gx, ge, gs, gq, gk
