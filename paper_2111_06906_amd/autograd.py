"""Differentiation form: deposited photon energy as a differentiable function of
per-material albedo and per-light radiant power.

E[r, p, c] = Phi[l(p), c] / N_l * prod_{i<=r} albedo[m(x_i), c]   (r < n_p; 0 beyond)

with the validity masks (which paths exist, how long they are, which surfaces
they hit) held fixed: they come from the stored path geometry.  The forward
recomputes the throughputs from the stored hit ids instead of storing them;
the backward is a hand-written kernel (prefix products and a reverse
recurrence, block partials reduced in FP64).  Both run in libpv.so.
"""
from __future__ import annotations

import torch


class EnergyFn(torch.autograd.Function):
    """E = EnergyFn.apply(albedo [M,3], power [L,3], ctx, store) -> [B, N, 3]."""

    @staticmethod
    def forward(fctx, albedo, power, context, store):
        if albedo.dtype != torch.float32 or power.dtype != torch.float32:
            raise TypeError("albedo and power must be float32")
        if not albedo.is_cuda or not power.is_cuda:
            raise TypeError("albedo and power must be device tensors")
        a = albedo.detach().contiguous()
        p = power.detach().contiguous()
        E = context.energy_forward(store, a, p)
        fctx.save_for_backward(a, p)
        fctx.context = context
        fctx.store = store
        return E

    @staticmethod
    def backward(fctx, gE):
        a, p = fctx.saved_tensors
        ga, gp = fctx.context.energy_backward(fctx.store, a, p, gE.contiguous().to(torch.float32))
        return ga, gp, None, None


def deposited_energy(context, store, albedo, power):
    """Differentiable deposited energy of every photon slot of the store."""
    return EnergyFn.apply(albedo, power, context, store)
