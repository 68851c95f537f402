"""Gradient of a liquid-composition loss through the hand-written adjoint step.

LiquidCompositionLoss is a torch.autograd.Function whose forward runs the model
on the GPU from a parameter vector theta = (k_ij for i < j, a_1..a_nc, b_1..b_nc)
and returns L = sum_i (x_i - x_target_i)^2 of the bulk liquid mole fractions
after `nsteps` steps; the same library call (lbm_adjoint) runs the discrete
adjoint back through the run from checkpoints every `checkpoint_every` steps,
and backward returns grad_output * dL/dtheta.  Only argument marshalling happens
here: every step, forward and reverse, runs in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lbm


def pair_index(nc):
    return [(i, j) for i in range(nc) for j in range(i + 1, nc)]


def theta_of(mix: dict) -> np.ndarray:
    nc = len(mix["a"])
    k = np.asarray(mix["k"], dtype=np.float64)
    return np.concatenate([[k[i, j] for i, j in pair_index(nc)], np.asarray(mix["a"], dtype=np.float64),
                           np.asarray(mix["b"], dtype=np.float64)])


def mixture_with(theta, base: dict) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    nc = len(base["a"])
    npair = nc * (nc - 1) // 2
    k = np.zeros((nc, nc))
    for v, (i, j) in zip(theta[:npair], pair_index(nc)):
        k[i, j] = k[j, i] = v
    out = dict(base)
    out["k"] = k
    out["a"] = theta[npair:npair + nc].copy()
    out["b"] = theta[npair + nc:].copy()
    return out


def pack_gradient(d_k, d_a, d_b) -> np.ndarray:
    nc = len(d_a)
    return np.concatenate([[d_k[i, j] for i, j in pair_index(nc)], d_a, d_b])


@dataclass
class AdjointSpec:
    """Everything but theta: the mixture's omega, M, R, the box and the loss."""
    mix: dict
    lattice: str
    shape: tuple
    T: float
    tau: float
    beta: float
    gamma: np.ndarray
    rho0: np.ndarray
    mask: np.ndarray
    x_target: np.ndarray
    nsteps: int
    checkpoint_every: int = 100
    storage: str = "f32"
    forcing: str = "edm"       # "edm" or "guo"
    collision: str = "bgk"     # "bgk" or "mrt"
    mrt_s: np.ndarray = None   # MRT relaxation rate per moment row


def run(theta, spec: AdjointSpec):
    """(loss, x_liq, dL/dtheta) for the parameter vector theta."""
    ctx = lbm.LbmContext(mixture_with(theta, spec.mix), spec.lattice, spec.shape, spec.T, spec.tau, spec.beta,
                         spec.gamma, spec.rho0, collision=spec.collision, forcing=spec.forcing, storage=spec.storage,
                         mrt_s=spec.mrt_s)
    try:
        r = ctx.adjoint(spec.nsteps, spec.checkpoint_every, spec.mask, spec.x_target)
    finally:
        ctx.close()
    return r["loss"], r["x_liq"], pack_gradient(r["d_k"], r["d_a"], r["d_b"])


def loss_only(theta, spec: AdjointSpec):
    """(loss, x_liq) for theta from the forward steps alone (no reverse pass): the
    liquid mole fractions over the mask from the final cell-volume densities."""
    ctx = lbm.LbmContext(mixture_with(theta, spec.mix), spec.lattice, spec.shape, spec.T, spec.tau, spec.beta,
                         spec.gamma, spec.rho0, collision=spec.collision, forcing=spec.forcing, storage=spec.storage,
                         mrt_s=spec.mrt_s)
    try:
        ctx.step(spec.nsteps)
        ctx.check()
        rho = ctx.moments(totals=False)["rho_s"].cpu().numpy()
    finally:
        ctx.close()
    M = np.asarray(spec.mix["M"], dtype=np.float64)
    mask = np.asarray(spec.mask, dtype=bool)
    N = np.array([rho[i][mask].sum() / M[i] for i in range(rho.shape[0])])
    x = N / N.sum()
    return float(np.sum((x - np.asarray(spec.x_target, dtype=np.float64)) ** 2)), x


def _function():
    import torch

    class LiquidCompositionLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, spec):
            th = theta.detach().cpu().double().numpy()
            if ctx.needs_input_grad[0]:
                loss, _, grad = run(th, spec)
                # the gradient is kept in float64; backward casts only what it returns
                ctx.save_for_backward(torch.as_tensor(grad, dtype=torch.float64, device=theta.device))
            else:                      # no gradient wanted: the forward steps only
                loss, _ = loss_only(th, spec)
            return torch.as_tensor(loss, dtype=theta.dtype, device=theta.device)

        @staticmethod
        def backward(ctx, grad_output):
            (g,) = ctx.saved_tensors
            return (grad_output.to(torch.float64) * g).to(grad_output.dtype), None

    return LiquidCompositionLoss


_FN = None


def liquid_composition_loss(theta, spec: AdjointSpec):
    """Differentiable L(theta) (torch scalar) for a theta tensor."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(theta, spec)
