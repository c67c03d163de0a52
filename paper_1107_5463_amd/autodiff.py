"""Derivatives of the Ising partition function through Monte Carlo chains.

With Z(J, beta) = sum_s exp(beta sum_b J_b x_b) (Eq. (1), x_b = s_i s_j the
product across bond b, real couplings J_b):

    d ln Z / d J_b   = beta <x_b>
    d ln Z / d beta  = sum_b J_b <x_b> = -<H>
    d <x_a> / d J_b  = beta Cov(x_a, x_b)
    d <x_a> / d beta = Cov(x_a, sum_b J_b x_b)

Every step runs in the library's kernels: `smc_chains_sample` sums x_b over
chains and sweeps; `smc_chains_mean` forms <x_b>; `smc_chains_covariance`
replays the same sweeps from the saved start state and counter
(counter-based random numbers make the replay exact) and sums (G - c) x_b for
G = sum_a g_a x_a, the vector-Jacobian product's weights, centred on
c = sum_a g_a <x_a> from `smc_chains_dot`; `smc_chains_vjp`,
`smc_chains_lnz_grad` and `smc_chains_fit_step` finish the gradients and the
moment-matching update in FP64.  Nothing is stored per sample.  This module
allocates the tensors, converts the cotangents to the library's dtypes and
calls the binding -- no arithmetic of the method runs in torch.

All arrays over bonds have the coupling layout [d, 2, N/2] (bond (mu, c, j)
from site (c, j) of colour plane c to its +mu neighbour).
"""
import torch

from . import Chains

__all__ = ["bond_correlations", "log_partition", "log_partition_grad", "fit_couplings",
           "BondCorrelations", "LogPartition"]


def _sample_mean(chains: Chains, beta: float, n_sweeps: int, n_burn: int):
    if n_burn:
        chains.sample(beta, n_burn)
    acc = chains.bond_zeros()
    chains.sample(beta, n_sweeps, acc)
    return chains.mean(acc, chains.n_chains * n_sweeps)


def _f32(J):
    return J.detach().to(torch.float32).contiguous()


class BondCorrelations(torch.autograd.Function):
    """<x_b> under couplings J at inverse temperature beta, differentiable in
    J and beta through the covariance replay."""

    @staticmethod
    def forward(ctx, J, beta, chains: Chains, n_sweeps: int, n_burn: int):
        b = float(beta)
        chains.set_couplings(J.detach())
        if n_burn:
            chains.sample(b, n_burn)
        start = chains.spins.clone()
        t0 = chains.t
        mean = _sample_mean(chains, b, n_sweeps, 0)
        ctx.chains, ctx.b, ctx.n_sweeps, ctx.t0 = chains, b, n_sweeps, t0
        ctx.beta_dtype = beta.dtype if torch.is_tensor(beta) else torch.float64
        ctx.J_dtype = J.dtype
        ctx.save_for_backward(_f32(J).clone(), mean, start)
        return mean.to(J.dtype)

    @staticmethod
    def backward(ctx, grad):
        J, mean, start = ctx.saved_tensors
        ch = ctx.chains
        # replay the forward sweeps from their start, then put the chains back
        end, t_end, J_now = ch.spins.clone(), ch.t, ch.J.clone()
        ch.set_couplings(J)
        ch.spins.copy_(start)
        ch.t = ctx.t0
        g = grad.to(torch.float64).contiguous()
        center = ch.dot(g, mean)
        cov_acc = torch.zeros_like(mean)
        G_acc = torch.zeros(2, dtype=torch.float64, device=mean.device)
        ch.covariance(ctx.b, ctx.n_sweeps, g, center, cov_acc, G_acc)
        grad_J, grad_beta = ch.vjp(ctx.b, ch.n_chains * ctx.n_sweeps, cov_acc, G_acc, mean, J)
        ch.spins.copy_(end)
        ch.t = t_end
        ch.set_couplings(J_now)
        return (grad_J.to(ctx.J_dtype), grad_beta.reshape(()).to(ctx.beta_dtype), None, None,
                None)


def bond_correlations(J, beta, chains: Chains, n_sweeps: int, n_burn: int = 0):
    """Estimate <x_b> (shape of J); differentiable in J and beta."""
    if not torch.is_tensor(beta):
        beta = torch.tensor(float(beta), dtype=torch.float64)
    return BondCorrelations.apply(J, beta, chains, n_sweeps, n_burn)


class LogPartition(torch.autograd.Function):
    """A zero-valued stand-in for ln Z whose gradients are those of ln Z:
    d/dJ_b = beta <x_b>, d/dbeta = sum_b J_b <x_b>.  Monte Carlo estimates
    the derivatives of ln Z, not ln Z itself, so the forward value is 0; add
    it to a loss (e.g. the negative log-likelihood -beta sum_b J_b x_b^data +
    ln Z) for its gradient."""

    @staticmethod
    def forward(ctx, J, beta, chains: Chains, n_sweeps: int, n_burn: int):
        b = float(beta)
        chains.set_couplings(J.detach())
        mean = _sample_mean(chains, b, n_sweeps, n_burn)
        ctx.chains, ctx.b = chains, b
        ctx.beta_dtype = beta.dtype if torch.is_tensor(beta) else torch.float64
        ctx.J_dtype = J.dtype
        ctx.save_for_backward(_f32(J), mean)
        return torch.zeros((), dtype=J.dtype, device=J.device)

    @staticmethod
    def backward(ctx, grad):
        J, mean = ctx.saved_tensors
        scale = grad.detach().to(torch.float64).reshape(1).contiguous()
        gJ, gb = ctx.chains.lnz_grad(ctx.b, mean, J, scale=scale)
        return gJ.to(ctx.J_dtype), gb.reshape(()).to(ctx.beta_dtype), None, None, None


def log_partition(J, beta, chains: Chains, n_sweeps: int, n_burn: int = 0):
    if not torch.is_tensor(beta):
        beta = torch.tensor(float(beta), dtype=torch.float64)
    return LogPartition.apply(J, beta, chains, n_sweeps, n_burn)


def log_partition_grad(J, beta: float, chains: Chains, n_sweeps: int, n_burn: int = 0):
    """(d ln Z / d J, d ln Z / d beta) = (beta <x>, sum_b J_b <x_b>): a float64
    tensor over the bonds and a Python float."""
    chains.set_couplings(J)
    mean = _sample_mean(chains, float(beta), n_sweeps, n_burn)
    gJ, gb = chains.lnz_grad(float(beta), mean, _f32(J), dtype=torch.float64)
    return gJ, float(gb.item())


def fit_couplings(target, beta: float, chains: Chains, steps: int, lr: float, n_sweeps: int,
                  n_burn: int = 0, J_init=None, history=None):
    """Moment matching: ascend the log-likelihood of data with bond
    correlations `target`, whose gradient in J is beta (target - <x>_J).
    Returns the fitted couplings (float32, coupling layout)."""
    J = (J_init if J_init is not None else chains.J).detach().to(torch.float32).clone()
    tgt = target.detach().to(torch.float64).contiguous()
    for _ in range(steps):
        chains.set_couplings(J)
        model = _sample_mean(chains, float(beta), n_sweeps, n_burn)
        chains.fit_step(float(beta), float(lr), tgt, model, J)
        if history is not None:
            history.append(J.clone())
    return J
