"""Derivatives of the Ising partition function through Monte Carlo chains.

With Z(J, beta) = sum_s exp(beta sum_b J_b x_b) (Eq. (1), x_b = s_i s_j the
product across bond b, real couplings J_b):

    d ln Z / d J_b   = beta <x_b>
    d ln Z / d beta  = sum_b J_b <x_b> = -<H>
    d <x_a> / d J_b  = beta Cov(x_a, x_b)
    d <x_a> / d beta = Cov(x_a, sum_b J_b x_b)

Expectations are estimated by the chains of a `Chains` object (all in the
library's kernels): `smc_chains_sample` sums x_b over chains and sweeps;
`smc_chains_covariance` replays the same sweeps from the saved start state and
counter (counter-based random numbers make the replay exact) and sums
G x_b for G = sum_a g_a x_a, the vector-Jacobian product's weights.  Nothing
is stored per sample.

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
    return acc.double() / float(chains.n_chains * n_sweeps)


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
        ctx.save_for_backward(J.detach().clone(), mean, start)
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
        g_center = float((g * mean).sum())
        cov_acc = torch.zeros_like(mean)
        G_acc = torch.zeros(2, dtype=torch.float64, device=mean.device)
        ch.covariance(ctx.b, ctx.n_sweeps, g, g_center, cov_acc, G_acc)
        S = float(ch.n_chains * ctx.n_sweeps)
        cov = cov_acc / S - (G_acc[0] / S) * mean  # Cov(G, x_b)
        ch.spins.copy_(end)
        ch.t = t_end
        ch.set_couplings(J_now)
        grad_J = (ctx.b * cov).to(J.dtype)
        grad_beta = (J.to(torch.float64) * cov).sum().to(ctx.beta_dtype)
        return grad_J, grad_beta, None, None, None


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
        ctx.b = b
        ctx.beta_dtype = beta.dtype if torch.is_tensor(beta) else torch.float64
        ctx.save_for_backward(J.detach(), mean)
        return torch.zeros((), dtype=J.dtype, device=J.device)

    @staticmethod
    def backward(ctx, grad):
        J, mean = ctx.saved_tensors
        gJ = (grad.to(torch.float64) * ctx.b * mean).to(J.dtype)
        gb = (grad.to(torch.float64) * (J.to(torch.float64) * mean).sum()).to(ctx.beta_dtype)
        return gJ, gb, None, None, None


def log_partition(J, beta, chains: Chains, n_sweeps: int, n_burn: int = 0):
    if not torch.is_tensor(beta):
        beta = torch.tensor(float(beta), dtype=torch.float64)
    return LogPartition.apply(J, beta, chains, n_sweeps, n_burn)


def log_partition_grad(J, beta: float, chains: Chains, n_sweeps: int, n_burn: int = 0):
    """(d ln Z / d J, d ln Z / d beta) = (beta <x>, sum_b J_b <x_b>)."""
    chains.set_couplings(J)
    mean = _sample_mean(chains, float(beta), n_sweeps, n_burn)
    return float(beta) * mean, float((J.to(torch.float64) * mean).sum())


def fit_couplings(target, beta: float, chains: Chains, steps: int, lr: float, n_sweeps: int,
                  n_burn: int = 0, J_init=None, history=None):
    """Moment matching: ascend the log-likelihood of data with bond
    correlations `target`, whose gradient in J is beta (target - <x>_J).
    Returns the fitted couplings (float32, coupling layout)."""
    J = (J_init if J_init is not None else chains.J).detach().to(torch.float32).clone()
    for _ in range(steps):
        chains.set_couplings(J)
        model = _sample_mean(chains, float(beta), n_sweeps, n_burn)
        J = J + (lr * float(beta) * (target.to(torch.float64) - model)).to(torch.float32)
        if history is not None:
            history.append(J.clone())
    return J
