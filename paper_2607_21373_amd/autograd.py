"""PyTorch autograd wrappers of libpat's forward map and prior factor.

``PatForward`` applies Y = G p0 (Sec. 3 eq. (discrete-wave-matrix)); its backward
is the hand-written transpose sweep G^T (Sec. 5.1, eqs. (backward-recursion) and
(adjoint-verlet)), which is the exact algebraic transpose, so gradients of any
loss of Y are exact.  ``PatPrior`` applies the prior factor L with backward L^T,
and ``PatSpectral`` the spectral-prior map P (latent grid -> nodes) with backward
P^T.  All run entirely in libpat's kernels.

``map_gradient_descent`` minimises the MAP objective of Sec. 5 eq. (MAP),
    f(p) = 1/(2 sigma^2) ||G p - y||^2 + 1/2 ||L p||^2,
by plain gradient descent with step 1/lambda_max(G^T G/sigma^2 + L^T L), the
gradient coming from torch.autograd through the two functions above.
"""
from __future__ import annotations

import torch

from . import pat as _pat


class PatForward(torch.autograd.Function):
    """y = G p0 for p0 [R][N] (float32 or float64 CUDA tensor); backward: G^T."""

    @staticmethod
    def forward(ctx, p0, problem):
        ctx.problem = problem
        return _pat.pat_forward(problem, p0.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return _pat.pat_adjoint(ctx.problem, gy.contiguous()), None


class PatPrior(torch.autograd.Function):
    """L x for x [R][N] float64, L = M_L^{-1/2}(M_L + a K1); backward: L^T."""

    @staticmethod
    def forward(ctx, x, problem, prior_a):
        ctx.problem = problem
        ctx.prior_a = prior_a
        return _pat.pat_prior_apply(problem, x.contiguous(), prior_a, transpose=False)

    @staticmethod
    def backward(ctx, gy):
        return _pat.pat_prior_apply(ctx.problem, gy.contiguous(), ctx.prior_a, transpose=True), None, None


class PatSpectral(torch.autograd.Function):
    """p0 = P w for latent w [R][n^3] (float64) with the handle's spectral prior
    (Sec. 4.1.2 eq. (matern-cov-op), Sec. 6.4); backward: P^T."""

    @staticmethod
    def forward(ctx, w, problem):
        ctx.problem = problem
        return _pat.spectral_apply(problem, w.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return _pat.spectral_apply(ctx.problem, gy.contiguous(), transpose=True), None


def spectral_op(problem, w):
    """Differentiable P w; w may be [n^3] or [R][n^3] (float64)."""
    if w.dim() == 1:
        return PatSpectral.apply(w[None], problem)[0]
    return PatSpectral.apply(w, problem)


def forward_op(problem, p0):
    """Differentiable G p0; p0 may be [N] or [R][N]."""
    if p0.dim() == 1:
        return PatForward.apply(p0[None], problem)[0]
    return PatForward.apply(p0, problem)


def prior_op(problem, x, prior_a):
    """Differentiable L x; x may be [N] or [R][N] (float64)."""
    if x.dim() == 1:
        return PatPrior.apply(x[None], problem, prior_a)[0]
    return PatPrior.apply(x, problem, prior_a)


def map_objective(problem, p, y_obs, sigma, prior_a):
    """1/(2 sigma^2) ||G p - y||^2 + 1/2 ||L p||^2 for p [N] (float64)."""
    r = forward_op(problem, p) - y_obs
    return 0.5 * torch.sum(r * r) / (sigma * sigma) + 0.5 * torch.sum(prior_op(problem, p, prior_a) ** 2)


def hessian_lambda_max(problem, sigma, prior_a, iters=30, seed=0):
    """Largest eigenvalue of H = G^T G / sigma^2 + L^T L by power iteration."""
    dev = torch.device("cuda")
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn(problem.n_nodes, generator=g, dtype=torch.float64).to(dev)
    lam = 0.0
    for _ in range(iters):
        x = x / torch.linalg.norm(x)
        Hx = (_pat.pat_adjoint(problem, _pat.pat_forward(problem, x[None].contiguous()))[0] / (sigma * sigma)
              + _pat.pat_prior_apply(problem, _pat.pat_prior_apply(problem, x[None].contiguous(), prior_a),
                                     prior_a, transpose=True)[0])
        lam = float(torch.dot(x, Hx))
        x = Hx
    return lam


def map_gradient_descent(problem, y_obs, sigma, prior_a, n_iter=200, step=None, p_init=None, history=False):
    """Gradient descent on the MAP objective; returns p (and the objective history)."""
    if step is None:
        step = 1.0 / (1.02 * hessian_lambda_max(problem, sigma, prior_a))
    p = (torch.zeros(problem.n_nodes, dtype=torch.float64, device=y_obs.device) if p_init is None
         else p_init.detach().clone())
    hist = []
    for _ in range(n_iter):
        p.requires_grad_(True)
        f = map_objective(problem, p, y_obs, sigma, prior_a)
        (grad,) = torch.autograd.grad(f, p)
        hist.append(float(f.detach()))
        with torch.no_grad():
            p = p - step * grad
    p = p.detach()
    return (p, hist, step) if history else p
