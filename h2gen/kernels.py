"""Kernel functions K(r) of the synthetic workloads and the dense entry rule.

A_ij = K(|x_i - x_j|) + alpha * delta_ij, where delta_ij compares indices (so the
nugget is added exactly once per diagonal entry).  K is evaluated at r = 0 by
its formula (the 2D Laplace kernel by its cell self-interaction).  The
exponential covariance and the 2D Laplace volume integral equation are the
paper's first two applications (Section 3.1); the Matern-3/2, Gaussian and
regularised 3D Laplace kernels are the other synthetic kernel matrices of the
measured workloads.
"""
import math

import numpy as np
import torch


def _exp(r, ell):
    return torch.exp(-r / ell)


def _matern32(r, ell):
    s = math.sqrt(3.0) * r / ell
    return (1.0 + s) * torch.exp(-s)


def _gauss(r, ell):
    return torch.exp(-(r * r) / (ell * ell))


def _laplace3d_reg(r, delta):
    return 1.0 / (4.0 * math.pi * (r + delta))


# mean of log|u| over the unit square centred at the origin:
# 1/2 log 2 - 3/2 + pi/4 over [0,1]^2, minus log 2 for the halved side
_LOG_MEAN_SQUARE = -0.5 * math.log(2.0) - 1.5 + 0.25 * math.pi


def _laplace2d(r, h):
    """Free-space Green's function of the 2D Laplace equation, -log(r)/(2 pi), for
    r > 0 (Section 3.1, second application).  At r = 0 (a point with itself) the
    entry is the kernel's mean over the point's grid cell of side h, the
    self-interaction of a piecewise-constant volume discretization:
    -(log h + mean of log|u| over the unit square)/(2 pi)."""
    self_term = -(math.log(h) + _LOG_MEAN_SQUARE) / (2.0 * math.pi)
    safe = torch.where(r > 0, r, torch.ones_like(r))
    return torch.where(r > 0, -torch.log(safe) / (2.0 * math.pi), torch.full_like(r, self_term))


KERNELS = {
    "exp": _exp,
    "matern32": _matern32,
    "gauss": _gauss,
    "laplace3d_reg": _laplace3d_reg,
    "laplace2d": _laplace2d,
}


class Kernel:
    """K(r) with one length parameter plus the diagonal nugget alpha."""

    def __init__(self, name, param, alpha):
        if name not in KERNELS:
            raise ValueError(f"unknown kernel {name}")
        self.name = name
        self.param = float(param)
        self.alpha = float(alpha)

    def radial(self, r):
        return KERNELS[self.name](r, self.param)

    def block(self, X, Y):
        """K(|x - y|) for point sets X (..., a, d) and Y (..., b, d), no nugget."""
        diff = X.unsqueeze(-2) - Y.unsqueeze(-3)
        r = torch.sqrt((diff * diff).sum(-1))
        return self.radial(r)

    def dense(self, pts):
        """The full N x N matrix of the kernel plus nugget in the given point order."""
        P = torch.as_tensor(np.asarray(pts), dtype=torch.float64)
        A = self.block(P, P)
        A += self.alpha * torch.eye(P.shape[0], dtype=torch.float64)
        return A.numpy()

    def spec(self):
        return {"name": self.name, "param": self.param, "alpha": self.alpha}
