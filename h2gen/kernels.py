"""Kernel functions K(r) of the synthetic workloads and the dense entry rule.

A_ij = K(|x_i - x_j|) + alpha * delta_ij, where delta_ij compares indices (so the
nugget is added exactly once per diagonal entry).  K is evaluated at r = 0 by
its formula.  The exponential covariance is the paper's first application
(Section 3.1); the Matern-3/2, Gaussian and regularised Laplace kernels are the
other synthetic kernel matrices of the measured workloads.
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


KERNELS = {
    "exp": _exp,
    "matern32": _matern32,
    "gauss": _gauss,
    "laplace3d_reg": _laplace3d_reg,
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
