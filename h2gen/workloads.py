"""The synthetic workloads (points, kernel, tree, tolerances, right-hand sides).

Every input is seeded (SplitMix64, see rng.py).  The five measured
configurations mirror the kernel-matrix families of the paper's Section 3
(exponential covariance in 2D/3D) plus the other kernels used for the
precision and scale studies; the smaller variants keep the same recipe at
sizes the CPU oracle finishes in seconds.

Fields: N, dim, point seed (or points="grid": the uniform grid's cell centres),
kernel (name, length or None for the grid's cell side, nugget), tree kind
("2d" = quadtree/octree, "kd" = binary KD), leaf size m, admissibility eta
(max-diameter form), factorization tolerance tol (construction uses tol/10),
number of right-hand sides and their seed, Chebyshev leaf order p0.
"""
import numpy as np

from . import blob as blobmod
from . import construct as cons
from . import kernels, rng

WORKLOADS = {
    # N=4096 2D exponential covariance, quadtree, tol 1e-8, 1 RHS
    "exp2d_4096": dict(N=4096, dim=2, seed=101, kernel=("exp", 0.1, 1e-2), tree="2d",
                       leaf=64, eta=0.7, tol=1e-8, nrhs=1, rhs_seed=201, p0=10),
    # N=65536 3D Matern-3/2, octree, tol 1e-10, 4 RHS
    "matern3d_65536": dict(N=65536, dim=3, seed=102, kernel=("matern32", 0.2, 1e-4), tree="2d",
                           leaf=64, eta=0.7, tol=1e-10, nrhs=4, rhs_seed=202, p0=6),
    # N=2^18 3D exponential covariance, KD tree, tol 1e-6, 8 RHS
    "exp3d_262144": dict(N=262144, dim=3, seed=104, kernel=("exp", 0.1, 1e-2), tree="kd",
                         leaf=64, eta=0.7, tol=1e-6, nrhs=8, rhs_seed=204, p0=5),
    # N=2^20 3D regularised Laplace, KD tree, tol 1e-6, 32 RHS
    "laplace3d_1048576": dict(N=1048576, dim=3, seed=105, kernel=("laplace3d_reg", 1e-3, 1.0),
                              tree="kd", leaf=64, eta=0.7, tol=1e-6, nrhs=32, rhs_seed=205, p0=5),
    # reduced sizes with the same recipes (parity tests)
    "exp2d_1024": dict(N=1024, dim=2, seed=111, kernel=("exp", 0.1, 1e-2), tree="2d",
                       leaf=64, eta=0.7, tol=1e-8, nrhs=2, rhs_seed=211, p0=10),
    "matern3d_8192": dict(N=8192, dim=3, seed=112, kernel=("matern32", 0.2, 1e-4), tree="2d",
                          leaf=64, eta=0.7, tol=1e-10, nrhs=4, rhs_seed=212, p0=6),
    "exp3d_16384": dict(N=16384, dim=3, seed=114, kernel=("exp", 0.1, 1e-2), tree="kd",
                        leaf=64, eta=0.7, tol=1e-6, nrhs=8, rhs_seed=214, p0=5),
    "laplace3d_8192": dict(N=8192, dim=3, seed=115, kernel=("laplace3d_reg", 1e-3, 1.0),
                           tree="kd", leaf=64, eta=0.7, tol=1e-6, nrhs=4, rhs_seed=215, p0=5),
    "gauss2d_3000": dict(N=3000, dim=2, seed=3000, kernel=("gauss", 0.05, 1e-3), tree="kd",
                         leaf=64, eta=0.7, tol=1e-8, nrhs=16, rhs_seed=4000, p0=10),
    # 2D Laplace volume integral equation (Section 3.1, Table 2: m 64, p0 8, alpha_r 1e-5,
    # eps 1e-7, eps_lu 1e-6) on the uniform grid of cell centres; the kernel's
    # parameter (None) is the grid's cell side
    "laplace2d_1024": dict(N=1024, dim=2, seed=0, points="grid", kernel=("laplace2d", None, 1e-5),
                           tree="2d", leaf=64, eta=0.7, tol=1e-6, nrhs=2, rhs_seed=221, p0=8),
    "laplace2d_4096": dict(N=4096, dim=2, seed=0, points="grid", kernel=("laplace2d", None, 1e-5),
                           tree="2d", leaf=64, eta=0.7, tol=1e-6, nrhs=4, rhs_seed=222, p0=8),
    "laplace2d_262144": dict(N=262144, dim=2, seed=0, points="grid",
                             kernel=("laplace2d", None, 1e-5), tree="2d", leaf=64, eta=0.7,
                             tol=1e-6, nrhs=8, rhs_seed=223, p0=8),
}


def batch_sizes(count=64, seed=303, lo=2048, hi=32768):
    """Instance sizes N_i = floor(lo * (hi/lo)^u_i), u_i uniform (log-uniform in [lo, hi])."""
    u = rng.uniform01(seed, count)
    return np.floor(lo * (hi / lo) ** u).astype(np.int64)


def batch_workload(i, n, leaf=64):
    """Instance i of the batched workload: 2D Gaussian kernel, KD tree, tol 1e-8, 16 RHS."""
    return dict(N=int(n), dim=2, seed=3000 + i, kernel=("gauss", 0.05, 1e-3), tree="kd",
                leaf=leaf, eta=0.7, tol=1e-8, nrhs=16, rhs_seed=4000 + i, p0=10)


def make(spec, device="cpu", want_blob=True, verbose=False):
    """Points, constructor output, serialized blob and right-hand sides of a workload."""
    if isinstance(spec, str):
        spec = WORKLOADS[spec]
    if spec.get("points") == "grid":
        pts = rng.grid_points(spec["N"], spec["dim"])
    else:
        pts = rng.points(spec["seed"], spec["N"], spec["dim"])
    kname, kpar, alpha = spec["kernel"]
    if kpar is None:  # the grid's cell side
        kpar = 1.0 / round(spec["N"] ** (1.0 / spec["dim"]))
    K = kernels.Kernel(kname, kpar, alpha)
    h = cons.construct(pts, K, spec["leaf"], spec["tree"], spec["eta"], 0, spec["tol"] / 10,
                       p0=spec["p0"], device=device, verbose=verbose)
    B = rng.rhs(spec["rhs_seed"], spec["N"], spec["nrhs"])
    buf = blobmod.write_blob(h) if want_blob else None
    return dict(spec=spec, points=pts, kernel=K, h=h, blob=buf, B=B)
