import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    # the oracle's many small LAPACK calls run fastest single-threaded
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1, user_api="blas")
    except Exception:
        pass


_CACHE = {}


def workload(name, spec=None):
    """Constructed workload (points, blob, rhs), cached per session."""
    from h2gen import workloads

    key = name
    if key not in _CACHE:
        _CACHE[key] = workloads.make(spec if spec is not None else name)
    return _CACHE[key]


def oracle_matrix(name, spec=None):
    from oracle import blob as ob

    key = ("H", name)
    if key not in _CACHE:
        _CACHE[key] = ob.parse(workload(name, spec)["blob"])
    return _CACHE[key]


def oracle_factor(name, tol=None, spec=None):
    from oracle import factor as of

    w = workload(name, spec)
    tol = w["spec"]["tol"] if tol is None else tol
    key = ("F", name, tol)
    if key not in _CACHE:
        _CACHE[key] = of.factor(oracle_matrix(name, spec), tol)
    return _CACHE[key]


# small 3D case shared by oracle pins and GPU parity (64 leaves, two skeletonized levels)
EXP3D_4096 = dict(N=4096, dim=3, seed=116, kernel=("exp", 0.1, 1e-2), tree="kd", leaf=64,
                  eta=0.7, tol=1e-6, nrhs=3, rhs_seed=216, p0=5)
# one leaf-level block row per cluster with no admissible pair: pure dense LU
NOFAR_256 = dict(N=256, dim=2, seed=121, kernel=("exp", 0.1, 1e-2), tree="2d", leaf=64,
                 eta=0.7, tol=1e-8, nrhs=2, rhs_seed=221, p0=10)

# the batched recipe (2D Gaussian kernel, KD tree, tol 1e-8) at the other leaf sizes the
# batched configuration's leaf choice may pick
GAUSS_L32 = dict(N=3000, dim=2, seed=3001, kernel=("gauss", 0.05, 1e-3), tree="kd", leaf=32,
                 eta=0.7, tol=1e-8, nrhs=4, rhs_seed=4001, p0=10)
GAUSS_L128 = dict(N=4096, dim=2, seed=3002, kernel=("gauss", 0.05, 1e-3), tree="kd", leaf=128,
                  eta=0.7, tol=1e-8, nrhs=4, rhs_seed=4002, p0=10)


def data_sections(blob):
    """Element counts of the U, E, D and S sections of a blob's data (in that
    order at the end of the blob), from the oracle's parse of its structure."""
    from oracle import blob as ob

    H = ob.parse(blob)
    size = H.idx_end - H.idx_begin
    leaf0 = H.level_ptr[H.L]
    nU = sum(int(size[q] * H.rank[q]) for q in range(leaf0, H.n_nodes))
    nE = sum(int(H.rank[c] * H.rank[H.parent[c]]) for c in range(1, H.n_nodes))
    nD = sum(int(size[q] * size[H.near_col[e]]) for q in range(leaf0, H.n_nodes)
             for e in range(H.near_ptr[q], H.near_ptr[q + 1]))
    nS = sum(int(H.rank[q] * H.rank[H.far_col[e]]) for q in range(H.n_nodes)
             for e in range(H.far_ptr[q], H.far_ptr[q + 1]))
    return nU, nE, nD, nS


def scaled_blob(blob, s, scale_norm=True):
    """The same H^2 matrix times s: near blocks D and couplings S scaled (the
    orthonormal bases unchanged), and the header's ||A||_2 (at byte 32) scaled
    too unless scale_norm is False."""
    import numpy as np

    b = np.array(blob, dtype=np.uint8)
    nU, nE, nD, nS = data_sections(b)
    start = b.nbytes - 8 * (nD + nS)
    d = b[start:].view(np.float64) * s
    b[start:] = d.view(np.uint8)
    if scale_norm:
        norm = b[32:40].view(np.float64)[0] * s
        b[32:40] = np.array([norm]).view(np.uint8)
    return b
