"""Synthetic inputs: tree, admissibility lists and H^2 construction.

The tree and lists are pinned by brute force (every same-level pair evaluated,
every point pair covered exactly once); the construction is pinned against the
dense kernel matrix evaluated directly from the points.
"""
import numpy as np
import pytest

from conftest import NOFAR_256, oracle_matrix, workload
from h2gen import rng, tree


def test_rng_moments_and_determinism():
    u = rng.uniform01(7, 200000)
    assert np.all((u >= 0) & (u < 1))
    assert abs(u.mean() - 0.5) < 3e-3
    z = rng.normal(8, 200000)
    assert abs(z.mean()) < 1e-2 and abs(z.std() - 1) < 1e-2
    assert np.array_equal(rng.uniform01(7, 10), rng.uniform01(7, 10))
    assert not np.array_equal(rng.uniform01(7, 10), rng.uniform01(8, 10))


def test_grid_points_are_the_cell_centres():
    p = rng.grid_points(1024, 2)
    assert p.shape == (1024, 2)
    # every cell of the 32 x 32 grid holds exactly one point, at its centre
    cells = np.floor(p * 32).astype(np.int64)
    assert len({(int(a), int(b)) for a, b in cells}) == 1024
    assert np.allclose(p, (cells + 0.5) / 32, rtol=0, atol=1e-15)
    assert np.array_equal(rng.grid_points(27, 3)[:4], [[1 / 6, 1 / 6, 1 / 6], [0.5, 1 / 6, 1 / 6],
                                                      [5 / 6, 1 / 6, 1 / 6], [1 / 6, 0.5, 1 / 6]])
    with pytest.raises(ValueError):
        rng.grid_points(1000, 2)


@pytest.mark.parametrize("h", [1 / 32, 1 / 512])
def test_laplace2d_self_term_is_the_cell_mean(h):
    """The diagonal of the 2D Laplace kernel matrix is the kernel's mean over
    the point's cell of side h; checked against a midpoint rule on a fine
    sub-grid of the cell, whose error is O(1/s) from the log singularity."""
    import math

    import torch
    from h2gen import kernels

    K = kernels.Kernel("laplace2d", h, 0.0)
    d = float(K.radial(torch.zeros(1, dtype=torch.float64))[0])
    s = 2000
    u = ((np.arange(s) + 0.5) / s - 0.5) * h
    X, Y = np.meshgrid(u, u)
    mean = np.mean(-np.log(np.sqrt(X * X + Y * Y)) / (2 * math.pi))
    assert abs(d - mean) <= 1e-4 * abs(mean)
    # off the diagonal: the free-space Green's function
    r = torch.tensor([0.25, 1.0], dtype=torch.float64)
    assert torch.allclose(K.radial(r), -torch.log(r) / (2 * math.pi), rtol=1e-15, atol=0)


@pytest.mark.parametrize("kind,dim,n,m", [("2d", 2, 1024, 64), ("kd", 3, 3000, 32), ("2d", 3, 4096, 64)])
def test_tree_balanced_and_partitioned(kind, dim, n, m):
    p = rng.points(5, n, dim)
    t = tree.build_tree(p, m, kind)
    assert sorted(t.perm.tolist()) == list(range(n))
    lp = t.level_ptr
    for lev in range(t.L + 1):
        a, b = lp[lev], lp[lev + 1]
        # ranges of one level tile 0..n in order
        assert t.idx_begin[a] == 0 and t.idx_end[b - 1] == n
        assert np.all(t.idx_begin[a + 1:b] == t.idx_end[a:b - 1])
    leaves = t.idx_end[lp[t.L]:] - t.idx_begin[lp[t.L]:]
    assert leaves.max() <= m and leaves.min() >= 1
    for q in range(1, t.n_nodes):
        par = t.parent[q]
        assert t.child_ptr[par] <= q < t.child_ptr[par + 1]
        assert t.idx_begin[par] <= t.idx_begin[q] and t.idx_end[q] <= t.idx_end[par]
    # tight boxes contain exactly their points
    P = p[t.perm]
    for q in range(t.n_nodes):
        pts = P[t.idx_begin[q]:t.idx_end[q]]
        assert np.allclose(pts.min(0), t.lo[q]) and np.allclose(pts.max(0), t.hi[q])


def _adm_bruteforce(lo_s, hi_s, lo_t, hi_t, eta):
    ds = np.linalg.norm(hi_s - lo_s)
    dt = np.linalg.norm(hi_t - lo_t)
    gap = [max(0.0, lo_t[a] - hi_s[a], lo_s[a] - hi_t[a]) for a in range(len(lo_s))]
    dist = np.linalg.norm(gap)
    return dist > 0 and dist >= eta * max(ds, dt)


@pytest.mark.parametrize("kind,dim,n", [("2d", 2, 1024), ("kd", 3, 2048)])
def test_lists_bruteforce(kind, dim, n):
    p = rng.points(9, n, dim)
    t = tree.build_tree(p, 64, kind)
    near_ptr, near_col, far_ptr, far_col = tree.dual_traversal(t, 0.7, 0)
    nearset = {(q, int(j)) for q in range(t.n_nodes) for j in near_col[near_ptr[q]:near_ptr[q + 1]]}
    farset = {(q, int(j)) for q in range(t.n_nodes) for j in far_col[far_ptr[q]:far_ptr[q + 1]]}
    lp = t.level_ptr
    assert nearset >= {(0, 0)}
    for lev in range(1, t.L + 1):
        for s in range(lp[lev], lp[lev + 1]):
            for u in range(lp[lev], lp[lev + 1]):
                parents_near = (t.parent[s], t.parent[u]) in nearset
                adm = s != u and _adm_bruteforce(t.lo[s], t.hi[s], t.lo[u], t.hi[u], 0.7)
                assert ((s, u) in nearset) == (parents_near and not adm)
                assert ((s, u) in farset) == (parents_near and adm)


@pytest.mark.parametrize("name", ["exp2d_1024"])
def test_blocks_cover_every_entry_once(name):
    H = oracle_matrix(name)
    N = H.N
    cover = np.zeros((N, N), dtype=np.int32)
    for (q, j) in H.D:
        cover[H.idx_begin[q]:H.idx_end[q], H.idx_begin[j]:H.idx_end[j]] += 1
    for (q, j) in H.S:
        cover[H.idx_begin[q]:H.idx_end[q], H.idx_begin[j]:H.idx_end[j]] += 1
    assert cover.min() == 1 and cover.max() == 1


def test_no_far_case_has_no_top_level():
    H = oracle_matrix("nofar_256", NOFAR_256)
    assert H.top is None and len(H.S) == 0


@pytest.mark.parametrize("name", ["exp2d_1024", "laplace2d_1024"])
def test_construction_error_and_orthonormal_bases(name):
    w = workload(name)
    H = oracle_matrix(name)
    A = w["kernel"].dense(w["points"])
    from oracle import h2ops

    AH = h2ops.dense(H)
    eps_c = w["spec"]["tol"] / 10
    assert np.linalg.norm(AH - A, 2) <= 10 * eps_c * np.linalg.norm(A, 2)
    for q, U in H.U.items():
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
    lp = H.level_ptr
    for lev in range(H.L):
        for q in range(lp[lev], lp[lev + 1]):
            if H.rank[q] == 0:
                continue
            Es = np.vstack([H.E[c] for c in range(H.child_ptr[q], H.child_ptr[q + 1])])
            assert np.allclose(Es.T @ Es, np.eye(H.rank[q]), atol=1e-12)
    # symmetric input: D_ji = D_ij^T and S_ji = S_ij^T
    for (q, j), Dq in H.D.items():
        assert np.allclose(Dq, H.D[(j, q)].T, atol=0, rtol=0)
    for (q, j), Sq in H.S.items():
        assert np.allclose(Sq, H.S[(j, q)].T, atol=1e-14 * np.abs(Sq).max() + 1e-300)
    assert abs(H.norm2 - np.linalg.norm(AH, 2)) <= 1e-6 * H.norm2
