"""Oracle H^2 products: matrix-vector product and the dense expansion.

TEST INFRASTRUCTURE ONLY (slow CPU reference; the product never imports it).

The H^2 matrix of Section 1.1: admissible blocks A_st = U_s S_st U_t^T with
nested bases U_tau = diag(U_children) [E_children], inadmissible leaf blocks
stored densely.  The product follows that definition literally: an upsweep
forms U^T x for every cluster, couplings act on far pairs, a downsweep
expands back through the transfers, and the near blocks act directly.
"""
import numpy as np

from .blob import children, far, near


def matvec(H, X):
    """Y = A_H X with X, Y in original point order (N x nrhs)."""
    X = np.asarray(X, dtype=np.float64)
    one = X.ndim == 1
    if one:
        X = X[:, None]
    x = X[H.perm]  # tree order
    nrhs = x.shape[1]
    L = H.L
    lp = H.level_ptr
    seg = lambda q: slice(H.idx_begin[q], H.idx_end[q])
    xh = {}
    for q in range(lp[L], lp[L + 1]):
        xh[q] = H.U[q].T @ x[seg(q)]
    for lev in range(L - 1, -1, -1):
        for q in range(lp[lev], lp[lev + 1]):
            acc = np.zeros((H.rank[q], nrhs))
            for c in children(H, q):
                acc += H.E[c].T @ xh[c]
            xh[q] = acc
    yh = {}
    for q in range(H.n_nodes):
        acc = np.zeros((H.rank[q], nrhs))
        for j in far(H, q):
            acc += H.S[(q, j)] @ xh[j]
        yh[q] = acc
    for lev in range(1, L + 1):
        for q in range(lp[lev], lp[lev + 1]):
            yh[q] = yh[q] + H.E[q] @ yh[H.parent[q]]
    y = np.zeros_like(x)
    for q in range(lp[L], lp[L + 1]):
        y[seg(q)] += H.U[q] @ yh[q]
        for j in near(H, q):
            y[seg(q)] += H.D[(q, j)] @ x[seg(j)]
    Y = np.empty_like(y)
    Y[H.perm] = y
    return Y[:, 0] if one else Y


def explicit_bases(H):
    """U_tau for every cluster as an explicit |tau| x k_tau matrix (nested expansion)."""
    L = H.L
    lp = H.level_ptr
    Ub = {q: H.U[q] for q in range(lp[L], lp[L + 1])}
    for lev in range(L - 1, -1, -1):
        for q in range(lp[lev], lp[lev + 1]):
            parts = [Ub[c] @ H.E[c] for c in children(H, q)]
            Ub[q] = np.vstack(parts) if parts else np.zeros((0, H.rank[q]))
    return Ub


def dense(H):
    """A_H as a dense N x N array in original point order."""
    N = H.N
    A = np.zeros((N, N))
    Ub = explicit_bases(H)
    seg = lambda q: slice(H.idx_begin[q], H.idx_end[q])
    for (q, j), S in H.S.items():
        A[seg(q), seg(j)] = Ub[q] @ S @ Ub[j].T
    for (q, j), D in H.D.items():
        A[seg(q), seg(j)] = D
    out = np.empty_like(A)
    out[np.ix_(H.perm, H.perm)] = A
    return out


def backward_error(H, X, B):
    """Per-column e_b = ||B_j - A_H X_j|| / ||B_j|| (Section 3.3)."""
    X = np.asarray(X).reshape(H.N, -1)
    B = np.asarray(B).reshape(H.N, -1)
    R = B - matvec(H, X)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
