"""Cluster tree, bounding boxes, admissibility and the dual-tree traversal.

Section 1.1 of the paper: indices are clustered hierarchically into a tree; a
dual traversal of same-level cluster pairs tests an admissibility predicate on
bounding boxes; admissible pairs become low-rank (far) blocks and inadmissible
pairs recurse into their child pairs until the leaves, where they are stored
densely (near blocks).

Trees are balanced (every leaf at depth L, leaf size <= m).  A node is split by
median bisections along coordinate axes: the index set is sorted by
(coordinate, original index) and the first floor(n/2) go left.
  * "kd": one bisection per level along the longest axis of the node's tight
    bounding box (ties go to the lowest axis) -- the paper's KD tree.
  * "2d": d bisections per level in axis order x, y, (z) giving a quadtree or
    octree; when the total number of bisections is not a multiple of d the
    root level takes the remainder.
"""
import numpy as np


class Tree:
    pass


def _num_bisections(n, leaf_size):
    b = 0
    while n > leaf_size * (1 << b):
        b += 1
    return b


def split_schedule(n, dim, leaf_size, kind):
    b = _num_bisections(n, leaf_size)
    if kind == "kd":
        return [1] * b
    if kind == "2d":
        if b == 0:
            return []
        levels = (b + dim - 1) // dim
        first = b - dim * (levels - 1)
        return [first] + [dim] * (levels - 1)
    raise ValueError(kind)


def build_tree(pts, leaf_size, kind="kd"):
    """Balanced median tree over the rows of pts (N x d)."""
    pts = np.asarray(pts, dtype=np.float64)
    n, dim = pts.shape
    sched = split_schedule(n, dim, leaf_size, kind)
    L = len(sched)
    perm = np.arange(n, dtype=np.int64)
    # segments of the current level: node k owns perm[seg[k]:seg[k+1]]
    seg = np.array([0, n], dtype=np.int64)
    level_segs = [seg]
    parent = [np.array([-1], dtype=np.int32)]
    for lev, nb in enumerate(sched):
        cur = seg
        # each bisection doubles the segments
        for bi in range(nb):
            cnt = np.diff(cur)
            nodes = np.repeat(np.arange(len(cur) - 1), cnt)
            if kind == "kd":
                lo = np.full((len(cur) - 1, dim), np.inf)
                hi = np.full((len(cur) - 1, dim), -np.inf)
                P = pts[perm]
                np.minimum.at(lo, nodes, P)
                np.maximum.at(hi, nodes, P)
                axis = np.argmax(hi - lo, axis=1)  # first max = lowest axis on ties
                coord = P[np.arange(n), axis[nodes]]
            else:
                coord = pts[perm, bi]
            order = np.lexsort((perm, coord, nodes))
            perm = perm[order]
            half = cnt // 2
            mids = cur[:-1] + half
            new = np.empty(2 * (len(cur) - 1) + 1, dtype=np.int64)
            new[0:-1:2] = cur[:-1]
            new[1::2] = mids
            new[-1] = n
            cur = new
        arity = 1 << nb
        nparent = len(seg) - 1
        parent.append(np.repeat(np.arange(nparent, dtype=np.int32), arity))
        seg = cur
        level_segs.append(seg)
    t = Tree()
    t.N = n
    t.dim = dim
    t.L = L
    t.kind = kind
    t.leaf_size = leaf_size
    t.perm = perm
    counts = [len(s) - 1 for s in level_segs]
    t.level_ptr = np.zeros(L + 2, dtype=np.int32)
    t.level_ptr[1:] = np.cumsum(counts)
    n_nodes = int(t.level_ptr[-1])
    t.n_nodes = n_nodes
    t.parent = np.full(n_nodes, -1, dtype=np.int32)
    t.idx_begin = np.zeros(n_nodes, dtype=np.int64)
    t.idx_end = np.zeros(n_nodes, dtype=np.int64)
    for lev in range(L + 1):
        a = t.level_ptr[lev]
        s = level_segs[lev]
        t.idx_begin[a:a + len(s) - 1] = s[:-1]
        t.idx_end[a:a + len(s) - 1] = s[1:]
        if lev > 0:
            t.parent[a:a + len(s) - 1] = parent[lev] + t.level_ptr[lev - 1]
    # BFS order: the children of node k are nodes child_ptr[k] .. child_ptr[k+1]-1
    nch = np.bincount(t.parent[1:], minlength=n_nodes)
    t.child_ptr = np.concatenate([[1], 1 + np.cumsum(nch)]).astype(np.int32)
    # tight boxes
    P = pts[perm]
    t.lo = np.zeros((n_nodes, dim))
    t.hi = np.zeros((n_nodes, dim))
    for lev in range(L + 1):
        a, b = t.level_ptr[lev], t.level_ptr[lev + 1]
        s = level_segs[lev]
        ids = np.repeat(np.arange(b - a), np.diff(s))
        lo = np.full((b - a, dim), np.inf)
        hi = np.full((b - a, dim), -np.inf)
        np.minimum.at(lo, ids, P)
        np.maximum.at(hi, ids, P)
        t.lo[a:b] = lo
        t.hi[a:b] = hi
    t.sched = sched
    return t


def admissible(lo_s, hi_s, lo_t, hi_t, same, eta, kind):
    """Vectorised admissibility on tight boxes.

    D(s) is the box diagonal, Dist(s,t) the Euclidean norm of the per-axis gaps.
    kind 0 ("max-diameter" form of the workloads): Dist >= eta * max(D(s), D(t)).
    kind 1 (Eq. 1.1 of the paper): (D(s) + D(t)) / 2 <= eta * Dist.
    A pair is never admissible with itself or with zero distance.
    """
    ds = np.sqrt(((hi_s - lo_s) ** 2).sum(-1))
    dt = np.sqrt(((hi_t - lo_t) ** 2).sum(-1))
    gap = np.maximum(0.0, np.maximum(lo_t - hi_s, lo_s - hi_t))
    dist = np.sqrt((gap * gap).sum(-1))
    if kind == 0:
        ok = dist >= eta * np.maximum(ds, dt)
    else:
        ok = 0.5 * (ds + dt) <= eta * dist
    return ok & (dist > 0) & (~same)


def dual_traversal(t, eta=0.7, adm_kind=0):
    """Near/far lists per level as CSR over all nodes (global ids, sorted).

    near^0 = {(root, root)}; near^l and far^l are the inadmissible / admissible
    child pairs of near^{l-1}.  Returns (near_ptr, near_col, far_ptr, far_col).
    """
    near_rows = [np.array([0])]
    near_cols = [np.array([0])]
    far_rows = [np.zeros(0, dtype=np.int64)]
    far_cols = [np.zeros(0, dtype=np.int64)]
    cp = t.child_ptr
    for lev in range(1, t.L + 1):
        a, b = near_rows[-1], near_cols[-1]
        na = (cp[a + 1] - cp[a]).astype(np.int64)
        nb = (cp[b + 1] - cp[b]).astype(np.int64)
        tot = na * nb
        pid = np.repeat(np.arange(len(a)), tot)
        loc = np.arange(tot.sum()) - np.repeat(np.cumsum(tot) - tot, tot)
        ci = cp[a][pid] + loc // nb[pid]
        cj = cp[b][pid] + loc % nb[pid]
        ok = admissible(t.lo[ci], t.hi[ci], t.lo[cj], t.hi[cj], ci == cj, eta, adm_kind)
        o = np.lexsort((cj[~ok], ci[~ok]))
        near_rows.append(ci[~ok][o])
        near_cols.append(cj[~ok][o])
        o = np.lexsort((cj[ok], ci[ok]))
        far_rows.append(ci[ok][o])
        far_cols.append(cj[ok][o])
    nr = np.concatenate(near_rows)
    nc = np.concatenate(near_cols)
    fr = np.concatenate(far_rows)
    fc = np.concatenate(far_cols)
    near_ptr = np.zeros(t.n_nodes + 1, dtype=np.int64)
    near_ptr[1:] = np.cumsum(np.bincount(nr, minlength=t.n_nodes))
    far_ptr = np.zeros(t.n_nodes + 1, dtype=np.int64)
    far_ptr[1:] = np.cumsum(np.bincount(fr, minlength=t.n_nodes)) if len(fr) else 0
    return near_ptr, nc.astype(np.int32), far_ptr, fc.astype(np.int32)


def top_level(t, far_ptr):
    """Smallest level that holds a far pair, or None when there is none."""
    for lev in range(t.L + 1):
        a, b = t.level_ptr[lev], t.level_ptr[lev + 1]
        if far_ptr[b] > far_ptr[a]:
            return lev
    return None


def chebyshev_order(p0, L, lev):
    """Interpolation order raised with every other level above the leaves."""
    return p0 + (L - lev) // 2


def sparsity_constant(t, near_ptr):
    """Maximum number of near blocks in any block row, over all levels."""
    return int(np.max(np.diff(near_ptr))) if t.n_nodes else 0

