"""Oracle strong recursive skeletonization factorization and solve (FP64, CPU).

TEST INFRASTRUCTURE ONLY: this is the slow, plain reference that the GPU
library is checked against.  Only the tests, the smoke check and the CPU
baseline of the benchmark import it; the product path never does.

It follows Section 2 of the paper step by step, in its notation:
  * Algorithm 1 (factorize): levels from the leaves (d = L) up to the top level
    t (first level with admissible blocks); at each level colour the near
    graph and skeletonize colour by colour; then dense LU of the remnant.
  * Algorithm 2 (skeletonizeColor), in its order for the clusters i of a
    colour: first, for every i, the truncated SVD of (I - V_i V_i^T) F_{i*}
    at eps_fill = eps_lu * ||A|| (Section 2.1: keep the left singular vectors
    that are needed) giving the augmented basis V~_i = [V_i, Vbar_i], its
    complement V~_i^perp and Q~_i = [V~_i^perp, V~_i] (redundant rows R first,
    skeleton rows S last); then, with all of them,
      - projection Q~^T D Q~ of the near blocks and V~^T F of the fill blocks
        (the V~^perp part of F is dropped: that is the truncation);
      - partial LU: LU of D_RR, elementary factors
        L-blocks X_j = D_{j,R} D_RR^{-1}, U-blocks Y_k = D_RR^{-1} D_{R,k},
        Schur updates -D_{j,R} D_RR^{-1} D_{R,k} on every pair of neighbours,
        which go to D for near pairs and to the fill matrix F otherwise.
  * Level close-out (Section 2.1, the merge step): skeleton blocks of near
    pairs, and zero-padded couplings S~ plus fill of far pairs, form the
    blocks of the next level; fill outside the next level's near pairs is
    lifted to the parent pair; the parent basis is the stacked [E_c; 0].
  * Algorithm 3 (solve): apply the inverse transforms up the tree, dense top
    solve, and back down.

Readings of points the paper leaves open are listed in the design notes
(colouring rule, truncation rule, where fill goes, loop bounds).
"""
import numpy as np
import scipy.linalg as sla

from .blob import children, far, near

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def node_hash(ids):
    """SplitMix64 output finaliser (Steele et al., OOPSLA 2014) of node ids,
    used as the colouring priority."""
    z = np.asarray(ids, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def greedy_colors(nodes, nbrs):
    """Colour the near graph of one level (Section 2.2): clusters joined by a
    near block get different colours.  Sequential greedy: vertices in
    decreasing (hash(id), id), each takes the smallest colour not used by an
    already coloured neighbour."""
    h = node_hash(nodes)
    order = sorted(range(len(nodes)), key=lambda a: (int(h[a]), int(nodes[a])), reverse=True)
    color = {}
    for a in order:
        q = int(nodes[a])
        used = {color[j] for j in nbrs[q] if j != q and j in color}
        c = 0
        while c in used:
            c += 1
        color[q] = c
    return color


class LevelFactor:
    pass


class Factor:
    pass


def _cgs2(Vb, V):
    """Classical Gram-Schmidt twice against the orthonormal columns of V."""
    for _ in range(2):
        Vb = Vb - V @ (V.T @ Vb)
    return Vb


def factor(H, tol, keep_trace=False):
    """Algorithm 1 with eps_lu = tol and eps_fill = tol * ||A||_2 (blob header)."""
    eps_fill = tol * H.norm2
    L, lp = H.L, H.level_ptr
    t = H.top
    Fz = Factor()
    Fz.N, Fz.L, Fz.t, Fz.perm = H.N, L, t, H.perm
    Fz.idx_begin, Fz.idx_end = H.idx_begin, H.idx_end
    Fz.levels = []

    # state at the leaf level
    n = {q: int(H.size[q]) for q in range(lp[L], lp[L + 1])}
    V = {q: H.U[q] for q in range(lp[L], lp[L + 1])}
    D = {key: blk.copy() for key, blk in H.D.items()}
    F = {}
    if t is None:
        # no admissible block anywhere: the remnant is the whole leaf level
        return _top(Fz, H, L, n, D)

    for lev in range(L, t - 1, -1):
        nodes = list(range(lp[lev], lp[lev + 1]))
        nb = {q: near(H, q) for q in nodes}
        nearset = {(q, j) for q in nodes for j in nb[q]}
        color = greedy_colors(np.array(nodes), nb)
        # fill pattern: lifted pairs plus every non-near pair of neighbours of a
        # common cluster (where a Schur update can land)
        fpat = set(F.keys())
        for i in nodes:
            for j in nb[i]:
                for k in nb[i]:
                    if (j, k) not in nearset:
                        fpat.add((j, k))
        for key in fpat:
            if key not in F:
                F[key] = np.zeros((n[key[0]], n[key[1]]))
        frow = {q: [] for q in nodes}
        fcol = {q: [] for q in nodes}
        for (j, k) in sorted(F):
            frow[j].append(k)
            fcol[k].append(j)
        Lf = LevelFactor()
        Lf.level, Lf.nodes, Lf.color, Lf.near = lev, nodes, color, nb
        Lf.children = {tau: children(H, tau) for tau in range(lp[lev - 1], lp[lev])}
        Lf.n = dict(n)
        Lf.fpat = sorted(fpat)
        Lf.Q, Lf.lu, Lf.r, Lf.kt, Lf.X, Lf.Y = {}, {}, {}, {}, {}, {}
        ncolors = max(color.values()) + 1
        Lf.ncolors = ncolors
        Lf.owners = {}
        for c in range(ncolors):
            members = [q for q in nodes if color[q] == c]
            # Section 2.2: several clusters of one colour may update the same
            # block; the contributors of each target, in the order their
            # updates are applied (ascending cluster id)
            for i in members:
                for j in nb[i]:
                    for k in nb[i]:
                        Lf.owners.setdefault((c, j, k), []).append(i)
            # Algorithm 2: the parallel loop computes every basis of the colour
            # from the fill present before the colour's projections ...
            for i in members:
                _augment(i, n, V, F, frow[i], eps_fill, Lf)
            # ... then D = Q^T D Q and F = Q^T F Q with all of them ...
            for i in members:
                _project(i, D, F, nb[i], frow[i], fcol[i], Lf)
            # ... then the partial LU of the colour, F = F + F^a
            for i in members:
                _partial_lu(i, D, F, nb[i], nearset, Lf)
        Fz.levels.append(Lf)
        if keep_trace:
            Lf.D_end = {key: blk.copy() for key, blk in D.items()}
        # ---- close-out: build level lev-1 ----
        n, V, D, F = _close_out(H, lev, n, V, D, F, Lf)
    return _top(Fz, H, t - 1, n, D)


def _augment(i, n, V, F, frow_i, eps_fill, Lf):
    """Algorithm 2, parallel loop: truncated SVD of the projected fill row
    (I - V V^T) F_{i*}, augmented basis V~ = [V, Vbar], complement, Q~."""
    ni = n[i]
    Vi = V[i]
    ki = Vi.shape[1]
    if frow_i:
        Y = np.hstack([F[(i, j)] for j in frow_i])
        P = Y - Vi @ (Vi.T @ Y)
        # Section 2.1, second option: QR of the transposed fill row, then the
        # SVD of R; the left singular vectors of P are those of R^T
        Rq = np.linalg.qr(P.T, mode="r")
        Us, s, _ = np.linalg.svd(Rq.T, full_matrices=False)
        rbar = int(np.sum(s > eps_fill))
        rbar = min(rbar, ni - ki)
        Vbar = Us[:, :rbar]
    else:
        Vbar = np.zeros((ni, 0))
        rbar = 0
    if rbar:
        Vbar = _cgs2(Vbar, Vi)
        Vbar, _ = np.linalg.qr(Vbar)
    Vt = np.hstack([Vi, Vbar])  # augmented basis [V, Vbar]
    kt = ki + rbar
    r = ni - kt
    # complement: last columns of the full orthogonal factor of V~
    Qfull, _ = np.linalg.qr(Vt, mode="complete") if kt else (np.eye(ni), None)
    Lf.Q[i] = np.hstack([Qfull[:, kt:], Vt])  # Q~ = [V~perp, V~]
    Lf.r[i], Lf.kt[i] = r, kt


def _project(i, D, F, Ni, frow_i, fcol_i, Lf):
    """D <- Q^T D Q and F <- Q^T F Q for cluster i; the V~perp part of F is
    dropped (the fill truncation)."""
    Qt, r = Lf.Q[i], Lf.r[i]
    D[(i, i)] = Qt.T @ D[(i, i)] @ Qt
    for j in Ni:
        if j != i:
            D[(i, j)] = Qt.T @ D[(i, j)]
            D[(j, i)] = D[(j, i)] @ Qt
    for j in frow_i:
        Fij = Qt.T @ F[(i, j)]
        Fij[:r, :] = 0.0
        F[(i, j)] = Fij
    for j in fcol_i:
        Fji = F[(j, i)] @ Qt
        Fji[:, :r] = 0.0
        F[(j, i)] = Fji


def _partial_lu(i, D, F, Ni, nearset, Lf):
    """Partial LU of the redundant rows/columns of i: LU(D_RR), elementary
    factors, Schur updates to D (near pairs) or to the fill F (others)."""
    r = Lf.r[i]
    if r == 0:
        return
    lu = sla.lu_factor(D[(i, i)][:r, :r])
    Lf.lu[i] = lu
    Cp, Rp = {}, {}
    for j in Ni:
        if j == i:
            C = D[(i, i)][:, :r].copy()
            C[:r, :] = 0.0  # only the skeleton rows of i are a neighbour row
            Rw = D[(i, i)][:r, :].copy()
            Rw[:, :r] = 0.0
        else:
            C = D[(j, i)][:, :r].copy()
            Rw = D[(i, j)][:r, :].copy()
        Cp[j], Rp[j] = C, Rw
    Xs = {j: sla.lu_solve(lu, Cp[j].T, trans=1, check_finite=False).T for j in Ni}
    Ys = {k: sla.lu_solve(lu, Rp[k], check_finite=False) for k in Ni}
    for j in Ni:
        for k in Ni:
            delta = -(Cp[j] @ Ys[k])
            if (j, k) in nearset:
                D[(j, k)] = D[(j, k)] + delta
            else:
                F[(j, k)] = F[(j, k)] + delta
    # eliminated rows and columns are zero in D
    for j in Ni:
        if j == i:
            D[(i, i)][r:, :r] = 0.0
            D[(i, i)][:r, r:] = 0.0
        else:
            D[(j, i)][:, :r] = 0.0
            D[(i, j)][:r, :] = 0.0
    Lf.X[i], Lf.Y[i] = Xs, Ys


def _close_out(H, lev, n, V, D, F, Lf):
    """Merge the skeleton parts of level lev into level lev-1."""
    lp = H.level_ptr
    parents = list(range(lp[lev - 1], lp[lev]))
    kt, r = Lf.kt, Lf.r
    n2, off, V2 = {}, {}, {}
    for tau in parents:
        o = 0
        blocks = []
        for c in children(H, tau):
            off[c] = o
            o += kt[c]
            Ec = H.E[c]  # k_c x k_tau
            pad = np.zeros((kt[c] - Ec.shape[0], Ec.shape[1]))
            blocks.append(np.vstack([Ec, pad]))
        n2[tau] = o
        V2[tau] = np.vstack(blocks) if blocks else np.zeros((0, H.rank[tau]))
    nearset = {(c, j) for c in range(lp[lev], lp[lev + 1]) for j in near(H, c)}
    farset = {(c, j) for c in range(lp[lev], lp[lev + 1]) for j in far(H, c)}
    pnear = {(tau, s) for tau in parents for s in near(H, tau)}
    D2 = {}
    for (tau, sg) in sorted(pnear):
        blk = np.zeros((n2[tau], n2[sg]))
        for c in children(H, tau):
            for c2 in children(H, sg):
                rs = slice(off[c], off[c] + kt[c])
                cs = slice(off[c2], off[c2] + kt[c2])
                if (c, c2) in nearset:
                    blk[rs, cs] = D[(c, c2)][r[c]:, r[c2]:]
                elif (c, c2) in farset:
                    S = H.S[(c, c2)]
                    sub = np.zeros((kt[c], kt[c2]))
                    sub[:S.shape[0], :S.shape[1]] = S  # zero-padded coupling S~
                    if (c, c2) in F:
                        sub += F[(c, c2)][r[c]:, r[c2]:]
                    blk[rs, cs] = sub
                else:
                    raise AssertionError("child pair of a near pair is neither near nor far")
        D2[(tau, sg)] = blk
    F2 = {}
    for (c, c2), Fb in F.items():
        pt, ps = H.parent[c], H.parent[c2]
        if (pt, ps) in pnear:
            assert (c, c2) in farset, "fill on a near pair"
            continue
        if (pt, ps) not in F2:
            F2[(pt, ps)] = np.zeros((n2[pt], n2[ps]))
        F2[(pt, ps)][off[c]:off[c] + kt[c], off[c2]:off[c2] + kt[c2]] += Fb[r[c]:, r[c2]:]
    return n2, V2, D2, F2


def _top(Fz, H, lev, n, D):
    """Dense LU (partial pivoting) of the remnant at level lev (Algorithm 1, last steps)."""
    lp = H.level_ptr
    nodes = list(range(lp[lev], lp[lev + 1]))
    off, o = {}, 0
    for q in nodes:
        off[q] = o
        o += n[q]
    M = np.zeros((o, o))
    for (q, s), blk in D.items():
        M[off[q]:off[q] + n[q], off[s]:off[s] + n[s]] = blk
    Fz.top_level = lev
    Fz.top_nodes, Fz.top_off, Fz.top_n = nodes, off, dict(n)
    Fz.n_top = o
    Fz.M = M
    Fz.top_lu = sla.lu_factor(M) if o else None
    return Fz


def solve(Fz, B):
    """Algorithm 3: X = (LU)^{-1} B with B in original point order."""
    B = np.asarray(B, dtype=np.float64)
    one = B.ndim == 1
    if one:
        B = B[:, None]
    b = B[Fz.perm]
    seg = {}
    if Fz.levels:
        lev0 = Fz.levels[0]
        for q in lev0.nodes:
            seg[q] = b[Fz.idx_begin[q]:Fz.idx_end[q]].copy()
    else:
        for q in Fz.top_nodes:
            seg[q] = b[Fz.idx_begin[q]:Fz.idx_end[q]].copy()
    saved = []
    for Lf in Fz.levels:
        ncol = Lf.ncolors
        for c in range(ncol):
            for i in [q for q in Lf.nodes if Lf.color[q] == c]:
                seg[i] = Lf.Q[i].T @ seg[i]
                r = Lf.r[i]
                if r == 0:
                    continue
                bR = seg[i][:r].copy()
                for j in Lf.near[i]:
                    seg[j] = seg[j] - Lf.X[i][j] @ bR
        for i in Lf.nodes:
            r = Lf.r[i]
            if r:
                seg[i][:r] = sla.lu_solve(Lf.lu[i], seg[i][:r])
        saved.append({i: seg[i][:Lf.r[i]].copy() for i in Lf.nodes})
        # upsweep: skeleton parts of the children form the parent vector
        seg = {tau: np.vstack([seg[c][Lf.r[c]:] for c in chs])
               for tau, chs in Lf.children.items()}
    # dense top solve
    if Fz.n_top:
        btop = np.vstack([seg[q] for q in Fz.top_nodes])
        ytop = sla.lu_solve(Fz.top_lu, btop)
    else:
        ytop = np.zeros((0, b.shape[1]))
    seg = {q: ytop[Fz.top_off[q]:Fz.top_off[q] + Fz.top_n[q]] for q in Fz.top_nodes}
    for Lf, z in zip(reversed(Fz.levels), reversed(saved)):
        # downsweep: split parent vectors into the children's skeleton parts
        down = {}
        for tau, chs in Lf.children.items():
            o = 0
            for c in chs:
                kt = Lf.kt[c]
                down[c] = np.vstack([z[c], seg[tau][o:o + kt]])
                o += kt
        seg = down
        for c in range(Lf.ncolors - 1, -1, -1):
            for i in [q for q in Lf.nodes if Lf.color[q] == c]:
                r = Lf.r[i]
                if r:
                    acc = np.zeros_like(seg[i][:r])
                    for k in Lf.near[i]:
                        acc += Lf.Y[i][k] @ seg[k]
                    seg[i][:r] -= acc
                seg[i] = Lf.Q[i] @ seg[i]
    y = np.zeros_like(b)
    for q, v in seg.items():
        y[Fz.idx_begin[q]:Fz.idx_end[q]] = v
    X = np.empty_like(y)
    X[Fz.perm] = y
    return X[:, 0] if one else X


def block_layout(Lf):
    """Section 2.2's memory layout of one level: the blocks of the level's
    pattern (near pairs and fill pairs; rows ascending, columns ascending)
    placed in one buffer for the near blocks and one for the fill blocks, each
    block n_j x n_k, at offsets that are exclusive prefix sums of the products
    of the block dimensions.  The input is symmetric (the standing assumption
    of Section 2), so the fill is too (F_kj = F_jk^T): the fill buffer holds
    one block per unordered pair, (j, k) with j < k, and the entry (k, j)
    names that block.  Returns records (j, k, kind, offset): kind 0 near,
    1 stored fill block, 2 fill entry stored as the transpose of (k, j)."""
    nearset = {(q, j) for q in Lf.nodes for j in Lf.near[q]}
    frow = {q: [] for q in Lf.nodes}
    for (a, k) in Lf.fpat:
        frow[a].append(k)
    out = []
    nxt = {False: 0, True: 0}
    fill_off = {}
    for j in Lf.nodes:
        cols = sorted(set(Lf.near[j]) | set(frow[j]))
        for k in cols:
            isf = (j, k) not in nearset
            if isf and k < j:
                out.append((j, k, 2, fill_off[(k, j)]))
                continue
            if isf:
                fill_off[(j, k)] = nxt[True]
            out.append((j, k, int(isf), nxt[isf]))
            nxt[isf] += Lf.n[j] * Lf.n[k]
    return out


def cluster_offsets(Lf):
    """Offsets of the level's n_i x n_i transforms Q~_i in one buffer
    (exclusive prefix sum of n_i^2, Section 2.2)."""
    out, o = [], 0
    for q in Lf.nodes:
        out.append(o)
        o += Lf.n[q] * Lf.n[q]
    return out


def owner_records(Lf):
    """Flattened (c, j, k, m, i_1..i_m) for every colour c ascending and every
    stored target (j, k) ascending that clusters of colour c update: near
    pairs, and fill pairs with j < k (the fill block of the pair; the update
    of (k, j) is its transpose, see block_layout)."""
    nearset = {(q, j) for q in Lf.nodes for j in Lf.near[q]}
    rec = []
    for (c, j, k) in sorted(Lf.owners):
        if k < j and (j, k) not in nearset:
            continue
        con = Lf.owners[(c, j, k)]
        rec += [c, j, k, len(con)] + list(con)
    return rec


def integer_outputs(Fz):
    """Per level: sizes n, augmented ranks k~, colours and fill pattern; and n_top."""
    out = []
    for Lf in Fz.levels:
        out.append({
            "level": Lf.level,
            "n": [Lf.n[q] for q in Lf.nodes],
            "kt": [Lf.kt[q] for q in Lf.nodes],
            "color": [Lf.color[q] for q in Lf.nodes],
            "fpat": list(Lf.fpat),
        })
    return {"levels": out, "n_top": Fz.n_top}
