"""H^2 construction: Chebyshev interpolation followed by algebraic recompression.

Section 3 of the paper builds its test matrices this way: a tensor grid of
p^d Chebyshev points on each cluster's bounding box, with the order p raised
from p0 at the leaves with every other level; then algebraic compression to a
tolerance eps reduces the ranks and orthogonalises the bases; a diagonal
regularisation alpha*I is added.

Steps (textbook H^2 recompression, Boerm):
  1. interpolation: leaf U = Lagrange polynomials at the points (U = I when
     p^d >= leaf size, the sample points then being the points themselves),
     transfers E_c = parent Lagrange polynomials at the child's sample points,
     couplings S = K(sample_s, sample_t);
  2. orthogonalisation upsweep: QR of the leaf bases and of the stacked
     R_c E_c; couplings become R_s S R_t^T;
  3. total-weight downsweep: W_t = R-factor (transposed) of
     [S_ts^T for s in far(t); (E_t W_parent)^T];
  4. truncation upsweep: SVD of W_t (leaves) or of [T_c E_c] W_t (inner
     nodes), keeping singular values > eps * ||A||; couplings T_s S T_t^T.
When eps >= 1e-7 the weights are kept as Gram matrices instead:
W_t W_t^T = sum over far s of S_ts S_ts^T + E_t (W_p W_p^T) E_t^T, and the
truncation takes the eigendecomposition of W_t W_t^T or Z W_t W_t^T Z^T
(Z = [T_c E_c]), whose eigenvectors and square-rooted eigenvalues are the
left singular vectors and values; this form resolves singular values down to
about 1e-8 of the largest, so it serves the coarser tolerances only, and it
avoids the tall QR factorizations that dominate the construction time.
Cluster bases above the first level with admissible blocks have rank 0.

Arithmetic is float64: kernel evaluations and products in torch on the
requested device, batched per level over zero-padded shapes; the small dense
QR factorizations and eigendecompositions in LAPACK on the host, spread over
its cores.  Far-field kernel blocks are generated in chunks and never stored
uncompressed.
"""
import numpy as np
import torch

from . import tree as treemod


def _cheb(p):
    a = np.arange(p)
    return np.cos((2 * a + 1) * np.pi / (2 * p))


def _lagrange(nodes1d, x):
    """1-D Lagrange basis on `nodes1d` (..., p) evaluated at x (..., n) -> (..., n, p)."""
    p = nodes1d.shape[-1]
    t = nodes1d.unsqueeze(-2)  # (..., 1, p)
    xx = x.unsqueeze(-1)  # (..., n, 1)
    out = torch.ones(x.shape + (p,), dtype=x.dtype, device=x.device)
    for b in range(p):
        tb = nodes1d[..., b:b + 1].unsqueeze(-2)  # (..., 1, 1)
        num = xx - tb
        den = t - tb
        den = torch.where(den == 0, torch.ones_like(den), den)
        f = num / den
        mask = torch.zeros(p, dtype=torch.bool, device=x.device)
        mask[b] = True
        f = torch.where(mask, torch.ones_like(f), f)
        out = out * f
    return out


class _Level:
    pass


def _grid_nodes(lo, hi, p, dev):
    """Chebyshev tensor grid (n, p^d, d) on boxes lo/hi (n, d); axis 0 fastest."""
    n, d = lo.shape
    c = torch.as_tensor(_cheb(p), dtype=torch.float64, device=dev)
    lo_t = torch.as_tensor(lo, dtype=torch.float64, device=dev)
    hi_t = torch.as_tensor(hi, dtype=torch.float64, device=dev)
    mid = 0.5 * (lo_t + hi_t)
    hw = torch.clamp(0.5 * (hi_t - lo_t), min=1e-9)
    nodes1d = mid.unsqueeze(-1) + hw.unsqueeze(-1) * c  # (n, d, p)
    # flat node index = sum_j a_j p^j (axis 0 fastest)
    flat = torch.arange(p ** d, device=dev)
    digits = [(flat // (p ** j)) % p for j in range(d)]
    pts = torch.stack([nodes1d[:, j, :][:, digits[j]] for j in range(d)], dim=-1)
    return pts, nodes1d, digits


def _lagrange_nd(nodes1d, digits, X):
    """Tensor Lagrange basis of boxes (n, d, p) at points X (n, m, d) -> (n, m, p^d)."""
    n, d, p = nodes1d.shape
    out = None
    for j in range(d):
        Lj = _lagrange(nodes1d[:, j, :], X[:, :, j])  # (n, m, p)
        Lj = Lj[:, :, digits[j]]  # (n, m, p^d)
        out = Lj if out is None else out * Lj
    return out


def _host_batched(fn, A, nout):
    """fn (a numpy LAPACK routine on stacked matrices) applied to the device
    batch A on the host: chunks of the batch on a pool of threads, each with a
    single-threaded BLAS (every matrix is factored on its own, so the result
    does not depend on the chunking); outputs return to A's device."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    a = A.detach().cpu().numpy()
    nthr = max(1, min(os.cpu_count() or 1, 32))
    parts = np.array_split(a, min(len(a), 4 * nthr)) if len(a) else [a]
    with threadpool_limits(1, user_api="blas"), ThreadPoolExecutor(nthr) as ex:
        res = list(ex.map(fn, parts))
    outs = [np.concatenate([r[i] for r in res]) for i in range(nout)]
    return tuple(torch.as_tensor(o, device=A.device) for o in outs)


def _bqr(A, mode, chunk=512):
    """Batched QR on the device in slices of at most `chunk` matrices (large
    batches exhaust the solver's workspace)."""
    if A.shape[0] <= chunk:
        return torch.linalg.qr(A, mode=mode)
    parts = [torch.linalg.qr(A[i:i + chunk], mode=mode) for i in range(0, A.shape[0], chunk)]
    return tuple(torch.cat([p[k] for p in parts], 0) for k in range(2))


def _qr_r(A):
    """R factor of batched A (b, m, n); returns (b, n, n) (zero padded when m < n)."""
    b, m, n = A.shape
    if m < n:
        A = torch.cat([A, torch.zeros(b, n - m, n, dtype=A.dtype, device=A.device)], 1)
    return _bqr(A, "r")[1][:, :n, :n]


def construct(pts, kernel, leaf_size=64, tree_kind="kd", eta=0.7, adm_kind=0,
              eps=1e-9, p0=None, device="cpu", chunk_pairs=20000, verbose=False):
    """Build the H^2 representation of kernel(pts) to tolerance eps.

    Returns a dict with the tree, near/far lists, ranks, U (leaf bases), E
    (transfers), D (leaf near blocks) and S (far couplings) as float64 numpy
    arrays, plus norm2 (power-iteration estimate of ||A_H||_2).
    """
    import sys
    import time as _time
    _t0 = _time.perf_counter()

    def say(msg):
        if verbose:
            print(f"[construct {_time.perf_counter() - _t0:7.1f}s] {msg}", file=sys.stderr, flush=True)

    dev = torch.device(device)
    pts = np.asarray(pts, dtype=np.float64)
    N, dim = pts.shape
    if p0 is None:
        p0 = 8 if dim == 2 else 4
    say(f"tree of {N} points")
    t = treemod.build_tree(pts, leaf_size, tree_kind)
    near_ptr, near_col, far_ptr, far_col = treemod.dual_traversal(t, eta, adm_kind)
    L = t.L
    top = treemod.top_level(t, far_ptr)
    lp = t.level_ptr
    P = torch.as_tensor(pts[t.perm], dtype=torch.float64, device=dev)
    sizes = (t.idx_end - t.idx_begin).astype(np.int64)

    say(f"tree: {L} levels, {len(near_col)} near and {len(far_col)} far pairs")
    # ---- dense near field (leaf level) ----
    leaf0 = lp[L]
    nleaf = lp[L + 1] - lp[L]
    mmax = int(sizes[leaf0:].max())
    leafpts = torch.zeros(nleaf, mmax, dim, dtype=torch.float64, device=dev)
    leafmask = torch.zeros(nleaf, mmax, dtype=torch.float64, device=dev)
    for q in range(nleaf):
        a, b = t.idx_begin[leaf0 + q], t.idx_end[leaf0 + q]
        leafpts[q, :b - a] = P[a:b]
        leafmask[q, :b - a] = 1.0

    rows = np.repeat(np.arange(t.n_nodes), np.diff(near_ptr))
    sel = np.nonzero(rows >= leaf0)[0]
    Dt = torch.zeros(len(sel), mmax, mmax, dtype=torch.float64, device=dev)
    for c0 in range(0, len(sel), chunk_pairs):
        e = sel[c0:c0 + chunk_pairs]
        i = rows[e] - leaf0
        j = near_col[e].astype(np.int64) - leaf0
        K = kernel.block(leafpts[i], leafpts[j])
        K = K * leafmask[i].unsqueeze(-1) * leafmask[j].unsqueeze(-2)
        diag = torch.as_tensor(i == j, device=dev)
        K = K + kernel.alpha * torch.diag_embed(leafmask[i]) * diag.view(-1, 1, 1)
        Dt[c0:c0 + len(e)] = K

    rank = np.zeros(t.n_nodes, dtype=np.int32)
    h = _pack(t, near_ptr, near_col, far_ptr, far_col, rank, eps, p0, eta, adm_kind, kernel, top)
    h.update(Dt=Dt, mmax=mmax, Ut=None, Et={}, St={})
    if top is None:
        h["norm2"] = power_norm(h)
        return h

    say("near field done")
    # ---- step 1: interpolation sample points per level (levels top..L) ----
    lev = {}
    for l in range(top, L + 1):
        Lv = _Level()
        a, b = lp[l], lp[l + 1]
        Lv.n = b - a
        p = treemod.chebyshev_order(p0, L, l)
        Lv.p = p
        k0 = p ** dim
        if l == L and k0 >= mmax:
            Lv.identity = True
            Lv.k0 = mmax
            Lv.xi = leafpts
            Lv.mask = leafmask
        else:
            Lv.identity = False
            Lv.k0 = k0
            Lv.xi, Lv.nodes1d, Lv.digits = _grid_nodes(t.lo[a:b], t.hi[a:b], p, dev)
            Lv.mask = torch.ones(Lv.n, k0, dtype=torch.float64, device=dev)
        lev[l] = Lv

    say("interpolation points done")
    # ---- step 2: orthogonalisation upsweep ----
    # Leaf: U0 (mmax x k0) -> Q, R
    Lv = lev[L]
    if Lv.identity:
        Lv.Uq = torch.diag_embed(leafmask)  # (n, mmax, mmax)
        Lv.R = torch.diag_embed(leafmask)
        Lv.k1 = mmax
    else:
        U0 = _lagrange_nd(Lv.nodes1d, Lv.digits, leafpts) * leafmask.unsqueeze(-1)
        Q, R = _host_batched(np.linalg.qr, U0, 2)
        Lv.Uq, Lv.R = Q, R
        Lv.k1 = R.shape[1]
    for l in range(L - 1, top - 1, -1):
        Lv, Lc = lev[l], lev[l + 1]
        a = lp[l]
        arity = int(t.child_ptr[a + 1] - t.child_ptr[a])
        # E0_c = parent Lagrange at child's sample points: (nchild, kc0, kp0)
        par = torch.as_tensor(t.parent[lp[l + 1]:lp[l + 2]] - a, device=dev).long()
        E0 = _lagrange_nd(Lv.nodes1d[par], Lv.digits, Lc.xi) * Lc.mask.unsqueeze(-1)
        RE = torch.bmm(Lc.R, E0)  # (nchild, kc1, kp0)
        Z = RE.reshape(Lv.n, arity * Lc.k1, Lv.k0)
        Q, R = _host_batched(np.linalg.qr, Z, 2)
        Lv.k1 = R.shape[1]
        Lv.R = R
        Lc.E1 = Q.reshape(Lv.n * arity, Lc.k1, Lv.k1)  # orthonormal stacked transfers

    # far pairs by level (local indices)
    far_rows = np.repeat(np.arange(t.n_nodes), np.diff(far_ptr))

    def far_of_level(l):
        a, b = lp[l], lp[l + 1]
        e = np.nonzero((far_rows >= a) & (far_rows < b))[0]
        return e, far_rows[e] - a, far_col[e].astype(np.int64) - a

    def coupling(l, i, j, Bi, Bj):
        """Bi K(xi_i, xi_j) Bj^T for local node index arrays i, j (chunked by caller)."""
        Lv = lev[l]
        K = kernel.block(Lv.xi[i], Lv.xi[j]) * Lv.mask[i].unsqueeze(-1) * Lv.mask[j].unsqueeze(-2)
        return torch.bmm(torch.bmm(Bi, K), Bj.transpose(1, 2))

    # norm estimate for the truncation threshold: Rayleigh quotient of the
    # all-ones vector, 1^T A 1 / N, from sampled rows (a lower bound of ||A||_2)
    ns = min(N, 256)
    rows_s = (np.arange(ns) * N) // ns
    acc = 0.0
    for c0 in range(0, ns, 16):
        Xr = P[rows_s[c0:c0 + 16]]
        acc += float(kernel.block(Xr.unsqueeze(0), P.unsqueeze(0)).sum()) + kernel.alpha * len(Xr)
    norm_pre = acc / ns
    thr = eps * norm_pre

    say("orthogonalisation done")
    # The weights in Gram form resolve singular values down to about
    # sqrt(unit roundoff) of the largest: used when the truncation threshold
    # eps stays above that with margin (eps >= 1e-7, eps^2 about 45 unit
    # roundoffs; the slack absorbs the rounding of tol / 10); otherwise the R
    # factors of the stacked rows are formed (QR).
    gram = eps >= 1e-7 * (1.0 - 1e-9)
    # ---- step 3: total-weight downsweep ----
    for l in range(top, L + 1):
        say(f"weights, level {l} ({'Gram' if gram else 'QR'})")
        Lv = lev[l]
        e, fi, fj = far_of_level(l)
        k1 = Lv.k1
        cnt = np.bincount(fi, minlength=Lv.n)
        cmax = max(int(cnt.max()), 1)
        order = np.argsort(fi, kind="stable")
        starts = np.concatenate([[0], np.cumsum(cnt)])
        if gram:
            # Gamma_t = W_t W_t^T = sum over far pairs (t, s) of S'_ts S'_ts^T
            # plus E1_t Gamma_parent E1_t^T
            Gm = torch.zeros(Lv.n, k1, k1, dtype=torch.float64, device=dev)
            node_chunk = max(1, int(2e8 // max(1, cmax * k1 * k1)))
        else:
            W = torch.zeros(Lv.n, k1, k1, dtype=torch.float64, device=dev)
            kp = lev[l - 1].W.shape[2] if l > top else 0
            maxrows = int(cnt.max()) * k1 + kp
            node_chunk = max(1, int(2e8 // max(1, maxrows * k1)))
        for n0 in range(0, Lv.n, node_chunk):
            n1 = min(Lv.n, n0 + node_chunk)
            sl = order[starts[n0]:starts[n1]]
            if gram:
                if len(sl):
                    ii, jj = fi[sl], fj[sl]
                    Sp = coupling(l, ii, jj, Lv.R[ii], Lv.R[jj])  # (npairs, k1, k1)
                    # the node's blocks side by side, in CSR order, zero
                    # padded: their product with their own transpose sums
                    # S' S'^T in a fixed order (no atomics)
                    slot = np.arange(starts[n0], starts[n1]) - starts[ii]
                    Y = torch.zeros(n1 - n0, cmax, k1, k1, dtype=torch.float64, device=dev)
                    Y[torch.as_tensor(ii - n0, device=dev), torch.as_tensor(slot, device=dev)] = Sp
                    Y = Y.permute(0, 2, 1, 3).reshape(n1 - n0, k1, cmax * k1)
                    Gm[n0:n1] = torch.bmm(Y, Y.transpose(1, 2))
                if l > top:
                    par = torch.as_tensor(t.parent[lp[l] + np.arange(n0, n1)] - lp[l - 1],
                                          device=dev).long()
                    E1 = Lv.E1[n0:n1]
                    Gm[n0:n1] += torch.bmm(torch.bmm(E1, lev[l - 1].Gm[par]), E1.transpose(1, 2))
            else:
                # W_t = R^T, R the R factor of the stacked rows
                # [S'_ts^T for s in far(t); (E1_t W_parent)^T]
                blocks = torch.zeros(n1 - n0, maxrows, k1, dtype=torch.float64, device=dev)
                if len(sl):
                    ii, jj = fi[sl], fj[sl]
                    Sp = coupling(l, ii, jj, Lv.R[ii], Lv.R[jj])
                    slot = np.arange(starts[n0], starts[n1]) - starts[ii]
                    # a view of the stacked blocks (slot, k1 x k1): the indexed
                    # assignment writes through to `blocks`
                    tmp = blocks[:, :int(cnt.max()) * k1].view(n1 - n0, int(cnt.max()), k1, k1)
                    tmp[torch.as_tensor(ii - n0, device=dev),
                        torch.as_tensor(slot, device=dev)] = Sp.transpose(1, 2)
                if l > top:
                    par = torch.as_tensor(t.parent[lp[l] + np.arange(n0, n1)] - lp[l - 1],
                                          device=dev).long()
                    EW = torch.bmm(Lv.E1[n0:n1], lev[l - 1].W[par])  # (nb, k1, kp)
                    blocks[:, maxrows - kp:maxrows, :] = EW.transpose(1, 2)
                W[n0:n1] = _qr_r(blocks).transpose(1, 2)
        if gram:
            Lv.Gm = Gm
        else:
            Lv.W = W

    say("weights done")
    # ---- step 4: truncation upsweep ----
    for l in range(L, top - 1, -1):
        say(f"truncation, level {l}")
        Lv = lev[l]
        if l < L:
            Lc = lev[l + 1]
            arity = Lc.n // Lv.n
            TE = torch.bmm(Lc.T, Lc.E1)  # (nchild, kc2max, k1)
            Z = TE.reshape(Lv.n, arity * Lc.T.shape[1], Lv.k1)
            Lv.Z = Z
        # coordinates that are padding (leaf points that do not exist, child
        # basis vectors beyond a child's rank)
        if l == L:
            valid = Lv.mask if Lv.identity else torch.ones(Lv.n, Lv.k1, dtype=torch.float64,
                                                            device=dev)
        else:
            kc = torch.as_tensor(Lc.k2, device=dev).view(Lv.n, arity, 1)
            valid = (torch.arange(Lc.T.shape[1], device=dev).view(1, 1, -1) < kc)
            valid = valid.reshape(Lv.n, -1).to(torch.float64)
        rows = valid.shape[1]
        if gram:
            MM = Lv.Gm if l == L else torch.bmm(torch.bmm(Z, Lv.Gm), Z.transpose(1, 2))
            # padding rows of M M^T are zero; a diagonal of -2 ||M M^T|| there
            # separates them from every kept eigenvector, which then has no
            # component on them
            MM = 0.5 * (MM + MM.transpose(1, 2))
            big = (MM.abs().amax(dim=(1, 2)) if rows else
                   torch.zeros(Lv.n, dtype=torch.float64, device=dev)).clamp(min=1.0)
            MM = MM * valid.unsqueeze(1) * valid.unsqueeze(2)
            MM = MM - torch.diag_embed((1.0 - valid) * 2.0 * big.view(-1, 1))
            # M M^T = P diag(sigma^2) P^T, eigenvalues descending; the small
            # batched eigenproblems run on the host (LAPACK)
            if rows:
                lam, Pm = _host_batched(np.linalg.eigh, MM, 2)
            else:
                lam, Pm = MM.new_zeros(Lv.n, 0), MM.new_zeros(Lv.n, 0, 0)
            lam, Pm = lam.flip(-1), Pm.flip(-1)
            sv = torch.sqrt(torch.clamp(lam, min=0.0))
        else:
            M = Lv.W if l == L else torch.bmm(Z, Lv.W)
            # the small batched SVDs run on the host (LAPACK)
            if rows:
                Pm, sv = _host_batched(lambda a: np.linalg.svd(a, full_matrices=False)[:2], M, 2)
            else:
                Pm, sv = M.new_zeros(Lv.n, 0, 0), M.new_zeros(Lv.n, 0)
        k2 = (sv > thr).sum(1).cpu().numpy()
        Lv.k2 = k2
        k2max = max(int(k2.max()), 0)
        Pk = Pm[:, :, :k2max] * (torch.arange(k2max, device=dev).view(1, 1, -1)
                                   < torch.as_tensor(k2, device=dev).view(-1, 1, 1))
        Pk = Pk * valid.unsqueeze(2)
        Lv.Pk = Pk
        if l == L:
            Lv.T = Pk.transpose(1, 2)  # (n, k2max, k1)
            Lv.Unew = torch.bmm(Lv.Uq, Pk)  # (n, mmax, k2max)
        else:
            Lv.T = torch.bmm(Pk.transpose(1, 2), Lv.Z)
        rank[lp[l]:lp[l + 1]] = k2

    # transfers (per level, padded) and leaf bases
    h["Ut"] = Lv.Unew if L == top else lev[L].Unew
    for l in range(top + 1, L + 1):
        Lv, Lp = lev[l], lev[l - 1]
        arity = Lv.n // Lp.n
        k2c = Lv.T.shape[1]
        kpm = Lp.Pk.shape[2]
        h["Et"][l] = Lp.Pk.reshape(Lp.n, arity, k2c, kpm).reshape(Lv.n, k2c, kpm)

    # couplings: S'' = (T R) K (T R)^T, padded per level
    say("bases done")
    for l in range(top, L + 1):
        say(f"couplings, level {l}")
        Lv = lev[l]
        B = torch.bmm(Lv.T, Lv.R)  # (n, k2max, k0)
        e, fi, fj = far_of_level(l)
        k2m = B.shape[1]
        Sl = torch.zeros(len(e), k2m, k2m, dtype=torch.float64, device=dev)
        for c0 in range(0, len(e), chunk_pairs):
            ii, jj = fi[c0:c0 + chunk_pairs], fj[c0:c0 + chunk_pairs]
            Sl[c0:c0 + len(ii)] = coupling(l, ii, jj, B[ii], B[jj])
        h["St"][l] = (e, fi, fj, Sl)
        lev[l] = None
    say("norm estimate")
    h["norm2"] = power_norm(h)
    say("done")
    return h


def _pack(t, near_ptr, near_col, far_ptr, far_col, rank, eps, p0, eta, adm_kind, kernel, top):
    return {
        "N": t.N, "dim": t.dim, "L": t.L, "n_nodes": t.n_nodes, "perm": t.perm,
        "level_ptr": t.level_ptr, "parent": t.parent, "child_ptr": t.child_ptr,
        "idx_begin": t.idx_begin, "idx_end": t.idx_end, "rank": rank,
        "near_ptr": near_ptr, "near_col": near_col, "far_ptr": far_ptr, "far_col": far_col,
        "eps": eps, "p0": p0, "eta": eta, "adm_kind": adm_kind, "kernel": kernel.spec(),
        "top": top, "tree": t,
    }


def matvec(h, X):
    """y = A_H x for the constructed representation (tree order in and out).

    Used only inside the generator to estimate ||A_H||_2; the oracle and the
    GPU path carry their own products.  X is a torch float64 (N, nrhs) tensor
    on the construction device.
    """
    dev = X.device
    lp, L, top = h["level_ptr"], h["L"], h["top"]
    ib, ie = h["idx_begin"], h["idx_end"]
    mmax = h["mmax"]
    nrhs = X.shape[1]
    leaf0 = lp[L]
    nleaf = lp[L + 1] - leaf0
    sizes = ie[leaf0:] - ib[leaf0:]
    # padded leaf segments
    rowi = np.repeat(np.arange(nleaf), sizes)
    rowp = np.arange(h["N"]) - np.repeat(ib[leaf0:], sizes)
    ri = torch.as_tensor(rowi, device=dev)
    rp = torch.as_tensor(rowp, device=dev)
    XL = torch.zeros(nleaf, mmax, nrhs, dtype=X.dtype, device=dev)
    XL[ri, rp] = X
    YL = torch.zeros_like(XL)
    if top is not None:
        xh = {L: torch.bmm(h["Ut"].transpose(1, 2), XL)}
        for l in range(L - 1, top - 1, -1):
            E = h["Et"][l + 1]
            n = lp[l + 1] - lp[l]
            t = torch.bmm(E.transpose(1, 2), xh[l + 1])
            arity = E.shape[0] // n
            xh[l] = t.reshape(n, arity, t.shape[1], nrhs).sum(1)
        yh = {}
        for l in range(top, L + 1):
            e, fi, fj, Sl = h["St"][l]
            y = torch.zeros_like(xh[l])
            if len(e):
                y.index_add_(0, torch.as_tensor(fi, device=dev),
                             torch.bmm(Sl, xh[l][torch.as_tensor(fj, device=dev)]))
            yh[l] = y
        for l in range(top + 1, L + 1):
            E = h["Et"][l]
            par = torch.as_tensor(h["parent"][lp[l]:lp[l + 1]] - lp[l - 1], device=dev).long()
            yh[l] = yh[l] + torch.bmm(E, yh[l - 1][par])
        YL += torch.bmm(h["Ut"], yh[L])
    rows = np.repeat(np.arange(h["n_nodes"]), np.diff(h["near_ptr"]))
    sel = np.nonzero(rows >= leaf0)[0]
    Dt = h["Dt"]
    for c0 in range(0, len(sel), 65536):
        e = sel[c0:c0 + 65536]
        i = torch.as_tensor(rows[e] - leaf0, device=dev)
        j = torch.as_tensor(h["near_col"][e].astype(np.int64) - leaf0, device=dev)
        YL.index_add_(0, i, torch.bmm(Dt[c0:c0 + len(e)], XL[j]))
    return YL[ri, rp]


def power_norm(h, iters=30):
    """||A_H||_2 by power iteration from the normalised all-ones vector."""
    dev = h["Dt"].device
    N = h["N"]
    x = torch.full((N, 1), 1.0 / np.sqrt(N), dtype=torch.float64, device=dev)
    nrm = 0.0
    for _ in range(iters):
        y = matvec(h, x)
        nrm = float(torch.linalg.norm(y))
        if nrm == 0.0:
            break
        x = y / nrm
    return nrm
