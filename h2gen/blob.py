"""Writer of the serialized H^2 matrix ("blob", format H2B1 version 1).

Little-endian.  A 128-byte header followed by 8-byte aligned sections:

  header  magic "H2B1", u32 version=1, u32 flags (bit0 = symmetric, required),
          u32 dim, i64 N, i32 L (leaf level, root = level 0),
          i32 n_nodes, f64 norm2 (||A_H||_2 estimate), f64 eps_construct,
          i32 p0, i32 adm_kind, f64 eta, i64 nnz_near, i64 nnz_far, i64 total_bytes
  perm       i64[N]          tree position -> original point index
  level_ptr  i32[L+2]        nodes of level l are level_ptr[l] .. level_ptr[l+1]-1 (BFS order)
  parent     i32[n_nodes]    -1 for the root
  child_ptr  i32[n_nodes+1]  children of k are child_ptr[k] .. child_ptr[k+1]-1
  idx_begin  i64[n_nodes], idx_end i64[n_nodes]   point range (tree order)
  rank       i32[n_nodes]    k of each cluster basis (0 allowed)
  near_ptr   i64[n_nodes+1], near_col i32[nnz_near]   same-level inadmissible pairs, sorted
  far_ptr    i64[n_nodes+1], far_col  i32[nnz_far]    same-level admissible pairs, sorted
  U          leaf bases, leaf order, m_i x k_i column-major f64
  E          transfers of every non-root node in node order, k_c x k_parent
  D          dense blocks of the leaf-level near pairs in CSR order, m_i x m_j
  S          couplings of all far pairs in CSR order, k_i x k_j

All data offsets are prefix sums of the block dimension products.
"""
import struct

import numpy as np

MAGIC = b"H2B1"
VERSION = 1
HEADER_BYTES = 128
# field byte offsets: magic 0, version 4, flags 8, dim 12, N 16, L 24, n_nodes 28,
# norm2 32, eps_construct 40, p0 48, adm_kind 52, eta 56, nnz_near 64, nnz_far 72,
# total_bytes 80
_HDR = "<4sIIIqiiddiidqqq"


def _align8(n):
    return (n + 7) & ~7


def write_blob(h):
    """Serialise the constructor output `h` into a numpy uint8 array."""
    import torch

    N, L, nn = int(h["N"]), int(h["L"]), int(h["n_nodes"])
    lp = h["level_ptr"]
    rank = h["rank"].astype(np.int32)
    sizes = (h["idx_end"] - h["idx_begin"]).astype(np.int64)
    parent = h["parent"]
    near_ptr, near_col = h["near_ptr"].astype(np.int64), h["near_col"].astype(np.int32)
    far_ptr, far_col = h["far_ptr"].astype(np.int64), h["far_col"].astype(np.int32)
    leaf0 = int(lp[L])
    rows = np.repeat(np.arange(nn), np.diff(near_ptr))
    dsel = np.nonzero(rows >= leaf0)[0]

    secs = [
        h["perm"].astype(np.int64), lp.astype(np.int32), parent.astype(np.int32),
        h["child_ptr"].astype(np.int32), h["idx_begin"].astype(np.int64),
        h["idx_end"].astype(np.int64), rank, near_ptr, near_col, far_ptr, far_col,
    ]
    nU = int(sum(sizes[q] * rank[q] for q in range(leaf0, nn)))
    nE = int(sum(int(rank[c]) * int(rank[parent[c]]) for c in range(1, nn)))
    nD = int(sum(sizes[rows[e]] * sizes[near_col[e]] for e in dsel)) if len(dsel) else 0
    frows = np.repeat(np.arange(nn), np.diff(far_ptr))
    nS = int((rank[frows].astype(np.int64) * rank[far_col].astype(np.int64)).sum())
    off = HEADER_BYTES
    for a in secs:
        off = _align8(off + a.nbytes)
    total = off + 8 * (nU + nE + nD + nS)
    buf = np.zeros(total, dtype=np.uint8)
    hdr = struct.pack(_HDR, MAGIC, VERSION, 1, int(h["dim"]), N, L, nn,
                      float(h["norm2"]), float(h["eps"]), int(h["p0"]), int(h["adm_kind"]),
                      float(h["eta"]), int(near_ptr[-1]), int(far_ptr[-1]), total)
    buf[:len(hdr)] = np.frombuffer(hdr, dtype=np.uint8)
    off = HEADER_BYTES
    for a in secs:
        buf[off:off + a.nbytes] = np.frombuffer(np.ascontiguousarray(a).tobytes(), dtype=np.uint8)
        off = _align8(off + a.nbytes)
    data = buf[off:].view(np.float64)
    pos = 0

    def put(block):
        nonlocal pos
        # column-major: the transpose of a row-major array, flattened
        flat = np.ascontiguousarray(block.T).reshape(-1)
        data[pos:pos + flat.size] = flat
        pos += flat.size

    if h["Ut"] is not None:
        Ut = h["Ut"].cpu().numpy()
        for q in range(leaf0, nn):
            put(Ut[q - leaf0, :sizes[q], :rank[q]])
    top = h["top"]
    for c in range(1, nn):
        l = int(np.searchsorted(lp, c, side="right") - 1)
        kc, kp = int(rank[c]), int(rank[parent[c]])
        if kc * kp:
            Et = h["Et"][l]
            put(Et[c - lp[l], :kc, :kp].cpu().numpy())
    Dt = h["Dt"]
    msz = sizes[leaf0:]
    if len(dsel) and np.all(msz == msz[0]) and msz[0] == Dt.shape[1]:
        m = int(msz[0])
        arr = Dt.transpose(1, 2).contiguous().reshape(-1).cpu().numpy()
        data[pos:pos + arr.size] = arr
        pos += arr.size
    else:
        Dn = Dt.cpu().numpy()
        for r, e in enumerate(dsel):
            put(Dn[r, :sizes[rows[e]], :sizes[near_col[e]]])
    if top is not None:
        for l in range(top, L + 1):
            e, fi, fj, Sl = h["St"][l]
            Sn = Sl.cpu().numpy()
            a = lp[l]
            for r in range(len(e)):
                ki, kj = rank[a + fi[r]], rank[a + fj[r]]
                if ki * kj:
                    put(Sn[r, :ki, :kj])
    assert pos == data.size, (pos, data.size)
    del torch
    return buf


def save(path, buf):
    buf.tofile(path)


def load(path):
    return np.fromfile(path, dtype=np.uint8)
