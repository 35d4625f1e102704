"""Oracle-side reader of the serialized H^2 matrix (format H2B1 version 1).

TEST INFRASTRUCTURE ONLY: the oracle is the slow CPU reference that the GPU
path is checked against; nothing in the product imports it.

The oracle parses the blob itself (it shares no parser with the library).
Blocks are returned as numpy float64 arrays in column-major (Fortran) order.
"""
import struct

import numpy as np


class H2:
    """Plain container of the symmetric H^2 matrix of Section 1.1:
    cluster tree, near/far lists, leaf bases U, transfers E, dense near blocks D
    and couplings S."""


def parse(buf):
    buf = np.asarray(buf, dtype=np.uint8)
    raw = buf.tobytes()
    magic, version, flags, dim = struct.unpack_from("<4sIII", raw, 0)
    if magic != b"H2B1" or version != 1:
        raise ValueError("not an H2B1 v1 blob")
    if not (flags & 1):
        raise ValueError("only symmetric matrices are supported")
    (N,) = struct.unpack_from("<q", raw, 16)
    L, nn = struct.unpack_from("<ii", raw, 24)
    norm2, eps = struct.unpack_from("<dd", raw, 32)
    p0, adm_kind = struct.unpack_from("<ii", raw, 48)
    (eta,) = struct.unpack_from("<d", raw, 56)
    nnz_near, nnz_far, total = struct.unpack_from("<qqq", raw, 64)
    if total != len(raw):
        raise ValueError("blob length mismatch")
    H = H2()
    H.N, H.dim, H.L, H.n_nodes = N, dim, L, nn
    H.norm2, H.eps, H.p0, H.adm_kind, H.eta = norm2, eps, p0, adm_kind, eta
    off = 128

    def take(dtype, count):
        nonlocal off
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=off).copy()
        off += a.nbytes
        off = (off + 7) & ~7
        return a

    H.perm = take(np.int64, N)
    H.level_ptr = take(np.int32, L + 2).astype(np.int64)
    H.parent = take(np.int32, nn).astype(np.int64)
    H.child_ptr = take(np.int32, nn + 1).astype(np.int64)
    H.idx_begin = take(np.int64, nn)
    H.idx_end = take(np.int64, nn)
    H.rank = take(np.int32, nn).astype(np.int64)
    H.near_ptr = take(np.int64, nn + 1)
    H.near_col = take(np.int32, nnz_near).astype(np.int64)
    H.far_ptr = take(np.int64, nn + 1)
    H.far_col = take(np.int32, nnz_far).astype(np.int64)
    data = np.frombuffer(raw, dtype=np.float64, offset=off)
    pos = 0

    def block(m, n):
        nonlocal pos
        a = data[pos:pos + m * n].reshape(n, m).T.copy(order="F")
        pos += m * n
        return a

    size = H.idx_end - H.idx_begin
    H.size = size
    leaf0 = H.level_ptr[L]
    H.U = {q: block(size[q], H.rank[q]) for q in range(leaf0, nn)}
    H.E = {c: block(H.rank[c], H.rank[H.parent[c]]) for c in range(1, nn)}
    H.D = {}
    for q in range(leaf0, nn):
        for e in range(H.near_ptr[q], H.near_ptr[q + 1]):
            j = H.near_col[e]
            H.D[(q, j)] = block(size[q], size[j])
    H.S = {}
    for q in range(nn):
        for e in range(H.far_ptr[q], H.far_ptr[q + 1]):
            j = H.far_col[e]
            H.S[(q, j)] = block(H.rank[q], H.rank[j])
    if pos != data.size:
        raise ValueError("blob data size mismatch")
    H.level_of = np.zeros(nn, dtype=np.int64)
    for lev in range(L + 1):
        H.level_of[H.level_ptr[lev]:H.level_ptr[lev + 1]] = lev
    H.top = None
    for lev in range(L + 1):
        a, b = H.level_ptr[lev], H.level_ptr[lev + 1]
        if H.far_ptr[b] > H.far_ptr[a]:
            H.top = lev
            break
    return H


def near(H, q):
    return [int(j) for j in H.near_col[H.near_ptr[q]:H.near_ptr[q + 1]]]


def far(H, q):
    return [int(j) for j in H.far_col[H.far_ptr[q]:H.far_ptr[q + 1]]]


def children(H, q):
    return list(range(int(H.child_ptr[q]), int(H.child_ptr[q + 1])))
