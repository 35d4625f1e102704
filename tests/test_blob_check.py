"""Load-time validation through the C ABI (h2_blob_check, host only): a
valid serialized matrix passes, and each kind of damage is reported as a
format error naming the failed check (symmetry and orthonormality are the
standing assumptions of the representation, Section 1.1 and Section 2)."""
import numpy as np
import pytest

from conftest import workload

H2_SUCCESS, H2_ERROR_FORMAT = 0, 2


@pytest.fixture(scope="module")
def h2():
    import paper_2509_11152_amd as h2

    return h2


@pytest.fixture(scope="module")
def base():
    from oracle import blob as ob

    blob = np.array(workload("exp2d_1024")["blob"], dtype=np.uint8)
    return blob, ob.parse(blob)


def _data_offsets(H, nbytes):
    """Byte offsets of the U, E, D and S blocks in the blob's data section
    (leaf U, transfers of nodes 1.., near blocks in CSR order, far couplings)."""
    size = H.idx_end - H.idx_begin
    leaf0 = H.level_ptr[H.L]
    shapes = []
    for q in range(leaf0, H.n_nodes):
        shapes.append((("U", q), size[q], H.rank[q]))
    for c in range(1, H.n_nodes):
        shapes.append((("E", c), H.rank[c], H.rank[H.parent[c]]))
    for q in range(leaf0, H.n_nodes):
        for e in range(H.near_ptr[q], H.near_ptr[q + 1]):
            shapes.append((("D", q, int(H.near_col[e])), size[q], size[H.near_col[e]]))
    for q in range(H.n_nodes):
        for e in range(H.far_ptr[q], H.far_ptr[q + 1]):
            shapes.append((("S", q, int(H.far_col[e])), H.rank[q], H.rank[H.far_col[e]]))
    total = sum(int(m) * int(n) for _, m, n in shapes)
    off = nbytes - 8 * total
    out = {}
    for key, m, n in shapes:
        out[key] = (off, int(m), int(n))
        off += 8 * int(m) * int(n)
    return out


def _poke(blob, byte_off, value):
    b = blob.copy()
    b[byte_off:byte_off + 8] = np.frombuffer(np.float64(value).tobytes(), dtype=np.uint8)
    return b


def _peek(blob, byte_off):
    return float(np.frombuffer(blob[byte_off:byte_off + 8].tobytes(), dtype=np.float64)[0])


def test_valid_blob_passes(h2, base):
    code, msg = h2.blob_check(base[0])
    assert code == H2_SUCCESS, msg


def test_bad_magic_and_truncation(h2, base):
    blob = base[0].copy()
    blob[0] = ord("X")
    code, msg = h2.blob_check(blob)
    assert code == H2_ERROR_FORMAT and "magic" in msg
    code, msg = h2.blob_check(base[0][:-8])
    assert code == H2_ERROR_FORMAT


def test_non_finite_entry(h2, base):
    blob, H = base
    offs = _data_offsets(H, blob.nbytes)
    key = next(k for k in offs if k[0] == "D")
    code, msg = h2.blob_check(_poke(blob, offs[key][0], np.nan))
    assert code == H2_ERROR_FORMAT and "non-finite" in msg


def test_asymmetric_near_block(h2, base):
    blob, H = base
    offs = _data_offsets(H, blob.nbytes)
    key = next(k for k in offs if k[0] == "D" and k[1] != k[2])
    o = offs[key][0] + 8 * 3  # entry (3, 0) of D_ij; D_ji keeps its value
    code, msg = h2.blob_check(_poke(blob, o, _peek(blob, o) + 1e-6 * H.norm2))
    assert code == H2_ERROR_FORMAT and "near blocks are not symmetric" in msg


def test_asymmetric_coupling(h2, base):
    blob, H = base
    offs = _data_offsets(H, blob.nbytes)
    key = next(k for k in offs if k[0] == "S" and offs[k][1] * offs[k][2] > 1)
    o = offs[key][0]
    code, msg = h2.blob_check(_poke(blob, o, _peek(blob, o) + 1e-6 * H.norm2))
    assert code == H2_ERROR_FORMAT and "couplings are not symmetric" in msg


def test_non_orthonormal_leaf_basis(h2, base):
    blob, H = base
    offs = _data_offsets(H, blob.nbytes)
    key = next(k for k in offs if k[0] == "U" and offs[k][2] > 0)
    o = offs[key][0]
    code, msg = h2.blob_check(_poke(blob, o, _peek(blob, o) * 1.001 + 1e-3))
    assert code == H2_ERROR_FORMAT and "leaf basis" in msg


def test_non_orthonormal_transfers(h2):
    from oracle import blob as ob

    blob = np.array(workload("exp2d_4096")["blob"], dtype=np.uint8)
    H = ob.parse(blob)
    offs = _data_offsets(H, blob.nbytes)
    key = next(k for k in offs if k[0] == "E" and offs[k][1] * offs[k][2] > 0)
    o = offs[key][0]
    code, msg = h2.blob_check(_poke(blob, o, _peek(blob, o) + 1e-3))
    assert code == H2_ERROR_FORMAT and "transfers" in msg


def test_bad_permutation(h2, base):
    blob = base[0].copy()
    # perm starts right after the 128-byte header: duplicate its first entry
    blob[128 + 8:128 + 16] = blob[128:136]
    code, msg = h2.blob_check(blob)
    assert code == H2_ERROR_FORMAT and "perm" in msg
