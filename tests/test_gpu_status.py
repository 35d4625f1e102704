"""Status codes of the C ABI on the device: every failure is reported as a
status with a message, never as an abort.  Also the factorization options
(norm override, device-memory cap) and the context's allocators."""
import numpy as np
import pytest

from conftest import EXP3D_4096, workload

pytestmark = pytest.mark.gpu

H2_ERROR_INVALID_ARGUMENT, H2_ERROR_FORMAT, H2_ERROR_OUT_OF_MEMORY, H2_ERROR_SINGULAR = 1, 2, 3, 4


@pytest.fixture(scope="module")
def lib():
    import torch

    assert torch.cuda.is_available()
    import paper_2509_11152_amd as h2

    return h2


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _cuda(a):
    import torch

    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_load_rejects_a_damaged_blob(lib, ctx):
    print("[gpu] load of a damaged blob", flush=True)
    blob = np.array(workload("exp2d_1024")["blob"], dtype=np.uint8)
    blob[0] = ord("X")
    with pytest.raises(lib.H2Error) as e:
        lib.Matrix(ctx, blob)
    assert e.value.code == H2_ERROR_FORMAT and "magic" in str(e.value)


def test_invalid_tolerance(lib, ctx):
    print("[gpu] invalid tolerance", flush=True)
    H = lib.Matrix(ctx, workload("exp2d_1024")["blob"])
    for tol in (float("nan"), -1.0, float("inf")):
        with pytest.raises(lib.H2Error) as e:
            lib.Factor(ctx, H, tol)
        assert e.value.code == H2_ERROR_INVALID_ARGUMENT
    with pytest.raises(lib.H2Error) as e:
        lib.Factor(ctx, H, 1e-8, lds_limit_kib=-1)
    assert e.value.code == H2_ERROR_INVALID_ARGUMENT


def test_memory_cap(lib, ctx):
    """A cap below what the factorization needs fails with OUT_OF_MEMORY and
    leaves the context usable; a cap above its measured peak succeeds."""
    print("[gpu] device-memory cap", flush=True)
    w = workload("exp3d_4096", EXP3D_4096)
    H = lib.Matrix(ctx, w["blob"])
    tol = w["spec"]["tol"]
    with pytest.raises(lib.H2Error) as e:
        lib.Factor(ctx, H, tol, pool_bytes=1 << 20)
    assert e.value.code == H2_ERROR_OUT_OF_MEMORY and "cap" in str(e.value)
    F = lib.Factor(ctx, H, tol)
    peak = F.stats()["peak_bytes"]
    F2 = lib.Factor(ctx, H, tol, pool_bytes=peak)
    B = _cuda(w["B"])
    assert np.array_equal(F.solve(B).cpu().numpy(), F2.solve(B).cpu().numpy())


def test_norm_override(lib, ctx):
    """eps_fill = tol ||A||_2: doubling the norm is doubling the tolerance,
    exactly (same ranks, same bits)."""
    print("[gpu] norm override", flush=True)
    w = workload("exp3d_4096", EXP3D_4096)
    H = lib.Matrix(ctx, w["blob"])
    tol = w["spec"]["tol"]
    Fa = lib.Factor(ctx, H, tol, norm2=2 * H.norm2)
    Fb = lib.Factor(ctx, H, 2 * tol)
    Fc = lib.Factor(ctx, H, tol)
    B = _cuda(w["B"])
    for lev in Fa.levels():
        assert (Fa.ints(lev, lib.INT_RANKS) == Fb.ints(lev, lib.INT_RANKS)).all()
    assert np.array_equal(Fa.solve(B).cpu().numpy(), Fb.solve(B).cpu().numpy())
    ra = sum(int(Fa.ints(lev, lib.INT_RANKS).sum()) for lev in Fa.levels())
    rc = sum(int(Fc.ints(lev, lib.INT_RANKS).sum()) for lev in Fc.levels())
    assert ra <= rc


def test_zero_pivot_is_singular(lib, ctx):
    """A matrix whose near blocks and couplings are all zero has zero
    redundant blocks: the factorization reports SINGULAR."""
    print("[gpu] singular matrix", flush=True)
    from oracle import blob as ob

    blob = np.array(workload("exp2d_1024")["blob"], dtype=np.uint8)
    Ho = ob.parse(blob)
    size = Ho.idx_end - Ho.idx_begin
    leaf0 = Ho.level_ptr[Ho.L]
    nU = sum(int(size[q] * Ho.rank[q]) for q in range(leaf0, Ho.n_nodes))
    nE = sum(int(Ho.rank[c] * Ho.rank[Ho.parent[c]]) for c in range(1, Ho.n_nodes))
    nD = sum(int(size[q] * size[Ho.near_col[e]]) for q in range(leaf0, Ho.n_nodes)
             for e in range(Ho.near_ptr[q], Ho.near_ptr[q + 1]))
    nS = sum(int(Ho.rank[q] * Ho.rank[Ho.far_col[e]]) for q in range(Ho.n_nodes)
             for e in range(Ho.far_ptr[q], Ho.far_ptr[q + 1]))
    start = blob.nbytes - 8 * (nU + nE + nD + nS) + 8 * (nU + nE)
    blob[start:] = 0
    H = lib.Matrix(ctx, blob)
    with pytest.raises(lib.H2Error) as e:
        lib.Factor(ctx, H, 1e-8)
    assert e.value.code == H2_ERROR_SINGULAR


def test_not_converged_reports_the_achieved_error(lib, ctx):
    print("[gpu] refinement without steps", flush=True)
    w = workload("exp3d_4096", EXP3D_4096)
    H = lib.Matrix(ctx, w["blob"])
    F = lib.Factor(ctx, H, w["spec"]["tol"], lib.H2_PREC_FP32)
    X, rep = lib.solve_ir(ctx, H, F, _cuda(w["B"]), target=1e-12, max_outer=0)
    assert not rep["converged"] and rep["max_bkwd"] > 1e-12


@pytest.mark.parametrize("allocator", ["pool", "torch"])
def test_allocators_agree(lib, allocator):
    """The pool allocator and torch's caching allocator back the same
    computation: identical results bit for bit."""
    print(f"[gpu] allocator {allocator}", flush=True)
    w = workload("exp3d_4096", EXP3D_4096)
    c = lib.Context(0, allocator=allocator)
    H = lib.Matrix(c, w["blob"])
    F = lib.Factor(c, H, w["spec"]["tol"])
    X = F.solve(_cuda(w["B"])).cpu().numpy()
    ref = lib.Context(0)
    Hr = lib.Matrix(ref, w["blob"])
    Xr = lib.Factor(ref, Hr, w["spec"]["tol"]).solve(_cuda(w["B"])).cpu().numpy()
    assert np.array_equal(X, Xr)
