"""The allocation-free product h2_matvec_noalloc, called through the C ABI,
against h2_matvec: two calls in a row (the second on a smaller input) give
the same products to the product's tolerance, neither call takes device
memory from the context's allocator, and an input whose work arrays exceed
the static scratch is refused with H2_ERROR_UNSUPPORTED."""
import ctypes

import numpy as np
import pytest

from conftest import workload

pytestmark = pytest.mark.gpu

H2_ERROR_UNSUPPORTED = 8


@pytest.fixture(scope="module")
def lib():
    import torch

    assert torch.cuda.is_available()
    import paper_2509_11152_amd as h2

    return h2


def _call(h2, ctx, H, X, Y):
    """h2_matvec_noalloc on column-major (nrhs, N) device buffers."""
    P = ctypes.c_void_p
    return h2.lib.h2_matvec_noalloc(ctx.ptr, H.ptr, P(X.data_ptr()), H.n, X.shape[0],
                                    P(Y.data_ptr()), H.n)


def test_noalloc_product_matches_h2_matvec(lib):
    import torch

    ctx = lib.Context(0)
    cases = [("exp2d_4096", 5), ("exp2d_1024", 2)]  # the second call's input is smaller
    for name, nrhs in cases:
        print(f"[gpu] allocation-free product {name} nrhs {nrhs}", flush=True)
        H = lib.Matrix(ctx, workload(name)["blob"])
        X = torch.tensor(np.random.default_rng(nrhs).standard_normal((nrhs, H.n)),
                         dtype=torch.float64, device="cuda")
        Y = torch.full_like(X, float("nan"))
        Yref = H.matvec(X.t()).t().contiguous()
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        assert _call(lib, ctx, H, X, Y) == 0, lib.lib.h2_last_error(ctx.ptr)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        err = float(torch.linalg.norm(Y - Yref) / torch.linalg.norm(Yref))
        print(f"[gpu] {name}: |Y - Y_matvec| / |Y_matvec| = {err:.2e}", flush=True)
        assert err <= 1e-13


def test_noalloc_product_refuses_oversized_work(lib):
    import torch

    ctx = lib.Context(0)
    H = lib.Matrix(ctx, workload("exp2d_1024")["blob"])
    nrhs = 4200  # 8 * 2 N * nrhs alone exceeds the 64 MiB scratch
    X = torch.zeros((nrhs, H.n), dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    print("[gpu] allocation-free product beyond its scratch", flush=True)
    assert _call(lib, ctx, H, X, Y) == H2_ERROR_UNSUPPORTED
    assert b"scratch" in lib.lib.h2_last_error(ctx.ptr)
