"""GPU parity at the benchmark's full size: N = 2^20 points in the unit cube,
the regularised 3D Laplace kernel, leaf 64, tol 1e-6, 32 right-hand sides, in
the configuration the benchmark times (FP32 factorization + FP64 GMRES-IR to
a backward error of 1e-12).

The oracle cannot factor this size in reasonable time, so the test checks what
holds at any size, against oracle-side computations where there are any:
- the backward error of the refined solution, recomputed with the oracle's own
  FP64 H^2 product (independent of the HIP path), is at most 1e-12;
- per skeletonized level, every augmented rank lies in [0, n_i];
- the next level's sizes are the sums of the children's augmented ranks (the
  level transition of Section 2.1);
- the colours are proper on the near graph (Algorithm 2's batches);
- the fill pattern is symmetric and disjoint from the near pairs (fill only
  arises at pairs outside the near field).

This file is collected after the parity tests. It builds the matrix on the
device (about 70 s), parses it on the host for the oracle and runs the
oracle's product (a few minutes in all).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_full_size_fp32_ir_properties():
    import torch

    import paper_2509_11152_amd as h2
    from h2gen import workloads
    from oracle import blob as ob
    from oracle import h2ops

    print("[gpu] full size laplace3d_1048576: construct", flush=True)
    spec = workloads.WORKLOADS["laplace3d_1048576"]
    w = workloads.make(spec, device="cuda")
    w.pop("h")
    torch.cuda.empty_cache()
    ctx = h2.Context(0)
    H = h2.Matrix(ctx, w["blob"])
    B = torch.tensor(w["B"], dtype=torch.float64, device="cuda")
    print("[gpu] full size: FP32 factor + GMRES-IR", flush=True)
    F = h2.Factor(ctx, H, spec["tol"], h2.H2_PREC_FP32)
    X, rep = h2.solve_ir(ctx, H, F, B, target=1e-12)
    assert rep["converged"], rep
    Xh = X.cpu().numpy()
    del X, B

    print("[gpu] full size: oracle product", flush=True)
    Ho = ob.parse(w["blob"])
    Bh = np.asarray(w["B"], dtype=np.float64)
    R = Bh - h2ops.matvec(Ho, Xh)
    eb = np.linalg.norm(R, axis=0) / np.linalg.norm(Bh, axis=0)
    assert eb.max() <= 1e-12, eb

    print("[gpu] full size: integer invariants", flush=True)
    lp = Ho.level_ptr
    levels = F.levels()
    assert levels == sorted(levels, reverse=True) and levels[0] == Ho.L
    for idx, lev in enumerate(levels):
        a, b = int(lp[lev]), int(lp[lev + 1])
        n = F.ints(lev, h2.INT_SIZES)
        kt = F.ints(lev, h2.INT_RANKS)
        col = F.ints(lev, h2.INT_COLORS)
        assert len(n) == len(kt) == len(col) == b - a
        assert (kt >= 0).all() and (kt <= n).all()
        near = set()
        for q in range(a, b):
            for j in ob.near(Ho, q):
                near.add((q, int(j)))
                if j != q:
                    assert col[q - a] != col[int(j) - a], (lev, q, int(j))
        fill = {tuple(x) for x in F.ints(lev, h2.INT_FILL).reshape(-1, 2).tolist()}
        assert all((k, j) in fill for (j, k) in fill)
        assert not (fill & near)
        if idx + 1 < len(levels):
            nxt = levels[idx + 1]
            n2 = F.ints(nxt, h2.INT_SIZES)
            for t, tau in enumerate(range(int(lp[nxt]), int(lp[nxt + 1]))):
                s = sum(int(kt[c - a]) for c in ob.children(Ho, tau))
                assert int(n2[t]) == s, (nxt, tau)
