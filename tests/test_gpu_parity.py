"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Integer outputs (per-level sizes, augmented ranks, colours, fill pattern,
order of the dense top block) must be identical; FP64 products and solutions
must agree to the stated tolerances; the FP32 factor with FP64 GMRES-IR must
reach a backward error of 1e-12 measured with the oracle's FP64 product.
"""
import numpy as np
import pytest

from conftest import (EXP3D_4096, GAUSS_L32, GAUSS_L128, NOFAR_256, oracle_factor, oracle_matrix,
                      workload)

pytestmark = pytest.mark.gpu

CASES = [
    ("exp2d_1024", None),
    ("exp2d_4096", None),
    ("exp3d_4096", EXP3D_4096),
    ("nofar_256", NOFAR_256),
    ("gauss2d_3000", None),
    ("gauss2d_leaf32", GAUSS_L32),
    ("gauss2d_leaf128", GAUSS_L128),
    # the scale workload's regularised 3D Laplace kernel at a size the oracle factors in seconds
    ("laplace3d_8192", None),
    # the 2D Laplace volume integral equation on its uniform grid (Section 3.1)
    ("laplace2d_4096", None),
]


@pytest.fixture(scope="module")
def lib():
    import torch

    assert torch.cuda.is_available()
    import paper_2509_11152_amd as h2

    return h2


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


_MATS = {}


def gpu_matrix(lib, ctx, name, spec):
    if name not in _MATS:
        _MATS[name] = lib.Matrix(ctx, workload(name, spec)["blob"])
    return _MATS[name]


def _cuda(a):
    import torch

    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name,spec", CASES)
def test_matvec(lib, ctx, name, spec):
    from oracle import h2ops

    print(f"[gpu] matvec {name}", flush=True)
    H = gpu_matrix(lib, ctx, name, spec)
    Ho = oracle_matrix(name, spec)
    X = np.random.default_rng(3).standard_normal((Ho.N, 5))
    Y = H.matvec(_cuda(X)).cpu().numpy()
    Yo = h2ops.matvec(Ho, X)
    assert np.linalg.norm(Y - Yo) <= 1e-13 * np.linalg.norm(Yo)


@pytest.mark.parametrize("name,spec", CASES)
def test_factor_integer_outputs(lib, ctx, name, spec):
    from oracle import factor as of

    print(f"[gpu] factor integers {name}", flush=True)
    H = gpu_matrix(lib, ctx, name, spec)
    tol = workload(name, spec)["spec"]["tol"]
    F = lib.Factor(ctx, H, tol, keep_owner_lists=True)
    Fo = oracle_factor(name, spec=spec)
    assert F.levels() == [Lf.level for Lf in Fo.levels]
    for Lf in Fo.levels:
        lev = Lf.level
        assert F.ints(lev, lib.INT_SIZES).tolist() == [Lf.n[q] for q in Lf.nodes]
        assert F.ints(lev, lib.INT_COLORS).tolist() == [Lf.color[q] for q in Lf.nodes]
        fill = F.ints(lev, lib.INT_FILL).reshape(-1, 2)
        assert [tuple(x) for x in fill.tolist()] == Lf.fpat
        assert F.ints(lev, lib.INT_RANKS).tolist() == [Lf.kt[q] for q in Lf.nodes]
        # Section 2.2's layout (prefix sums of block dimension products) and
        # the per-colour Schur target lists
        lay = F.ints(lev, lib.INT_OFFSETS).reshape(-1, 4)
        assert [tuple(x) for x in lay.tolist()] == of.block_layout(Lf)
        assert F.ints(lev, lib.INT_CLUSTER_OFFSETS).tolist() == of.cluster_offsets(Lf)
        assert F.ints(lev, lib.INT_OWNERS).tolist() == of.owner_records(Lf)
    assert int(F.ints(0, lib.INT_NTOP)[0]) == Fo.n_top


@pytest.mark.parametrize("name,spec", CASES)
def test_solve_fp64(lib, ctx, name, spec):
    from oracle import factor as of
    from oracle import h2ops

    print(f"[gpu] solve fp64 {name}", flush=True)
    w = workload(name, spec)
    H = gpu_matrix(lib, ctx, name, spec)
    Ho = oracle_matrix(name, spec)
    F = lib.Factor(ctx, H, w["spec"]["tol"])
    B = w["B"]
    X = F.solve(_cuda(B)).cpu().numpy()
    Xo = of.solve(oracle_factor(name, spec=spec), B)
    rel = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    res = np.linalg.norm(h2ops.matvec(Ho, X - Xo)) / np.linalg.norm(B)
    ew = np.abs(X - Xo).max() / np.abs(Xo).max()
    print(f"[gpu] {name}: |X - Xo| / |Xo| = {rel:.3e}, |A (X - Xo)| / |B| = {res:.3e}, "
          f"max |X - Xo| / max |Xo| = {ew:.3e}", flush=True)
    assert rel <= 1e-10 and res <= 1e-10 and ew <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_right_hand_sides(lib, ctx, prec):
    """40 right-hand sides (products tiled over three 16-column tiles, several
    columns per wave in the triangular solves): solve and product against the
    oracle column by column."""
    from oracle import factor as of
    from oracle import h2ops

    name, spec = "exp3d_4096", EXP3D_4096
    print(f"[gpu] 40 right-hand sides {prec} {name}", flush=True)
    w = workload(name, spec)
    H = gpu_matrix(lib, ctx, name, spec)
    Ho = oracle_matrix(name, spec)
    B = np.random.default_rng(40).standard_normal((Ho.N, 40))
    Y = H.matvec(_cuda(B)).cpu().numpy()
    Yo = h2ops.matvec(Ho, B)
    assert np.linalg.norm(Y - Yo) <= 1e-13 * np.linalg.norm(Yo)
    if prec == "fp64":
        X = lib.Factor(ctx, H, w["spec"]["tol"]).solve(_cuda(B)).cpu().numpy()
        Xo = of.solve(oracle_factor(name, spec=spec), B)
        ew = np.abs(X - Xo).max() / np.abs(Xo).max()
        rel = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
        assert rel.max() <= 1e-10 and ew <= 1e-10, (rel.max(), ew)
    else:
        F32 = lib.Factor(ctx, H, w["spec"]["tol"], lib.H2_PREC_FP32)
        X, rep = lib.solve_ir(ctx, H, F32, _cuda(B), target=1e-12)
        eb = h2ops.backward_error(Ho, X.cpu().numpy(), B)
        assert rep["converged"] and eb.max() <= 1e-12, (rep, eb.max())


# LDS budgets (KiB) below the default 150: at 8 KiB every fill-row QR, augmentation, LU of
# D_RR and multiplier solve of order above ~40 (FP64) runs its global-memory variant; at
# 48 KiB the launches mix both variants (orders up to ~110 in LDS, larger ones in global
# memory)
@pytest.mark.parametrize("lds_kib", [8, 48])
@pytest.mark.parametrize("name,spec", [("exp2d_4096", None), ("exp3d_4096", EXP3D_4096)])
def test_global_memory_variants(lib, ctx, name, spec, lds_kib):
    """The kernels' global-memory variants (taken by large clusters) give the
    oracle's ranks and solution like the on-chip ones."""
    from oracle import factor as of
    from oracle import h2ops

    print(f"[gpu] global-memory variants (LDS {lds_kib} KiB) {name}", flush=True)
    w = workload(name, spec)
    H = gpu_matrix(lib, ctx, name, spec)
    Fo = oracle_factor(name, spec=spec)
    F = lib.Factor(ctx, H, w["spec"]["tol"], lds_limit_kib=lds_kib)
    for Lf in Fo.levels:
        assert F.ints(Lf.level, lib.INT_RANKS).tolist() == [Lf.kt[q] for q in Lf.nodes]
    B = w["B"]
    X = F.solve(_cuda(B)).cpu().numpy()
    Xo = of.solve(Fo, B)
    rel = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    res = np.linalg.norm(h2ops.matvec(oracle_matrix(name, spec), X - Xo)) / np.linalg.norm(B)
    ew = np.abs(X - Xo).max() / np.abs(Xo).max()
    print(f"[gpu] {name} LDS {lds_kib} KiB: rel {rel:.3e} res {res:.3e} elementwise {ew:.3e}",
          flush=True)
    assert rel <= 1e-10 and res <= 1e-10 and ew <= 1e-10
    # FP32 storage through the same variants still refines to 1e-12
    F32 = lib.Factor(ctx, H, w["spec"]["tol"], lib.H2_PREC_FP32_QR, lds_limit_kib=lds_kib)
    X32, rep = lib.solve_ir(ctx, H, F32, _cuda(B), target=1e-12)
    eb = h2ops.backward_error(oracle_matrix(name, spec), X32.cpu().numpy(), B)
    assert rep["converged"] and eb.max() <= 1e-12, (rep, eb)


@pytest.mark.parametrize("name,spec", [("exp2d_4096", None), ("exp3d_4096", EXP3D_4096),
                                       ("laplace3d_8192", None), ("laplace2d_4096", None)])
@pytest.mark.parametrize("mode", ["chol", "qr", "gram"])
def test_fp32_factor_with_fp64_refinement(lib, ctx, name, spec, mode):
    from oracle import h2ops

    print(f"[gpu] fp32 ({mode} augmentation) + GMRES-IR {name}", flush=True)
    w = workload(name, spec)
    H = gpu_matrix(lib, ctx, name, spec)
    Ho = oracle_matrix(name, spec)
    prec = {"chol": lib.H2_PREC_FP32, "qr": lib.H2_PREC_FP32_QR, "gram": lib.H2_PREC_FP32_GRAM}[mode]
    F32 = lib.Factor(ctx, H, w["spec"]["tol"], prec)
    X, rep = lib.solve_ir(ctx, H, F32, _cuda(w["B"]), target=1e-12)
    X = X.cpu().numpy()
    eb = h2ops.backward_error(Ho, X, w["B"])
    assert rep["converged"] and eb.max() <= 1e-12, (rep, eb)


def test_batched_equals_single(lib, ctx):
    print("[gpu] batched factor/solve", flush=True)
    names = [("exp2d_1024", None), ("exp3d_4096", EXP3D_4096), ("gauss2d_3000", None)]
    Hs = [gpu_matrix(lib, ctx, n, s) for n, s in names]
    tol = 1e-8
    Fb = lib.factor_batched(ctx, Hs, tol)
    Bs = [_cuda(workload(n, s)["B"][:, :2]) for n, s in names]
    Xb = lib.solve_batched(ctx, Fb, Bs)
    for (n, s), H, F, B, X in zip(names, Hs, Fb, Bs, Xb):
        Fs = lib.Factor(ctx, H, tol)
        Xs = Fs.solve(B)
        for lev in Fs.levels():
            assert (F.ints(lev, lib.INT_RANKS) == Fs.ints(lev, lib.INT_RANKS)).all()
        assert np.array_equal(X.cpu().numpy(), Xs.cpu().numpy()), n


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_graph_replays_match_eager(lib, ctx, prec):
    """Solves after the first with one factor launch the recorded plan as one
    HIP graph.  Every replay, with eager work and synchronisations in between,
    equals the first (launch-by-launch) solve bit for bit; the graph reads the
    new input (2B gives exactly 2X, the solve being linear and the scaling
    exact); the unrecorded multi-factor path gives the same bits."""
    name, spec = "exp3d_4096", EXP3D_4096
    print(f"[gpu] solve graph replays {prec} {name}", flush=True)
    w = workload(name, spec)
    H = gpu_matrix(lib, ctx, name, spec)
    p = lib.H2_PREC_FP64 if prec == "fp64" else lib.H2_PREC_FP32
    F = lib.Factor(ctx, H, w["spec"]["tol"], p)
    B = _cuda(w["B"][:, :2])
    X0 = F.solve(B).cpu().numpy()
    for rep in range(3):
        X = F.solve(B).cpu().numpy()
        assert np.array_equal(X, X0), rep
        H.matvec(B)
        ctx.sync()
    X2 = F.solve(2 * B).cpu().numpy()
    assert np.array_equal(X2, 2 * X0)
    st = F.stats()
    # five solves through the recorded plan, every one after the first as a
    # single graph launch
    assert st["solves"] == 5 and st["solve_graph_launches"] == 4, st
    Xd = lib.solve_batched(ctx, [F, F], [B, B])
    assert np.array_equal(Xd[0].cpu().numpy(), X0)
    assert np.array_equal(Xd[1].cpu().numpy(), X0)


def test_choose_leaf_returns_the_fastest_candidate(lib, ctx):
    """The leaf-size choice times every candidate and returns the fastest."""
    from h2gen import workloads

    from paper_2509_11152_amd import tune
    print("[gpu] leaf choice", flush=True)

    def build(leaf):
        w = workloads.make(workloads.batch_workload(0, 2500, leaf=leaf))
        return w["blob"], w["B"][:, :2]

    best, times = tune.choose_leaf(ctx, build, 1e-8, candidates=(32, 64), reps=1)
    assert set(times) == {32, 64}
    assert all(t > 0 for t in times.values())
    assert best == min(times, key=lambda k: (times[k], k))
