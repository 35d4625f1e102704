"""Benchmark of the H^2 strong recursive skeletonization factor + solve on one MI355X.

One step = the whole hot path on one synthetic system: FP32 factorization
(MFMA, FP32 accumulation) followed by FP64 GMRES-IR to a backward error of
1e-12 (the FP64 H^2 product supplies the residuals).  The default workload is
the scale configuration: N = 2^20 points uniform in the unit cube, the
regularised Laplace kernel 1/(4 pi (r + 1e-3)) + I, leaf size 64, tol 1e-6,
32 right-hand sides.  The FP64 path (FP64 factor + the same refinement, and
the plain FP64 factor + one solve) is timed in the same run for comparison.
Inputs are resident in HBM before timing starts; construction of the
synthetic H^2 matrix and its upload are reported under "setup_s", untimed.

The whole run keeps to a wall-clock budget (--budget-s from process start):
warm-up and timed steps stop early when the remaining ones would not fit, and
the line reports the counts that ran ("steps", "warmup") next to the ones
asked for.  The batched configuration (64 independent 2D systems, N_i
log-uniform in [2048, 32768], FP64, leaf size chosen by timing; one batched
factor and one batched solve call) runs when enough budget is left, under
"batched" (work-model GFLOP/s).  The CPU oracle baseline runs in a child
process on the host cores while the device works.  "roofline" gives the
dominant factor kernel's achieved rate and, from the committed PMC summary,
its HBM traffic per launch.

Prints one JSON line.  Only one GPU is used: --gpus > 1 exits with a message.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
T0 = time.perf_counter()

METRIC = "N=2^20 factor+solve s, FP32+IR vs FP64 @ bkwd err 1e-12; batched GFLOP/s"
PEAK = {"f64": 78.6, "f32": 157.3}  # TFLOP/s, dense MFMA
HBM_PEAK = 8000.0  # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="laplace3d_1048576")
    p.add_argument("--budget-s", type=float, default=540.0,
                   help="wall-clock budget of the whole run from process start: warm-up and "
                        "timed steps stop early (the line reports how many ran) when the rest "
                        "would not fit")
    p.add_argument("--reserve-s", type=float, default=90.0,
                   help="part of the budget kept for the FP64 comparison and the report")
    p.add_argument("--batched", action="store_true",
                   help="always run the 64-instance batched measurement")
    p.add_argument("--batched-s", type=float, default=240.0,
                   help="run the batched measurement only when this much budget is left")
    p.add_argument("--no-fp64", action="store_true",
                   help="skip the FP64 comparison (profiling runs)")
    p.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-batched", action="store_true",
                   help="skip the 64-instance batched measurement")
    p.add_argument("--construct-device", default="cuda")
    p.add_argument("--save-blob", default=None,
                   help="after construction, write the serialized matrix and right-hand sides to "
                        "PATH.blob.npy and PATH.rhs.npy")
    p.add_argument("--load-blob", default=None,
                   help="skip construction: read the files --save-blob wrote for this workload")
    p.add_argument("--sweep", default=None, choices=sorted(SWEEPS),
                   help="time and peak device memory over N for a workload family (prints "
                        "one JSON line with the fitted log-log slopes) instead of the bench")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run plain 256 MiB device copies (reference reading for HBM "
                        "byte counters) and print their size")
    return p.parse_args()


def copy_calibration():
    """Plain device-to-device copies of a known size: the FETCH_SIZE and
    WRITE_SIZE counters of these dispatches give the scale factor between
    counter readings and bytes moved."""
    import torch
    n = 1 << 26  # float32 elements = 256 MiB
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": 4 * n, "dispatches": 5,
                      "kernel": "torch elementwise copy"}), flush=True)


# device phases of the factorization (h2_stats indices 0..7) and their kernels
PHASES = ["fill_row_qr", "augment", "project", "lu", "multipliers", "schur", "close_out", "top_lu"]
KERNEL_OF = {"fill_row_qr": "k_rfactor", "augment": "k_augment", "project": "k_strip",
             "lu": "k_lu", "multipliers": "k_trsm_wave + k_trsm",
             "schur": "k_schur_enum + k_schur_apply", "close_out": "k_closeout",
             "top_lu": "k_panel_lu + k_laswp + k_trsm_block + k_gemm"}
# the FP32 factorization reduces a fill row through its FP64 Gram matrix (FP64
# MFMA) and a pivoted Cholesky instead of the Householder QR
KERNEL_OF_F32 = dict(KERNEL_OF, fill_row_qr="k_gram + k_pchol_wave/k_pchol")
# phases whose arithmetic runs on the vector ALU (Householder reductions,
# Jacobi rotations, small LU and triangular solves); the others are priced
# against MFMA or HBM by their algorithmic intensity
ALU_PHASES = {"fill_row_qr", "augment", "lu", "multipliers"}
ALU_PHASES_F32 = {"augment", "lu", "multipliers"}


def roofline(st, dt):
    """Per-phase achieved rate: the library's algorithmic flop and byte counts
    for the phase divided by its device time (HIP events around the phase's
    launches on the library's stream, summed over the factorization).  Each
    phase 0..7 is one kernel, so rate = (work per launch) / (mean launch time)."""
    peak_f = PEAK[dt]
    kernels = KERNEL_OF_F32 if dt == "f32" else KERNEL_OF
    alu = ALU_PHASES_F32 if dt == "f32" else ALU_PHASES
    out = {}
    best = None
    for i, name in enumerate(PHASES):
        t = st["time_ms"][i] * 1e-3
        fl, by, nl = st["phase_flops"][i], st["phase_bytes"][i], st["launches"][i]
        if t <= 0 or (fl <= 0 and by <= 0):
            continue
        # the FP32 fill-row Gram matrices are FP64 MFMA products
        pk = PEAK["f64"] if (dt == "f32" and name == "fill_row_qr") else peak_f
        f_time = fl / (pk * 1e12)
        b_time = by / (HBM_PEAK * 1e9)
        if name in alu:
            bound, ach, peak, unit = "alu", fl / t / 1e12, pk, "TFLOP/s"
        elif f_time >= b_time:
            bound, ach, peak, unit = "mfma", fl / t / 1e12, pk, "TFLOP/s"
        else:
            bound, ach, peak, unit = "hbm", by / t / 1e9, HBM_PEAK, "GB/s"
        out[name] = {"kernel": kernels[name], "ms": t * 1e3, "launches": nl,
                     "ms_per_launch": t * 1e3 / max(nl, 1),
                     "flops": fl, "bytes": by, "bound": bound, "achieved": ach, "peak": peak,
                     "unit": unit, "frac": ach / peak}
        if best is None or t > out[best]["ms"] * 1e-3:
            best = name
    r = out[best]
    roof = {"bound": r["bound"], "achieved": r["achieved"], "peak": r["peak"], "unit": r["unit"],
            "frac": r["frac"], "traffic": None, "kernel": r["kernel"], "phase": best,
            "launches": r["launches"], "ms_per_launch": r["ms_per_launch"]}
    return roof, out


# FP32 kernels of the phases whose HBM traffic the PMC summary records
PMC_KERNEL = {"fill_row_qr": "h2k::k_gram<float>",
              "augment": "h2k::k_augment<float, float, false>",
              "schur": "h2k::k_schur_apply<float>"}


def measured_traffic(workload, phase):
    """HBM bytes per launch of the phase's kernel from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None when
    there is none for this workload and kernel or the kernel source changed since
    the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.md")
    if phase not in PMC_KERNEL or not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    src = os.path.join(ROOT, "paper_2509_11152_amd", "csrc", "h2_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    k = rec.get("kernels", {}).get(PMC_KERNEL[phase])
    if rec.get("workload") != workload or rec.get("kernel_source_sha256") != sha or k is None:
        return None
    return k["traffic_bytes_per_launch"]


def batched_bench(args, h2, ctx):
    """The batched configuration: 64 independent systems, N_i log-uniform in
    [2048, 32768] (2D Gaussian kernel, KD tree, tol 1e-8, 16 RHS each, leaf size
    chosen by paper_2509_11152_amd.tune on the largest instance), factored
    by one h2_factor_batched call and solved by one h2_solve_batched call in
    FP64.  Rate = sum over instances of the work model's (factor + solve) flops
    / wall time of factor + solve (median of the timed repetitions)."""
    import numpy as np
    import torch

    from h2gen import workloads
    from paper_2509_11152_amd import tune
    sizes = workloads.batch_sizes()
    # leaf size: the fastest of 32, 64, 128 on the largest instance (it
    # dominates the batch's time)
    big = int(np.argmax(sizes))
    big_spec = workloads.batch_workload(big, int(sizes[big]))

    def build(leaf):
        w = workloads.make(workloads.batch_workload(big, int(sizes[big]), leaf=leaf),
                           device=args.construct_device)
        return w["blob"], w["B"]

    t0 = time.perf_counter()
    leaf, tune_s = tune.choose_leaf(ctx, build, big_spec["tol"])
    log(f"[bench] batched: leaf {leaf} chosen in {time.perf_counter() - t0:.1f} s "
        f"({', '.join(f'{k}: {v:.3f} s' for k, v in tune_s.items())})")
    t0 = time.perf_counter()
    Hs, Bs, tol = [], [], None
    for i, n in enumerate(sizes):
        spec = workloads.batch_workload(i, int(n), leaf=leaf)
        w = workloads.make(spec, device=args.construct_device)
        Hs.append(h2.Matrix(ctx, w["blob"]))
        Bs.append(torch.tensor(w["B"], dtype=torch.float64, device="cuda"))
        tol = spec["tol"]
        del w
        if i % 8 == 7:
            log(f"[bench] batched: constructed {i + 1} instances ({time.perf_counter() - t0:.1f} s)")
    log(f"[bench] batched: {len(Hs)} instances, sum N = {int(sizes.sum())}, constructed in "
        f"{time.perf_counter() - t0:.1f} s")
    tf, ts = [], []
    Fs = Xs = None
    # one untimed and three timed repetitions (the headline's step counts do
    # not apply to this secondary figure)
    for rep in range(1 + 3):
        Fs = Xs = None
        torch.cuda.synchronize()
        a = time.perf_counter()
        Fs = h2.factor_batched(ctx, Hs, tol, h2.H2_PREC_FP64)
        torch.cuda.synchronize()
        b = time.perf_counter()
        Xs = h2.solve_batched(ctx, Fs, Bs)
        torch.cuda.synchronize()
        c = time.perf_counter()
        if rep >= 1:
            tf.append(b - a)
            ts.append(c - b)
        log(f"[bench] batched rep {rep}: factor {b - a:.3f}s solve {c - b:.3f}s")
    nrhs = Bs[0].shape[1]
    fl_f = sum(F.stats()["factor_flops"] for F in Fs)
    fl_s = sum(F.stats()["solve_flops_per_rhs"] * nrhs for F in Fs)
    eb = 0.0
    for H, B, X in zip(Hs, Bs, Xs):
        R = B - H.matvec(X)
        eb = max(eb, float((torch.linalg.norm(R, dim=0) / torch.linalg.norm(B, dim=0)).max()))
    f, so = float(np.median(tf)), float(np.median(ts))
    return {"instances": len(Hs), "sum_N": int(sizes.sum()), "nrhs": int(nrhs), "tol": tol,
            "dtype": "f64", "factor_s": f, "solve_s": so,
            "gflops": (fl_f + fl_s) / (f + so) / 1e9, "factor_gflops": fl_f / f / 1e9,
            "max_bkwd": eb, "leaf": leaf, "leaf_tuning_s": {str(k): v for k, v in tune_s.items()},
            "workload": "gauss2d batch, 64 x N_i log-uniform in [2048, 32768]"}


def cpu_baseline(spec_name, threads=1):
    """The oracle (numpy FP64) on a bounded sample of the same recipe (same
    kernel, tree, leaf size, tolerance and right-hand sides, fewer points),
    extrapolated linearly in N (the method is O(N) in time), with its BLAS
    limited to `threads` threads."""
    from threadpoolctl import threadpool_limits

    from h2gen import workloads
    from oracle import blob as ob
    from oracle import factor as of
    from oracle import ir as oir

    full = workloads.WORKLOADS[spec_name]
    sample = dict(full)
    sample["N"] = 8192 if full["dim"] == 3 else 16384
    w = workloads.make(sample)
    H = ob.parse(w["blob"])
    with threadpool_limits(threads, user_api="blas"):
        t0 = time.perf_counter()
        Fz = of.factor(H, sample["tol"])
        X, eb, its = oir.gmres_ir(H, Fz, w["B"], target=1e-12)
        dt = time.perf_counter() - t0
    return {
        "value": dt * full["N"] / sample["N"],
        "unit": "s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"oracle FP64 factor + GMRES-IR to 1e-12 at N={sample['N']} (same recipe, "
                  f"{sample['nrhs']} RHS) took {dt:.2f} s with {threads} BLAS thread(s); "
                  f"value = that x N/{sample['N']} (linear complexity)",
    }


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                info["cpu"] = ln.split(":", 1)[1].strip()
                break
        for ln in open("/proc/meminfo"):
            if ln.startswith("MemTotal"):
                info["mem_gb"] = round(int(ln.split()[1]) / 1e6, 1)
                break
    except OSError:
        pass
    return info


def cpu_baseline_main(args):
    """Child process: the oracle baseline at one BLAS thread and at every host
    core, printed as one JSON line."""
    out = {"one_core": cpu_baseline(args.workload, 1)}
    n = os.cpu_count() or 1
    if n > 1:
        out["all_cores"] = cpu_baseline(args.workload, n)
    out["host"] = host_info()
    print(json.dumps(out), flush=True)


def start_cpu_baseline(args):
    """Start the oracle baseline in a child process before this process touches
    the GPU; it runs on the host cores while the device works."""
    import subprocess

    env = dict(os.environ)
    env.setdefault("OMP_NUM_THREADS", str(os.cpu_count() or 1))
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                             "--workload", args.workload], stdout=subprocess.PIPE,
                            stderr=subprocess.DEVNULL, text=True, env=env)


def finish_cpu_baseline(proc, wait_s):
    if proc is None:
        return None
    try:
        out, _ = proc.communicate(timeout=max(wait_s, 1.0))
    except Exception:
        proc.kill()
        proc.communicate()
        return None
    for ln in reversed(out.splitlines()):
        if ln.startswith("{"):
            return json.loads(ln)
    return None


# workload families of the linear-complexity sweep: the recipe and its sizes
SWEEPS = {
    "laplace3d": ("laplace3d_1048576", [2 ** 16, 2 ** 17, 2 ** 18, 2 ** 19, 2 ** 20]),
    "laplace2d": ("laplace2d_262144", [4 ** 7, 4 ** 8, 4 ** 9, 4 ** 10]),
}


def loglog_slope(xs, ys):
    """Least-squares slope of log y against log x."""
    import numpy as np

    return float(np.polyfit(np.log(np.asarray(xs, dtype=np.float64)),
                            np.log(np.asarray(ys, dtype=np.float64)), 1)[0])


def sweep_main(args):
    """Linear time and memory on the device (Section 2.4, Section 3.3): for each
    size of a workload family, the median of two FP32 factorizations and their
    refinements to 1e-12 and one FP64 factorization (each after an untimed run),
    the peak device bytes of both factors and the matrix's bytes; then the
    fitted log-log slopes over N."""
    import numpy as np
    import torch

    import paper_2509_11152_amd as h2
    from h2gen import workloads

    name, sizes = SWEEPS[args.sweep]
    base = workloads.WORKLOADS[name]
    ctx = h2.Context(0)
    rows = []
    for N in sizes:
        spec = dict(base, N=N)
        t0 = time.perf_counter()
        w = workloads.make(spec, device=args.construct_device)
        H = h2.Matrix(ctx, w["blob"])
        B = torch.tensor(w["B"], dtype=torch.float64, device="cuda")
        del w
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        tol = spec["tol"]
        f32, ir32 = [], []
        for rep in range(3):
            torch.cuda.synchronize()
            a = time.perf_counter()
            F = h2.Factor(ctx, H, tol, h2.H2_PREC_FP32)
            torch.cuda.synchronize()
            b = time.perf_counter()
            X, rep_ir = h2.solve_ir(ctx, H, F, B, target=1e-12)
            torch.cuda.synchronize()
            c = time.perf_counter()
            if rep:
                f32.append(b - a)
                ir32.append(c - b)
            s32 = F.stats()
            del F, X
        f64 = []
        for rep in range(2):
            torch.cuda.synchronize()
            a = time.perf_counter()
            F = h2.Factor(ctx, H, tol, h2.H2_PREC_FP64)
            torch.cuda.synchronize()
            f64.append(time.perf_counter() - a)
            s64 = F.stats()
            del F
        row = {"N": N, "build_s": t_build, "fp32_factor_s": float(np.median(f32)),
               "fp32_ir_s": float(np.median(ir32)), "fp64_factor_s": f64[-1],
               "peak_fp32_bytes": s32["peak_bytes"], "peak_fp64_bytes": s64["peak_bytes"],
               "matrix_bytes": H.device_bytes, "ir_converged": bool(rep_ir["converged"]),
               "ir_bkwd": rep_ir["max_bkwd"]}
        rows.append(row)
        log(f"[sweep] {name} N={N}: build {t_build:.1f} s, fp32 factor {row['fp32_factor_s']:.3f} s "
            f"+ IR {row['fp32_ir_s']:.3f} s, fp64 factor {row['fp64_factor_s']:.3f} s, peak "
            f"{row['peak_fp32_bytes'] / 1e9:.2f} / {row['peak_fp64_bytes'] / 1e9:.2f} GB")
        del H, B
        torch.cuda.empty_cache()
    Ns = [r["N"] for r in rows]
    keys = ["fp32_factor_s", "fp32_ir_s", "fp64_factor_s", "peak_fp32_bytes", "peak_fp64_bytes",
            "matrix_bytes"]
    print(json.dumps({"sweep": args.sweep, "workload": name, "rows": rows,
                      "slopes": {k: loglog_slope(Ns, [r[k] for r in rows]) for k in keys}}),
          flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.sweep:
        sweep_main(args)
        return
    if args.cpu_baseline_only:
        cpu_baseline_main(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "described but not built", file=sys.stderr)
        sys.exit(2)
    cpu_proc = None if args.no_cpu_baseline else start_cpu_baseline(args)
    import numpy as np
    import torch

    import paper_2509_11152_amd as h2
    from h2gen import workloads

    def left():
        return args.budget_s - (time.perf_counter() - T0)

    spec = workloads.WORKLOADS[args.workload]
    t0 = time.perf_counter()
    if args.load_blob:
        log(f"[bench] reading {args.load_blob}.blob.npy / .rhs.npy ({args.workload})")
        w = {"blob": np.load(args.load_blob + ".blob.npy", mmap_mode="r"),
             "B": np.load(args.load_blob + ".rhs.npy")}
        if w["B"].shape[0] != spec["N"]:
            raise SystemExit(f"{args.load_blob}: right-hand sides of N={w['B'].shape[0]}, "
                             f"workload {args.workload} has N={spec['N']}")
    else:
        log(f"[bench] constructing {args.workload} (N={spec['N']}) on {args.construct_device}")
        w = workloads.make(spec, device=args.construct_device, verbose=True)
        w.pop("h", None)
        torch.cuda.empty_cache()
        log(f"[bench] construction {time.perf_counter() - t0:.1f} s, blob {w['blob'].nbytes / 1e9:.2f} GB")
        if args.save_blob:
            np.save(args.save_blob + ".blob.npy", w["blob"])
            np.save(args.save_blob + ".rhs.npy", w["B"])
            log(f"[bench] wrote {args.save_blob}.blob.npy / .rhs.npy")
    t_construct = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    ctx = h2.Context(0)
    t0 = time.perf_counter()
    H = h2.Matrix(ctx, w["blob"])
    B = torch.tensor(w["B"], dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    blob_gb = w["blob"].nbytes / 1e9
    del w
    log(f"[bench] load + upload {t_load:.1f} s; {left():.0f} s of the budget left")
    tol = spec["tol"]

    def step32():
        torch.cuda.synchronize()
        a = time.perf_counter()
        F = h2.Factor(ctx, H, tol, h2.H2_PREC_FP32)
        torch.cuda.synchronize()
        b = time.perf_counter()
        X, rep = h2.solve_ir(ctx, H, F, B, target=1e-12)
        torch.cuda.synchronize()
        c = time.perf_counter()
        return F, X, rep, b - a, c - a

    # FP32 factor + FP64 GMRES-IR: warm-up steps (at least one: first-use
    # allocations), then the timed steps; both stop early, and say so, when
    # the remaining steps would not fit in the time budget
    reserve = args.reserve_s
    per = None
    warm = 0
    while warm < max(args.warmup, 1):
        if warm >= 1 and left() - reserve < 2.5 * per:
            break
        log(f"[bench] warmup {warm}")
        a = time.perf_counter()
        F32, X32, rep32, _, _ = step32()
        del F32, X32
        per = time.perf_counter() - a
        warm += 1
    t32, tf32 = [], []
    F32 = X32 = rep32 = None
    for i in range(args.steps):
        if i >= 1 and left() - reserve < 1.5 * max(t32):
            log(f"[bench] time budget: {i} of {args.steps} steps timed")
            break
        F32 = X32 = None
        F32, X32, rep32, tf, tt = step32()
        t32.append(tt)
        tf32.append(tf)
        log(f"[bench] step {i}: fp32+IR {tt:.3f}s (factor {tf:.3f}s); {left():.0f} s left")
    s32 = F32.stats()
    med = lambda v: float(np.median(v)) if v else None

    def bkwd(X):
        R = B - H.matvec(X)
        return float((torch.linalg.norm(R, dim=0) / torch.linalg.norm(B, dim=0)).max())

    eb32 = bkwd(X32)
    del F32, X32
    torch.cuda.empty_cache()
    # the FP64 path: FP64 factor + the same refinement, and the plain FP64
    # factor + one solve (its backward error stated), timed once after an
    # untimed run when the budget allows
    fp64 = {}
    t64 = t64p = tf64 = None
    eb64 = eb64p = None
    s64 = None
    reps64 = 0
    est64 = 2.0 * value_or(med(t32), 1.0)
    for rep in range(0 if args.no_fp64 else 2):
        if rep == 0 and left() - est64 * 2 < 60:
            continue  # no time for an untimed run
        if left() < est64 + 30:
            break
        torch.cuda.synchronize()
        a = time.perf_counter()
        F64 = h2.Factor(ctx, H, tol, h2.H2_PREC_FP64)
        torch.cuda.synchronize()
        d = time.perf_counter()
        X64p = F64.solve(B)
        torch.cuda.synchronize()
        e = time.perf_counter()
        X64, rep64 = h2.solve_ir(ctx, H, F64, B, target=1e-12)
        torch.cuda.synchronize()
        f = time.perf_counter()
        tf64, t64p, t64 = d - a, e - a, (f - e) + (d - a)
        est64 = t64 + t64p - tf64
        reps64 = rep + 1
        eb64, eb64p = bkwd(X64), bkwd(X64p)
        s64 = F64.stats()
        fp64 = {"ir": rep64}
        # the allocator keeps the freed blocks for the next run (as in the
        # FP32 steps); the first run, when there is time for two, warms it
        del F64, X64, X64p
        log(f"[bench] fp64 run {rep}: fp64+IR {t64:.3f}s plain fp64 {t64p:.3f}s; {left():.0f} s left")
    torch.cuda.empty_cache()
    value = med(t32)
    roof, phases = roofline(s32, "f32")
    roof["traffic"] = measured_traffic(args.workload, roof["phase"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": len(t32),
        "warmup": warm,
        "ms_per_step": value * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "N": spec["N"], "dim": spec["dim"], "kernel": list(spec["kernel"]), "tree": spec["tree"],
            "leaf": spec["leaf"], "tol": tol, "nrhs": spec["nrhs"], "eta": spec["eta"],
            "p0": spec["p0"],
        },
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "setup_s": {"construct": t_construct, "load_upload": t_load, "blob_gb": blob_gb},
        "fp32_ir": {"factor_s": med(tf32), "total_s": value, "bkwd": eb32, "ir": rep32,
                    "factor_gflops": s32["factor_flops"] / med(tf32) / 1e9,
                    "phase_ms": dict(zip(h2.PHASES, s32["time_ms"])),
                    "peak_bytes": s32["peak_bytes"], "matrix_bytes": H.device_bytes},
        "n_top": s32["n_top"],
        "roofline": roof,
        "phases_fp32": phases,
    }
    if s64 is not None:
        _, phases64 = roofline(s64, "f64")
        out["fp64_ir"] = {"factor_s": tf64, "total_s": t64, "bkwd": eb64, "ir": fp64["ir"],
                          "runs": reps64, "phase_ms": dict(zip(h2.PHASES, s64["time_ms"])),
                          "peak_bytes": s64["peak_bytes"]}
        out["fp64_plain"] = {"total_s": t64p, "bkwd": eb64p}
        out["phases_fp64"] = phases64
    else:
        out["fp64_ir"] = {"skipped": "not asked for" if args.no_fp64 else "time budget"}
    if args.batched or (not args.no_batched and left() > args.batched_s):
        del H, B
        torch.cuda.empty_cache()
        out["batched"] = batched_bench(args, h2, ctx)
    else:
        out["batched"] = {"skipped": f"time budget ({left():.0f} s left, the batched leg needs "
                                     f"about {args.batched_s:.0f} s)"}
    cb = finish_cpu_baseline(cpu_proc, min(left(), 120.0))
    if cb is not None:
        best = cb.get("all_cores") if cb.get("all_cores", {}).get("value", 1e300) < \
            cb["one_core"]["value"] else cb["one_core"]
        out["cpu_baseline"] = dict(best)
        out["cpu_baseline"]["one_core_value"] = cb["one_core"]["value"]
        if "all_cores" in cb:
            out["cpu_baseline"]["all_cores_value"] = cb["all_cores"]["value"]
        out["cpu_baseline"]["host"] = cb.get("host")
    print(json.dumps(out), flush=True)


def value_or(v, d):
    return d if v is None else v


if __name__ == "__main__":
    main()
