"""Host logic of the benchmark line: per-phase roofline classification and the
HBM traffic lookup from the committed PMC summary (no GPU needed)."""
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _stats(ms, flops, bytes_, launches):
    n = len(bench.PHASES)
    pad = lambda v: list(v) + [0.0] * (n + 2 - len(v))
    return {"time_ms": pad(ms), "phase_flops": pad(flops), "phase_bytes": pad(bytes_),
            "launches": pad(launches)}


def test_roofline_picks_the_longest_phase_and_its_bound():
    # fill_row_qr 10 ms (FP32: Gram matrices on FP64 MFMA; FP64: Householder
    # on the ALU), augment 5 ms, project 30 ms with high intensity (MFMA),
    # schur 40 ms with low intensity (HBM)
    ms = [10, 5, 30, 0, 0, 40, 0, 0]
    fl = [1e12, 1e10, 3e14, 0, 0, 1e9, 0, 0]
    by = [1e9, 1e8, 1e9, 0, 0, 2e11, 0, 0]
    nl = [10, 2, 6, 0, 0, 4, 0, 0]
    roof, phases = bench.roofline(_stats(ms, fl, by, nl), "f32")
    assert roof["phase"] == "schur" and roof["bound"] == "hbm"
    assert abs(roof["achieved"] - 2e11 / 0.040 / 1e9) < 1e-6
    assert abs(roof["frac"] - roof["achieved"] / bench.HBM_PEAK) < 1e-12
    assert roof["ms_per_launch"] == 10.0
    assert phases["fill_row_qr"]["bound"] == "mfma"
    assert phases["fill_row_qr"]["peak"] == bench.PEAK["f64"]
    assert phases["augment"]["bound"] == "alu"
    assert phases["project"]["bound"] == "mfma"
    assert phases["project"]["peak"] == bench.PEAK["f32"]
    assert "lu" not in phases  # no time, no work: not reported
    _, p64 = bench.roofline(_stats(ms, fl, by, nl), "f64")
    assert p64["fill_row_qr"]["bound"] == "alu" and p64["fill_row_qr"]["kernel"] == "k_rfactor"


def test_traffic_lookup_requires_workload_phase_and_source_hash():
    assert bench.measured_traffic("no_such_workload", "augment") is None
    assert bench.measured_traffic("laplace3d_1048576", "project") is None
    path = os.path.join(ROOT, "profiles", "pmc_traffic_laplace3d_1048576.md")
    rec = json.loads(re.search(r"```json\n(.*?)\n```", open(path).read(), re.S).group(1))
    src = os.path.join(ROOT, "paper_2509_11152_amd", "csrc", "h2_kernels.hip")
    current = hashlib.sha256(open(src, "rb").read()).hexdigest() == rec["kernel_source_sha256"]
    for phase, kernel in bench.PMC_KERNEL.items():
        t = bench.measured_traffic("laplace3d_1048576", phase)
        if current:
            assert t == rec["kernels"][kernel]["traffic_bytes_per_launch"] and t > 0
        else:
            assert t is None


def test_loglog_slope_of_power_laws():
    import bench

    Ns = [2 ** 16, 2 ** 17, 2 ** 18, 2 ** 19, 2 ** 20]
    assert abs(bench.loglog_slope(Ns, [3e-6 * n for n in Ns]) - 1.0) < 1e-12
    assert abs(bench.loglog_slope(Ns, [n ** 1.5 for n in Ns]) - 1.5) < 1e-12
    assert set(bench.SWEEPS) == {"laplace2d", "laplace3d"}
