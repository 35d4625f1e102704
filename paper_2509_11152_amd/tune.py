"""Leaf-size choice for a family of systems, such as the batched configuration's
instances.

The leaf size m sets how work splits between the dense leaf blocks and the
skeletonization levels. A small m gives more, cheaper levels; a large m gives
fewer levels with larger dense blocks. Which is faster depends on the kernel,
the tolerance and the device. `choose_leaf` times factor + solve of one
representative system at each candidate leaf size on the device and returns
the fastest. Building the system is the caller's: `build(leaf)` returns the
serialized matrix and right-hand sides at that leaf size.
"""
import time

from . import H2_PREC_FP64, Factor, Matrix


def choose_leaf(ctx, build, tol, candidates=(32, 64, 128), prec=H2_PREC_FP64, reps=2):
    """Return (best_leaf, {leaf: seconds}): the median over `reps` timed
    factor + solve runs (after one untimed run) of the system `build(leaf)`
    returns, for each candidate leaf size."""
    import torch

    times = {}
    for leaf in candidates:
        blob, B = build(leaf)
        H = Matrix(ctx, blob)
        Bt = torch.as_tensor(B, dtype=torch.float64).cuda()
        runs = []
        for rep in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F = Factor(ctx, H, tol, prec)
            F.solve(Bt)
            torch.cuda.synchronize()
            if rep > 0:
                runs.append(time.perf_counter() - t0)
            del F
        del H
        runs.sort()
        times[leaf] = runs[len(runs) // 2]
    best = min(times, key=lambda k: (times[k], k))
    return best, times
