"""Oracle GMRES-based iterative refinement (FP64).

TEST INFRASTRUCTURE ONLY.

Three-precision GMRES-IR in the form of Carson and Higham (SIAM J. Sci.
Comput. 2018): x0 = M^{-1} b with the factorization as M; then repeat
r = b - A x, stop when ||r|| / ||b|| <= target, solve A d = r by GMRES
left-preconditioned with M^{-1}, x = x + d.  Here every step is FP64; the
loop logic is what the oracle pins.
"""
import numpy as np

from . import factor as of
from . import h2ops


def gmres_left(apply_A, apply_M, r, restart=30, rtol=1e-8):
    """GMRES(restart) on M^{-1} A d = M^{-1} r from d = 0, one cycle."""
    z = apply_M(r)
    beta = np.linalg.norm(z)
    n = r.shape[0]
    if beta == 0.0:
        return np.zeros(n), 0
    V = np.zeros((n, restart + 1))
    Hh = np.zeros((restart + 1, restart))
    V[:, 0] = z / beta
    g = np.zeros(restart + 1)
    g[0] = beta
    cs = np.zeros(restart)
    sn = np.zeros(restart)
    k_done = 0
    for k in range(restart):
        w = apply_M(apply_A(V[:, k]))
        for i in range(k + 1):  # modified Gram-Schmidt
            Hh[i, k] = V[:, i] @ w
            w = w - Hh[i, k] * V[:, i]
        Hh[k + 1, k] = np.linalg.norm(w)
        if Hh[k + 1, k] > 0:
            V[:, k + 1] = w / Hh[k + 1, k]
        for i in range(k):  # previous Givens rotations
            a, b = Hh[i, k], Hh[i + 1, k]
            Hh[i, k] = cs[i] * a + sn[i] * b
            Hh[i + 1, k] = -sn[i] * a + cs[i] * b
        a, b = Hh[k, k], Hh[k + 1, k]
        den = np.hypot(a, b)
        cs[k], sn[k] = (1.0, 0.0) if den == 0 else (a / den, b / den)
        Hh[k, k] = cs[k] * a + sn[k] * b
        Hh[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        k_done = k + 1
        if abs(g[k + 1]) <= rtol * beta or Hh[k + 1, k] == 0 and den == 0:
            break
    y = np.zeros(k_done)
    for i in range(k_done - 1, -1, -1):
        y[i] = (g[i] - Hh[i, i + 1:k_done] @ y[i + 1:]) / Hh[i, i]
    return V[:, :k_done] @ y, k_done


def gmres_ir(H, Fz, B, target=1e-12, restart=30, max_outer=20, inner_rtol=1e-8):
    """Refine X = M^{-1} B column by column until e_b <= target."""
    B = np.asarray(B, dtype=np.float64).reshape(H.N, -1)
    X = of.solve(Fz, B)
    apply_A = lambda v: h2ops.matvec(H, v)
    apply_M = lambda v: of.solve(Fz, v)
    iters = []
    eb = []
    for j in range(B.shape[1]):
        b = B[:, j]
        x = X[:, j].copy()
        nb = np.linalg.norm(b)
        it = 0
        for _ in range(max_outer):
            r = b - apply_A(x)
            e = np.linalg.norm(r) / nb
            if e <= target:
                break
            d, k = gmres_left(apply_A, apply_M, r, restart, inner_rtol)
            it += k
            x = x + d
        else:
            e = np.linalg.norm(b - apply_A(x)) / nb
        X[:, j] = x
        iters.append(it)
        eb.append(e)
    return X, np.array(eb), iters
