"""Conjugate gradients preconditioned by the hp-multigrid V-cycle (Sec. 6.4).

Textbook PCG (Hestenes-Stiefel): alpha = r.z / p.Ap, x += alpha p,
r -= alpha Ap, z = B r, beta = r_new.z_new / r.z, p = z + beta p.
Stop when ||r||_2 <= rtol ||b||_2 on the recurrence residual; the returned
relative residual is recomputed from b - A x.

Test infrastructure only; see the package docstring.
"""
import numpy as np


def pcg(A, b, B, x0=None, rtol=1e-8, maxit=500):
    """Return (x, iterations, true relative residual, history of ||r||/||b||)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A(x) if x0 is not None else b.copy()
    bnorm = float(np.linalg.norm(b))
    hist = [float(np.linalg.norm(r)) / bnorm]
    it = 0
    if hist[-1] > rtol:
        z = B(r)
        p = z.copy()
        rz = float(np.vdot(r, z))
        while it < maxit:
            q = A(p)
            alpha = rz / float(np.vdot(p, q))
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            hist.append(float(np.linalg.norm(r)) / bnorm)
            if hist[-1] <= rtol:
                break
            z = B(r)
            rz_new = float(np.vdot(r, z))
            p = z + (rz_new / rz) * p
            rz = rz_new
    true_rel = float(np.linalg.norm(b - A(x))) / bnorm
    return x, it, true_rel, hist


def solve(hier, b, x0=None, rtol=1e-8, maxit=500):
    """MG-PCG on the finest level of ``hier`` for b[Z, Y, X]."""
    L = hier.levels[0]
    return pcg(L.A, b, hier.vcycle, x0=x0, rtol=rtol, maxit=maxit)
