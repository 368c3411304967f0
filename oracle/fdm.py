"""Exact solve of the discrete Poisson system by fast diagonalisation.

On a uniform Cartesian mesh the SIPDG matrix is the Kronecker sum
A = A1x(x)Mz(x)My + ... (Sec. 3.5), with diagonal masses.  With
S = M1^{-1/2} and the symmetric eigendecomposition S A1 S = Q Lambda Q^T per
axis,
    A^{-1} = S3 (Qz(x)Qy(x)Qx) diag(1/(lz+ly+lx)) (Qz(x)Qy(x)Qx)^T S3,
S3 = Sz(x)Sy(x)Sx.  This is the exact solution of the linear system the
method's CG iteration approximates (Lynch, Rice & Thomas 1964).

Test infrastructure only; see the package docstring.
"""
import numpy as np


class FDM:
    def __init__(self, axes):
        self.axes = axes
        self.S, self.Q, self.lam = [], [], []
        for a in axes:
            s = 1.0 / np.sqrt(a.m)
            lam, Q = np.linalg.eigh(s[:, None] * a.A * s[None, :])
            self.S.append(s)
            self.Q.append(Q)
            self.lam.append(lam)
        lx, ly, lz = self.lam
        self.denom = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]

    def solve(self, b):
        """u = A^{-1} b for b[Z, Y, X]."""
        sx, sy, sz = self.S
        Qx, Qy, Qz = self.Q
        t = np.asarray(b, dtype=np.float64) * (sz[:, None, None] * sy[None, :, None] * sx[None, None, :])
        t = np.einsum("Xa,zyX->zya", Qx, t, optimize=True)
        t = np.einsum("Yb,zYx->zbx", Qy, t, optimize=True)
        t = np.einsum("Zc,Zyx->cyx", Qz, t, optimize=True)
        t = t / self.denom
        t = np.einsum("Xa,zya->zyX", Qx, t, optimize=True)
        t = np.einsum("Yb,zbx->zYx", Qy, t, optimize=True)
        t = np.einsum("Zc,cyx->Zyx", Qz, t, optimize=True)
        return t * (sz[:, None, None] * sy[None, :, None] * sx[None, None, :])
