"""hp-multigrid V-cycle for the SIPDG Poisson matrix (Sec. 6.4).

The paper coarsens the polynomial degree q down to 1 and then coarsens the
mesh geometrically along a nested hierarchy; smoother, transfers, coarse
operators and coarsest solver are not stated.  Readings used here:

* degree sequence p -> p//2 -> ... -> 1 (4 -> 2 -> 1, 3 -> 1), then halve the
  element count at p = 1 while every axis count is even, until the coarsest
  level has at most ``max_coarse_nodes`` nodes per axis or ``n_levels`` is met;
* every level is the SIPDG matrix rediscretised at its own (p, h, sigma);
* prolongation P is nodal interpolation of the coarse polynomial at the fine
  nodes (degree step: same element; mesh step: parent element), R = P^T;
* smoother: Chebyshev acceleration of Jacobi, D = diag(A), of ``degree`` steps
  (``degree_h`` on the degree-1 levels below the finest, the mesh-coarsening
  part of the hierarchy) on [lam_hi/ratio, lam_hi] with lam_hi = safety * (largest Ritz value of
  D^{-1/2} A D^{-1/2} after ``lanczos_steps`` Lanczos steps); the same
  polynomial before and after the coarse correction, so V is symmetric;
* coarsest level: exact fast-diagonalisation solve.

Test infrastructure only; see the package docstring.
"""
import numpy as np

from . import nodes as _nodes
from . import sipdg as _sipdg
from .fdm import FDM
from .layout import to_global


def hierarchy(E, p, n_levels=None, max_coarse_nodes=16):
    """List of (E3, p) from fine to coarse."""
    levels = [(tuple(E), p)]
    while True:
        Ec, pc = levels[-1]
        if n_levels is not None and len(levels) >= n_levels:
            break
        if pc > 1:
            levels.append((Ec, pc // 2))
            continue
        if n_levels is None and max(Ec) * (pc + 1) <= max_coarse_nodes:
            break
        if any(e % 2 for e in Ec):
            if n_levels is not None:
                raise ValueError("cannot build the requested number of levels")
            break
        levels.append((tuple(e // 2 for e in Ec), 1))
    return levels


def prolongation_1d(fine, coarse):
    """1D interpolation matrix from a coarse Axis1D to a fine Axis1D."""
    nf, nc = fine.n, coarse.n
    P = np.zeros((fine.N, coarse.N))
    if fine.E == coarse.E:
        I = _nodes.lagrange_eval(coarse.xi, fine.xi)
        for e in range(fine.E):
            P[e * nf:(e + 1) * nf, e * nc:(e + 1) * nc] = I
    elif fine.E == 2 * coarse.E:
        for ef in range(fine.E):
            ec, c = divmod(ef, 2)
            I = _nodes.lagrange_eval(coarse.xi, (fine.xi + 2 * c - 1) / 2.0)
            P[ef * nf:(ef + 1) * nf, ec * nc:(ec + 1) * nc] = I
    else:
        raise ValueError("levels are not nested")
    return P


def hash_vector(n_total):
    """Deterministic start vector: v[idx] = ((idx*2654435761 + 12345) mod 2^32)/2^32 - 1/2.

    ``idx`` is the element-major storage index.
    """
    idx = np.arange(n_total, dtype=np.uint64)
    h = (idx * np.uint64(2654435761) + np.uint64(12345)) & np.uint64(0xFFFFFFFF)
    return h.astype(np.float64) / 4294967296.0 - 0.5


def lanczos_max(apply_sym, v0, steps):
    """Largest Ritz value of a symmetric operator after ``steps`` Lanczos steps."""
    v = v0 / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for k in range(steps):
        w = apply_sym(v) - beta * v_prev
        alpha = float(np.vdot(w, v))
        w = w - alpha * v
        alphas.append(alpha)
        beta = float(np.linalg.norm(w))
        if k == steps - 1 or beta == 0.0:
            break
        betas.append(beta)
        v_prev, v = v, w / beta
    T = np.diag(alphas) + np.diag(betas[:len(alphas) - 1], 1) + np.diag(betas[:len(alphas) - 1], -1)
    return float(np.linalg.eigvalsh(T).max())


class Level:
    def __init__(self, E, p, lo, hi, eps=_sipdg.PENALTY_EPS, family="gll"):
        self.E, self.p, self.n = tuple(E), p, p + 1
        self.axes = _sipdg.make_axes(E, p, lo, hi, eps, family)
        self.D = _sipdg.diagonal(self.axes)
        self.shape = self.D.shape

    def A(self, u):
        return _sipdg.apply(self.axes, u)


class Hierarchy:
    """Levels, transfers, smoother parameters and the V-cycle."""

    def __init__(self, E, p, lo, hi, n_levels=None, degree=6, ratio=60.0, safety=1.1,
                 lanczos_steps=30, max_coarse_nodes=16, eps=_sipdg.PENALTY_EPS, degree_h=10, family="gll"):
        self.specs = hierarchy(E, p, n_levels, max_coarse_nodes)
        self.levels = [Level(Es, ps, lo, hi, eps, family) for Es, ps in self.specs]
        self.P = []
        for lf, lc in zip(self.levels[:-1], self.levels[1:]):
            self.P.append([prolongation_1d(lf.axes[d], lc.axes[d]) for d in range(3)])
        self.degree = degree
        self.degrees = [degree_h if (l >= 1 and ps == 1 and degree_h > 0) else degree
                        for l, (_, ps) in enumerate(self.specs)]
        self.coarse = FDM(self.levels[-1].axes)
        self.lam = []
        for L in self.levels[:-1]:
            v0 = to_global(hash_vector(L.D.size), L.E, L.n)
            dm = 1.0 / np.sqrt(L.D)
            lmax = lanczos_max(lambda v: dm * L.A(dm * v), v0, min(lanczos_steps, L.D.size))
            hi_ = safety * lmax
            self.lam.append((hi_ / ratio, hi_))

    # ---- transfers
    def prolong(self, l, uc):
        Px, Py, Pz = self.P[l]
        return np.einsum("Zc,Yb,Xa,cba->ZYX", Pz, Py, Px, uc, optimize=True)

    def restrict(self, l, rf):
        Px, Py, Pz = self.P[l]
        return np.einsum("Zc,Yb,Xa,ZYX->cba", Pz, Py, Px, rf, optimize=True)

    # ---- smoother: Chebyshev acceleration of Jacobi (Saad, Iterative Methods, Alg. 12.1)
    def chebyshev(self, l, f, z):
        L = self.levels[l]
        lo, hi = self.lam[l]
        theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
        sigma1 = theta / delta
        rho = 1.0 / sigma1
        r = f - L.A(z)
        d = r / L.D / theta
        m = self.degrees[l]
        for k in range(m):
            z = z + d
            if k == m - 1:
                break
            r = r - L.A(d)
            rho_new = 1.0 / (2.0 * sigma1 - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * (r / L.D)
            rho = rho_new
        return z

    def vcycle(self, f, l=0):
        """z = B f, one symmetric V-cycle applied to the residual f on level l."""
        if l == len(self.levels) - 1:
            return self.coarse.solve(f)
        L = self.levels[l]
        z = self.chebyshev(l, f, np.zeros_like(f))
        rc = self.restrict(l, f - L.A(z))
        z = z + self.prolong(l, self.vcycle(rc, l + 1))
        z = self.chebyshev(l, f, z)
        return z
