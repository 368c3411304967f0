"""Closed forms for s-type Gaussians: orbitals, densities, potentials, energies.

* Normalised primitive chi_a(r) = (2 a/pi)^{3/4} exp(-a |r - A|^2).
* Gaussian product theorem: exp(-a|r-A|^2) exp(-b|r-B|^2)
  = exp(-a b |A-B|^2/(a+b)) exp(-(a+b)|r-P|^2), P = (a A + b B)/(a+b).
* Potential of exp(-c|r-P|^2): (pi/c)^{3/2} erf(sqrt(c) d)/d, d = |r-P|;
  its value at d = 0 is 2 pi/c.
* Potential of the normalised density (a/pi)^{3/2} exp(-a|r-C|^2):
  erf(sqrt(a) d)/d (value 2 sqrt(a/pi) at d = 0).
* Coulomb energy of two unnormalised Gaussians exp(-p|r-P|^2), exp(-q|r-Q|^2):
  2 pi^{5/2} / (p q sqrt(p+q)) F0(p q |P-Q|^2/(p+q)),
  F0(t) = (1/2) sqrt(pi/t) erf(sqrt t), F0(0) = 1.
"""
import numpy as np
from scipy.special import erf


def prim_norm(a):
    return (2.0 * a / np.pi) ** 0.75


def boys0(t):
    t = np.asarray(t, dtype=np.float64)
    out = np.ones_like(t)
    big = t > 1e-12
    st = np.sqrt(t[big])
    out[big] = 0.5 * np.sqrt(np.pi) * erf(st) / st
    small = ~big
    out[small] = 1.0 - t[small] / 3.0
    return out


def erf_over_r(c_sqrt, d):
    """erf(c d)/d with its limit 2c/sqrt(pi) at d = 0."""
    d = np.asarray(d, dtype=np.float64)
    out = np.empty(np.broadcast(c_sqrt, d).shape)
    cd = c_sqrt * d
    small = np.abs(cd) < 1e-6
    with np.errstate(divide="ignore", invalid="ignore"):
        val = erf(cd) / d
    lim = 2.0 * c_sqrt / np.sqrt(np.pi) * (1.0 - cd ** 2 / 3.0)
    out[...] = np.where(small, lim, val)
    return out


class Primitives:
    """A pool of normalised s-type primitives (exponents ``alpha``, centres ``centres``)."""

    def __init__(self, alpha, centres):
        self.alpha = np.asarray(alpha, dtype=np.float64)
        self.centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
        self.norm = prim_norm(self.alpha)

    def __len__(self):
        return len(self.alpha)

    def overlap(self):
        a, b = self.alpha[:, None], self.alpha[None, :]
        d2 = np.sum((self.centres[:, None, :] - self.centres[None, :, :]) ** 2, axis=-1)
        p = a + b
        return (self.norm[:, None] * self.norm[None, :] * (np.pi / p) ** 1.5
                * np.exp(-a * b / p * d2))

    def values(self, X, Y, Z):
        """chi_a at the points, shape [npr] + broadcast(X, Y, Z).shape."""
        X, Y, Z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (X, Y, Z)))
        out = np.empty((len(self),) + X.shape)
        for a in range(len(self)):
            A = self.centres[a]
            out[a] = self.norm[a] * np.exp(-self.alpha[a] * ((X - A[0]) ** 2 + (Y - A[1]) ** 2 + (Z - A[2]) ** 2))
        return out

    def product_terms(self):
        """For every unordered primitive pair (a <= b): prefactor, exponent, centre."""
        ia, ib = np.triu_indices(len(self))
        a, b = self.alpha[ia], self.alpha[ib]
        p = a + b
        d2 = np.sum((self.centres[ia] - self.centres[ib]) ** 2, axis=-1)
        K = self.norm[ia] * self.norm[ib] * np.exp(-a * b / p * d2)
        P = (a[:, None] * self.centres[ia] + b[:, None] * self.centres[ib]) / p[:, None]
        return ia, ib, K, p, P

    def pair_potentials(self, X, Y, Z):
        """Potential of chi_a chi_b (a <= b) at the points: [npairs_prim, npts]."""
        X, Y, Z = (np.asarray(v, dtype=np.float64).reshape(-1) for v in np.broadcast_arrays(X, Y, Z))
        ia, ib, K, p, P = self.product_terms()
        out = np.empty((len(ia), X.size))
        for t in range(len(ia)):
            d = np.sqrt((X - P[t, 0]) ** 2 + (Y - P[t, 1]) ** 2 + (Z - P[t, 2]) ** 2)
            out[t] = K[t] * (np.pi / p[t]) ** 1.5 * erf_over_r(np.sqrt(p[t]), d)
        return out

    def coulomb_pair_matrix(self):
        """(ab|cd) for unordered primitive pairs, matrix over pair indices."""
        ia, ib, K, p, P = self.product_terms()
        pp, qq = p[:, None], p[None, :]
        d2 = np.sum((P[:, None, :] - P[None, :, :]) ** 2, axis=-1)
        return (K[:, None] * K[None, :] * 2.0 * np.pi ** 2.5 / (pp * qq * np.sqrt(pp + qq))
                * boys0(pp * qq / (pp + qq) * d2))


def _t(a, device):
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64)
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device=device)


def erf_over_r_torch(c_sqrt, d):
    """erf(c d)/d with its limit 2c/sqrt(pi) at d = 0 (torch tensors)."""
    import torch
    cd = c_sqrt * d
    lim = 2.0 * c_sqrt / np.sqrt(np.pi) * (1.0 - cd * cd / 3.0)
    val = torch.erf(cd) / torch.where(d > 0, d, torch.ones_like(d))
    return torch.where(cd.abs() < 1e-6, lim, val)


def lowdin(C, S):
    """C <- C (C^T S C)^{-1/2}: orbitals orthonormal in the analytic overlap S."""
    G = C.T @ S @ C
    lam, U = np.linalg.eigh(G)
    return C @ (U * lam ** -0.5) @ U.T


class Orbitals:
    """Orbitals phi_i = sum_a C[a, i] chi_a over a primitive pool."""

    def __init__(self, prims, C):
        self.prims = prims
        self.C = np.asarray(C, dtype=np.float64)

    @property
    def norb(self):
        return self.C.shape[1]

    def pairs(self):
        return [(i, j) for i in range(self.norb) for j in range(i, self.norb)]

    def values(self, X, Y, Z):
        chi = self.prims.values(X, Y, Z)
        return np.tensordot(self.C.T, chi, axes=1)

    def _pair_coeffs(self):
        """Coefficient of chi_a chi_b (a <= b) in phi_i phi_j, for every orbital pair."""
        ia, ib, _, _, _ = self.prims.product_terms()
        rows = []
        for i, j in self.pairs():
            c = self.C[ia, i] * self.C[ib, j] + self.C[ib, i] * self.C[ia, j]
            c = np.where(ia == ib, 0.5 * c, c)
            rows.append(c)
        return np.array(rows)

    def values_torch(self, X, Y, Z, device="cpu"):
        """The orbitals at the points with torch (float64, on ``device``): [norb, npts]."""
        import torch
        X, Y, Z = (_t(v, device).reshape(-1) for v in (X, Y, Z))
        pr = self.prims
        chi = torch.empty((len(pr), X.numel()), dtype=torch.float64, device=X.device)
        for a in range(len(pr)):
            A = pr.centres[a]
            chi[a] = pr.norm[a] * torch.exp(-pr.alpha[a] * ((X - A[0]) ** 2 + (Y - A[1]) ** 2 + (Z - A[2]) ** 2))
        return _t(self.C.T, device) @ chi

    def pair_potentials_torch(self, X, Y, Z, device="cpu", chunk=512):
        """pair_potentials with torch (float64, on ``device``): [npairs, npts], summed over
        chunks of primitive pairs."""
        import torch
        X, Y, Z = (_t(v, device).reshape(-1) for v in (X, Y, Z))
        ia, ib, K, p, P = self.prims.product_terms()
        coef = _t(self._pair_coeffs(), device)
        out = torch.zeros((coef.shape[0], X.numel()), dtype=torch.float64, device=X.device)
        for t0 in range(0, len(ia), chunk):
            sl = slice(t0, min(len(ia), t0 + chunk))
            Pc = _t(P[sl], device)
            pc = _t(p[sl], device)[:, None]
            d = torch.sqrt((X[None] - Pc[:, 0:1]) ** 2 + (Y[None] - Pc[:, 1:2]) ** 2 + (Z[None] - Pc[:, 2:3]) ** 2)
            V = _t(K[sl], device)[:, None] * (np.pi / pc) ** 1.5 * erf_over_r_torch(torch.sqrt(pc), d)
            out += coef[:, sl] @ V
        return out

    def pair_potentials(self, X, Y, Z):
        """Full-space potential of every pair density phi_i phi_j (i <= j) at the points."""
        V = self.prims.pair_potentials(X, Y, Z)
        shape = np.broadcast(X, Y, Z).shape
        return (self._pair_coeffs() @ V).reshape((-1,) + shape)

    def pair_coulomb(self):
        """Continuum (ij|ij) for every pair i <= j."""
        Cp = self._pair_coeffs()
        G = self.prims.coulomb_pair_matrix()
        return np.einsum("ka,ab,kb->k", Cp, G, Cp)


class GaussianDensity:
    """rho = sum_c w_c (a_c/pi)^{3/2} exp(-a_c |r - R_c|^2) and its potential."""

    def __init__(self, w, alpha, centres):
        self.w = np.asarray(w, dtype=np.float64)
        self.alpha = np.asarray(alpha, dtype=np.float64)
        self.centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)

    def density(self, X, Y, Z):
        out = 0.0
        for w, a, C in zip(self.w, self.alpha, self.centres):
            out = out + w * (a / np.pi) ** 1.5 * np.exp(-a * ((X - C[0]) ** 2 + (Y - C[1]) ** 2 + (Z - C[2]) ** 2))
        return out

    def potential(self, X, Y, Z):
        out = 0.0
        for w, a, C in zip(self.w, self.alpha, self.centres):
            d = np.sqrt((X - C[0]) ** 2 + (Y - C[1]) ** 2 + (Z - C[2]) ** 2)
            out = out + w * erf_over_r(np.sqrt(a), d)
        return out

    def coulomb_self(self):
        """int int rho rho'/|r-r'| for the whole density."""
        tot = 0.0
        for w1, a1, C1 in zip(self.w, self.alpha, self.centres):
            for w2, a2, C2 in zip(self.w, self.alpha, self.centres):
                pre = w1 * w2 * (a1 / np.pi) ** 1.5 * (a2 / np.pi) ** 1.5
                d2 = float(np.sum((C1 - C2) ** 2))
                tot += pre * 2.0 * np.pi ** 2.5 / (a1 * a2 * np.sqrt(a1 + a2)) * float(boys0(a1 * a2 / (a1 + a2) * d2))
        return tot
