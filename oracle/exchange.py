"""Exchange potentials and pair energies on the auxiliary grid (Sec. 6.1).

For orbitals phi_1..phi_N sampled at the nodes, every pair density
rho_ij = phi_i phi_j (i <= j) is the source of one Poisson problem
-Lap v_ij = 4 pi rho_ij (eq. fock_poisson with u = phi_i, psi_s = phi_j).
From the potentials:

* W_k = sum_s phi_s v_ks with v_ks = v_sk: the exchange action on u = phi_k,
  evaluated pointwise at the quadrature points (positive sign, as in the
  integrand of the exchange action; the HF prefactor is the caller's);
* K_ij = sum over nodes of M rho_ij v_ij (GLL quadrature of int rho_ij v_ij);
* E_X = sum over ordered pairs = sum_i K_ii + 2 sum_{i<j} K_ij.

Pair index: idx(i, j) = i*N - i(i-1)/2 + (j - i) for i <= j.

Test infrastructure only; see the package docstring.
"""
import numpy as np

from . import sipdg as _sipdg


def pair_index(i, j, norb):
    if i > j:
        i, j = j, i
    return i * norb - i * (i - 1) // 2 + (j - i)


def pairs(norb):
    return [(i, j) for i in range(norb) for j in range(i, norb)]


def pair_densities(phi):
    norb = len(phi)
    return [phi[i] * phi[j] for i, j in pairs(norb)]


def exchange(axes, phi, faces_pairs, solve):
    """Return (v list, W list, K array, E_X).

    phi: list of arrays [Z, Y, X]; faces_pairs: list (pair order) of face
    lists; solve: callable b -> v for the discrete system.
    """
    norb = len(phi)
    M = _sipdg.mass(axes)
    rhos = pair_densities(phi)
    v = [solve(_sipdg.rhs(axes, rho, fc)) for rho, fc in zip(rhos, faces_pairs)]
    K = np.array([float(np.sum(M * rho * vv)) for rho, vv in zip(rhos, v)])
    W = []
    for k in range(norb):
        acc = np.zeros_like(phi[0])
        for s in range(norb):
            acc = acc + phi[s] * v[pair_index(k, s, norb)]
        W.append(acc)
    EX = sum(K[pair_index(i, i, norb)] for i in range(norb)) + \
        2.0 * sum(K[pair_index(i, j, norb)] for i, j in pairs(norb) if i < j)
    return v, W, K, float(EX)
