"""Consumers of the auxiliary-grid potentials: the Hartree and exchange actions projected on a
basis, and the adaptively compressed exchange (Sec. 6.1, Sec. 7.2).

Every integral is the grid's quadrature rule (Sec. 6.1: the interpolating grid defines the
quadrature, each factor of the integrand evaluated pointwise at the nodes); with the GLL grid
the weights are the lumped mass ``sipdg.mass``.  Functions are arrays [Z, Y, X] at the nodes.

* Hartree action on u projected on basis functions phi_i (the equation after
  eq. hartreecoulomb): out[i, a] = sum_q w_q phi_i u_a v_H.
* Exchange action on u projected on phi_i (eq. fock_exchange and the equation after it): for
  every occupied psi_s, v_as solves -Lap v = 4 pi u_a psi_s on the grid (eq. fock_poisson);
  W_a = sum_s psi_s v_as; out[i, a] = sum_q w_q phi_i W_a.  Positive sign (the integrand as
  written); the Hartree-Fock prefactor of the operator is the caller's.
* Adaptively compressed exchange (Sec. 7.2, the construction of the cited reference): from
  W_k, the exchange action on the occupied orbitals psi_k, form M_kl = (psi_k, W_l)_w, take its
  symmetric part (the discrete operator with Dirichlet data is symmetric only up to the data's
  consistency), factor M = L L^T (Cholesky) and set xi = L^-1 W (row k of xi is a combination of
  W_1..W_k).  The compressed operator K_ace = sum_k xi_k (xi_k, .)_w has rank N_occ and equals
  the exchange operator on span(psi): K_ace psi_j = W_j.
  out[i, a] = sum_k (phi_i, xi_k)_w (xi_k, u_a)_w.

Test infrastructure only; see the package docstring.
"""
import numpy as np
import scipy.linalg

from . import sipdg as _sipdg


def weights(axes):
    """Quadrature weights of the grid (the lumped GLL mass), [Z, Y, X]."""
    return _sipdg.mass(axes)


def inner(w, f, g):
    """Matrix of quadrature inner products (f_i, g_a)_w for stacks f [n, ...], g [m, ...]."""
    f = np.asarray(f).reshape(len(f), -1)
    g = np.asarray(g).reshape(len(g), -1)
    return f @ (w.reshape(-1)[:, None] * g.T)


def hartree_action(w, phi, u, vH):
    """out[i, a] = sum_q w_q phi_i u_a vH."""
    return inner(w * vH, phi, u)


def exchange_potentials(axes, u, psi, faces, solve):
    """v[a][s] solving the discrete problem with source u_a psi_s and Dirichlet data faces[a][s]
    (a face list each); solve: b -> v."""
    return [[solve(_sipdg.rhs(axes, u[a] * psi[s], faces[a][s])) for s in range(len(psi))]
            for a in range(len(u))]


def exchange_w(psi, v):
    """W_a = sum_s psi_s v_as."""
    W = []
    for a in range(len(v)):
        acc = np.zeros_like(psi[0])
        for s in range(len(psi)):
            acc = acc + psi[s] * v[a][s]
        W.append(acc)
    return W


def exchange_action(axes, phi, u, psi, faces, solve):
    """(out[i, a], W): the projected exchange action and the pointwise W_a."""
    w = weights(axes)
    W = exchange_w(psi, exchange_potentials(axes, u, psi, faces, solve))
    return inner(w, phi, W), W


def ace(w, psi, W):
    """(xi, M, L): the compressed exchange vectors from the occupied orbitals and their W."""
    M = inner(w, psi, W)
    M = 0.5 * (M + M.T)
    L = np.linalg.cholesky(M)
    Wf = np.asarray(W).reshape(len(W), -1)
    xi = scipy.linalg.solve_triangular(L, Wf, lower=True).reshape(np.asarray(W).shape)
    return xi, M, L


def ace_action(w, phi, u, xi):
    """out[i, a] = sum_k (phi_i, xi_k)_w (xi_k, u_a)_w."""
    return inner(w, phi, xi) @ inner(w, xi, u)
