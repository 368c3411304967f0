"""Element-by-element assembly of the SIPDG matrix and RHS (independent construction).

This builds the same discrete problem as ``sipdg`` directly from the 3D
bilinear form eq. (sip_bilinear): for every element the volume integral of
grad(phi_a).grad(phi_b); for every interior face the terms
-[[phi_a]].{grad phi_b} - {grad phi_a}.[[phi_b]] + sigma [[phi_a]].[[phi_b]]
with the vector jump of eq. (jump_operator) and full 3D gradients; and for
boundary faces the Nitsche terms with [[phi]] = phi n and {grad phi} = grad phi.
Integrals use the tensor rule of the node family (GLL or GL) on the element and
on the face (the nodal points define the quadrature, Sec. 6.1); face traces are
the basis functions evaluated on the face.  Nothing here uses the Kronecker-sum
form, so agreement with ``sipdg.dense_matrix`` pins that construction.

Only for tiny meshes (dense matrices).  Test infrastructure only.
"""
import itertools

import numpy as np

from . import nodes as _nodes
from .sipdg import penalty, PENALTY_EPS


def _dof(E, n, e3, l3):
    """Flattened [Z, Y, X] index of local node l3=(i, j, k) in element e3=(ex, ey, ez)."""
    NX, NY = E[0] * n, E[1] * n
    X = e3[0] * n + l3[0]
    Y = e3[1] * n + l3[1]
    Z = e3[2] * n + l3[2]
    return (Z * NY + Y) * NX + X


def _basis_at(xi, pts_ref):
    """Values and reference derivatives of the 1D Lagrange basis at points."""
    return _nodes.lagrange_eval(xi, pts_ref), _nodes.lagrange_derivative(xi, pts_ref)


def assemble(E, p, lo, hi, f=None, faces=None, eps=PENALTY_EPS, family="gll"):
    """Dense A (and b if f, faces given) in flattened [Z, Y, X] order.

    f: callable f(x, y, z) or None;  faces: callable g(x, y, z) giving the
    Dirichlet value at boundary points, or None.
    """
    n = p + 1
    xi, w, _ = _nodes.gll(p) if family == "gll" else _nodes.gl(p)
    h = [(hi[d] - lo[d]) / E[d] for d in range(3)]
    J = [hd / 2.0 for hd in h]
    NX, NY, NZ = E[0] * n, E[1] * n, E[2] * n
    Ntot = NX * NY * NZ
    A = np.zeros((Ntot, Ntot))
    b = np.zeros(Ntot)
    local = list(itertools.product(range(n), range(n), range(n)))  # (i, j, k)
    V1, G1 = _basis_at(xi, xi)  # quadrature points are the nodes

    def phys(e3, d, r):
        return lo[d] + e3[d] * h[d] + J[d] * (r + 1.0)

    # ---- volume terms
    for e3 in itertools.product(range(E[0]), range(E[1]), range(E[2])):
        idx = [_dof(E, n, e3, l3) for l3 in local]
        for q3 in local:
            W = J[0] * J[1] * J[2] * w[q3[0]] * w[q3[1]] * w[q3[2]]
            val = np.array([V1[q3[0], a[0]] * V1[q3[1], a[1]] * V1[q3[2], a[2]] for a in local])
            grad = np.array([[G1[q3[0], a[0]] / J[0] * V1[q3[1], a[1]] * V1[q3[2], a[2]],
                              V1[q3[0], a[0]] * G1[q3[1], a[1]] / J[1] * V1[q3[2], a[2]],
                              V1[q3[0], a[0]] * V1[q3[1], a[1]] * G1[q3[2], a[2]] / J[2]]
                             for a in local])
            A[np.ix_(idx, idx)] += W * grad @ grad.T
            if f is not None:
                X = [phys(e3, d, xi[q3[d]]) for d in range(3)]
                b[idx] += W * 4.0 * np.pi * f(*X) * val

    # trace of the element basis on a face: reference coordinate along d fixed at s = -1 or +1
    def traces(e3, d, s, fq):
        """Values and 3D gradients of all local basis functions at face point fq.

        fq: reference coordinates of the face point in the two tangential
        directions, as a 3-tuple with the normal entry ignored.
        """
        rv = [fq[0], fq[1], fq[2]]
        rv[d] = s
        Vs = [_basis_at(xi, np.array([rv[c]])) for c in range(3)]
        val = np.array([Vs[0][0][0, a[0]] * Vs[1][0][0, a[1]] * Vs[2][0][0, a[2]] for a in local])
        grad = np.array([[Vs[0][1][0, a[0]] / J[0] * Vs[1][0][0, a[1]] * Vs[2][0][0, a[2]],
                          Vs[0][0][0, a[0]] * Vs[1][1][0, a[1]] / J[1] * Vs[2][0][0, a[2]],
                          Vs[0][0][0, a[0]] * Vs[1][0][0, a[1]] * Vs[2][1][0, a[2]] / J[2]]
                         for a in local])
        return val, grad

    # ---- face terms
    for d in range(3):
        t1, t2 = [c for c in range(3) if c != d]
        for e3 in itertools.product(range(E[0]), range(E[1]), range(E[2])):
            for q1, q2 in itertools.product(range(n), range(n)):
                W = J[t1] * J[t2] * w[q1] * w[q2]
                fq = [0.0, 0.0, 0.0]
                fq[t1], fq[t2] = xi[q1], xi[q2]
                nrm = np.zeros(3); nrm[d] = 1.0
                # interior face on the + side of e3 along d
                if e3[d] + 1 < E[d]:
                    e3p = list(e3); e3p[d] += 1; e3p = tuple(e3p)
                    hF = min(h[d], h[d])
                    sig = penalty(p, hF, eps)
                    vm, gm = traces(e3, d, +1.0, fq)
                    vp, gp = traces(e3p, d, -1.0, fq)
                    idx = [_dof(E, n, e3, l3) for l3 in local] + [_dof(E, n, e3p, l3) for l3 in local]
                    jump = np.concatenate([vm[:, None] * nrm[None, :], vp[:, None] * (-nrm)[None, :]])
                    avg = np.concatenate([0.5 * gm, 0.5 * gp])
                    blk = -(jump @ avg.T) - (avg @ jump.T) + sig * (jump @ jump.T)
                    A[np.ix_(idx, idx)] += W * blk
                # boundary faces
                for side, s in ((0, -1.0), (E[d] - 1, +1.0)):
                    if e3[d] != side:
                        continue
                    sig = penalty(p, h[d], eps)
                    vb, gb = traces(e3, d, s, fq)
                    nb = s * nrm
                    idx = [_dof(E, n, e3, l3) for l3 in local]
                    jump = vb[:, None] * nb[None, :]
                    blk = -(jump @ gb.T) - (gb @ jump.T) + sig * (jump @ jump.T)
                    A[np.ix_(idx, idx)] += W * blk
                    if faces is not None:
                        X = [phys(e3, c, (s if c == d else fq[c])) for c in range(3)]
                        g = faces(*X)
                        b[idx] += W * g * (sig * vb - gb @ nb)
    return A, b
