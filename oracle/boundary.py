"""Dirichlet data of the auxiliary-mesh Poisson problem by quadrature (Sec. 6.3).

The full-space problem -Lap u = 4 pi f with u -> 0 at infinity is restated on
the mesh domain Omega with Dirichlet data equal to the Coulomb potential of f
on the boundary:  u(r) = int_Omega f(r') / |r - r'| dr',  r on dOmega.  The
integral is evaluated with the quadrature rule of the mesh's own nodal grid.
Here the grid is the GLL grid of the discretisation, so the rule is the lumped
mass: weight W_q = J_x w_i * J_y w_j * J_z w_k at node x_q, and

    g(r) = sum_q W_q f(x_q) / |r - x_q|.

Reading: on a GLL grid every boundary node r is itself a node x_q of the
grid, where the integrand is singular.  The method relies on f vanishing at
the boundary to machine precision, so that term is taken as zero: terms whose
distance is below 1e-6 of the smallest element width are left out (any other
node is at least a few tenths of an element width away).

Test infrastructure only; see the package docstring.
"""
import numpy as np

from . import layout, sipdg

COINCIDENT = 1e-6      # fraction of the smallest element width below which a term is left out


def weights(axes):
    """Quadrature weight of every node, array [Z, Y, X] (the lumped mass)."""
    return sipdg.mass(axes)


def drop_radius(axes):
    return COINCIDENT * min(ax.h for ax in axes)


def potential_at(axes, f, points, chunk=None):
    """g at arbitrary points.

    f: sources sampled at the nodes, array [..., Z, Y, X] (leading axes are
    several sources); points: array [P, 3].  Returns [..., P].
    """
    f = np.asarray(f, dtype=np.float64)
    lead = f.shape[:-3]
    X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
    xq = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)      # [N, 3]
    F = (weights(axes) * f).reshape(-1, xq.shape[0]).T                        # [N, S]
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty((pts.shape[0], F.shape[1]))
    rmin = drop_radius(axes)
    if chunk is None:                      # rows per block of the distance matrix (memory only)
        chunk = int(max(16, min(256, 2e7 // xq.shape[0])))
    for s in range(0, pts.shape[0], chunk):
        d = np.sqrt(np.sum((pts[s:s + chunk, None, :] - xq[None, :, :]) ** 2, axis=-1))    # [c, N]
        K = np.where(d > rmin, 1.0 / np.where(d > rmin, d, 1.0), 0.0)
        out[s:s + chunk] = K @ F
    return out.T.reshape(lead + (pts.shape[0],))


def boundary_points(axes):
    """The face points (the boundary nodes for GLL) in face order (x-, x+, y-, y+, z-, z+),
    array [n_face, 3]."""
    fp = sipdg.face_points(axes)
    fx, fy, fz = ([fp[f][c] for f in range(6)] for c in range(3))
    return np.stack([layout.join_faces(fx), layout.join_faces(fy), layout.join_faces(fz)], axis=1)


def dirichlet_data(axes, f):
    """Face list [gxm, gxp, gym, gyp, gzm, gzp] of g for one source f[Z, Y, X]."""
    g = potential_at(axes, f, boundary_points(axes))
    E = [ax.E for ax in axes]
    return layout.split_faces(g, E, axes[0].n)
