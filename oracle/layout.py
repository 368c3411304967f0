"""Storage orders used at the library boundary, and their global-tensor views.

Field order (library boundary): ``[ez][ey][ex][k][j][i]`` -- elements
lexicographic with x fastest, then the element's (p+1)^3 nodes with the local
x index i fastest.  Inside the oracle a field is the array ``u[Z, Y, X]`` over
global 1D node indices X = ex*(p+1) + i (and likewise Y, Z), which makes the
Kronecker-sum structure of the operator explicit.

Face order (library boundary): six faces x-, x+, y-, y+, z-, z+ concatenated;
an x face is ``[Z][Y]`` (Y fastest), a y face ``[Z][X]``, a z face ``[Y][X]``.

Test infrastructure only; see the package docstring.
"""
import numpy as np


def to_global(u_em, E, n):
    """Element-major vector (length Ez*Ey*Ex*n^3) -> array u[Z, Y, X]."""
    Ex, Ey, Ez = E
    a = np.asarray(u_em).reshape(Ez, Ey, Ex, n, n, n)      # ez ey ex k j i
    a = a.transpose(0, 3, 1, 4, 2, 5)                      # ez k ey j ex i
    return a.reshape(Ez * n, Ey * n, Ex * n)


def to_element_major(u, E, n):
    """Array u[Z, Y, X] -> element-major vector."""
    Ex, Ey, Ez = E
    a = np.asarray(u).reshape(Ez, n, Ey, n, Ex, n)         # ez k ey j ex i
    a = a.transpose(0, 2, 4, 1, 3, 5)                      # ez ey ex k j i
    return np.ascontiguousarray(a).reshape(-1)


def face_sizes(E, n):
    """Number of nodes on the faces x-, x+, y-, y+, z-, z+."""
    NX, NY, NZ = (E[0] * n, E[1] * n, E[2] * n)
    return [NZ * NY, NZ * NY, NZ * NX, NZ * NX, NY * NX, NY * NX]


def split_faces(g, E, n):
    """Concatenated face vector -> list of 2D arrays [gxm, gxp, gym, gyp, gzm, gzp]."""
    NX, NY, NZ = (E[0] * n, E[1] * n, E[2] * n)
    shapes = [(NZ, NY), (NZ, NY), (NZ, NX), (NZ, NX), (NY, NX), (NY, NX)]
    out, off = [], 0
    g = np.asarray(g)
    for s in shapes:
        cnt = s[0] * s[1]
        out.append(g[off:off + cnt].reshape(s))
        off += cnt
    if off != g.size:
        raise ValueError("face vector has wrong length")
    return out


def join_faces(faces):
    return np.concatenate([np.asarray(f).reshape(-1) for f in faces])


def boundary_faces_of(u):
    """Sample a global field u[Z, Y, X] on the six boundary faces (node values)."""
    return [u[:, :, 0], u[:, :, -1], u[:, 0, :], u[:, -1, :], u[0, :, :], u[-1, :, :]]
