"""SIPDG Laplacian on a uniform hexahedral auxiliary mesh, and the Poisson RHS.

Bilinear form (eq. sip_bilinear, Sec. 3.4): volume term sum_K int grad u . grad v
plus, on every interior face, -[[u]].{grad v} - {grad u}.[[v]] + sigma [[u]].[[v]].
Penalty (Sec. 3.5, eq. pen_poly): sigma >= C^2/(eps h) with C^2 = (p+1)^2/h and
eps = 1/8.  Read with equality and with the 1/h that makes sigma scale as
1/length: sigma_F = (p+1)^2 / (eps h_F), h_F the smaller width of the two
elements along the face normal.  On tensor-product elements the face terms act
along the normal only, so the 3D penalty is the 1D one along that axis.

The Poisson problem on the auxiliary mesh (Sec. 6.3) carries inhomogeneous
Dirichlet data on the outer boundary.  It is imposed weakly by the symmetric
interior-penalty boundary terms (Nitsche), which keep the matrix symmetric
positive definite; a boundary face uses its own element's width in sigma.

Quadrature: the nodal points define the quadrature rule (Sec. 6.1), so volume
and face integrals use collocation at the nodes; the mass is diagonal.  Two node
families: Gauss-Lobatto-Legendre (``family="gll"``, the default: the end points
are nodes, so face values are node values; the mass is lumped) and Gauss-Legendre
(``family="gl"``, the family Sec. 6.2 names: no node on a face, face values and
derivatives are interpolated, and the (p+1)-point rule integrates every product
that appears exactly, so the diagonal mass is the exact one).  With either rule
the 3D matrix is exactly the Kronecker sum (Sec. 3.5)
    A = A1_x (x) M1_y (x) M1_z + M1_x (x) A1_y (x) M1_z + M1_x (x) M1_y (x) A1_z.

The right-hand side of -Lap v = 4 pi f (eq. hartree_poisson, eq. fock_poisson)
is sampled pointwise at the nodes: b = 4 pi M f + boundary lift of g.

Test infrastructure only; see the package docstring.
"""
import numpy as np

from . import nodes as _nodes

PENALTY_EPS = 1.0 / 8.0


def penalty(p, h, eps=PENALTY_EPS):
    """sigma_F = (p+1)^2 / (eps h_F)   (eq. pen_poly with the 1/length reading)."""
    return (p + 1) ** 2 / (eps * h)


class Axis1D:
    """One coordinate direction: E uniform elements of degree p on [a, b].

    Attributes (all FP64, global 1D node index X = e*(p+1) + i):
      x      node coordinates, length E*(p+1)
      m      mass at the nodes  J*omega_i            (diagonal of M1)
      A      1D SIPDG matrix with Nitsche Dirichlet faces (dense)
      liftL  right-hand-side vector multiplying the left boundary value
      liftR  right-hand-side vector multiplying the right boundary value
      eL, eR values of the element's basis functions at its left / right end
      dL, dR their derivatives there (physical units)
    """

    def __init__(self, E, p, a, b, eps=PENALTY_EPS, family="gll"):
        self.E, self.p, self.a, self.b = int(E), int(p), float(a), float(b)
        n = p + 1
        self.n = n
        self.family = family
        self.h = (self.b - self.a) / E
        J = self.h / 2.0
        if family == "gll":
            xi, w, Dh = _nodes.gll(p)
        elif family == "gl":
            xi, w, Dh = _nodes.gl(p)
        else:
            raise ValueError(f"unknown node family {family!r}")
        self.xi, self.w, self.Dhat = xi, w, Dh
        self.sigma = penalty(p, self.h, eps)
        N = E * n
        self.x = np.concatenate([self.a + e * self.h + J * (xi + 1.0) for e in range(E)])
        self.m = np.tile(J * w, E)
        A = np.zeros((N, N))
        Kloc = Dh.T @ np.diag(w) @ Dh / J              # int_e l_i' l_j' dx
        for e in range(E):
            A[e * n:(e + 1) * n, e * n:(e + 1) * n] += Kloc
        # traces: u -> u(left end), u(right end), u'(left end), u'(right end) of an element
        eL = _nodes.lagrange_eval(xi, -1.0)[0]
        eR = _nodes.lagrange_eval(xi, 1.0)[0]
        dL = _nodes.lagrange_derivative(xi, -1.0)[0] / J
        dR = _nodes.lagrange_derivative(xi, 1.0)[0] / J

        def vec(e, local):
            v = np.zeros(N)
            v[e * n:(e + 1) * n] = local
            return v

        s = self.sigma
        for e in range(E - 1):
            # face between e (minus side, normal +1) and e+1 (plus side, normal -1)
            jmp = vec(e, eR) - vec(e + 1, eL)              # [[u]] along +x
            avg = 0.5 * vec(e, dR) + 0.5 * vec(e + 1, dL)  # {u'}
            A += -(np.outer(jmp, avg) + np.outer(avg, jmp)) + s * np.outer(jmp, jmp)
        # Dirichlet faces: [[u]] = u n, {u'} = u' on the boundary face
        jl, gl_ = vec(0, eL), -vec(0, dL)                  # left: n = -1, d_n u = -u'
        jr, gr_ = vec(E - 1, eR), vec(E - 1, dR)           # right: n = +1
        for jv, gv in ((jl, gl_), (jr, gr_)):
            A += -(np.outer(jv, gv) + np.outer(gv, jv)) + s * np.outer(jv, jv)
        self.A = A
        # lift: int_face g (sigma v - d_n v)
        self.liftL = s * jl - gl_
        self.liftR = s * jr - gr_
        self.eL, self.eR, self.dL, self.dR = eL, eR, dL, dR

    @property
    def N(self):
        return self.E * self.n


def make_axes(E, p, lo, hi, eps=PENALTY_EPS, family="gll"):
    """Three Axis1D objects (x, y, z) for an Ex*Ey*Ez mesh on the box [lo, hi]."""
    return [Axis1D(E[d], p, lo[d], hi[d], eps, family) for d in range(3)]


def apply(axes, u):
    """y = A u for u[Z, Y, X] (matrix-free Kronecker sum)."""
    ax, ay, az = axes
    u = np.asarray(u, dtype=np.float64)
    yx = (u @ ax.A.T) * ay.m[None, :, None] * az.m[:, None, None]              # A1 along X
    yy = np.matmul(ay.A, u) * ax.m[None, None, :] * az.m[:, None, None]        # A1 along Y
    yz = np.tensordot(az.A, u, axes=(1, 0)) * ax.m[None, None, :] * ay.m[None, :, None]  # along Z
    return yx + yy + yz


def mass(axes):
    """Diagonal of the 3D lumped mass as an array [Z, Y, X]."""
    ax, ay, az = axes
    return az.m[:, None, None] * ay.m[None, :, None] * ax.m[None, None, :]


def diagonal(axes):
    """diag(A) as an array [Z, Y, X]."""
    ax, ay, az = axes
    dx, dy, dz = np.diag(ax.A), np.diag(ay.A), np.diag(az.A)
    return (dx[None, None, :] * ay.m[None, :, None] * az.m[:, None, None]
            + ax.m[None, None, :] * dy[None, :, None] * az.m[:, None, None]
            + ax.m[None, None, :] * ay.m[None, :, None] * dz[:, None, None])


def dense_matrix(axes):
    """The Kronecker-sum matrix, rows/cols in the flattened [Z, Y, X] order."""
    ax, ay, az = axes
    Ix, Iy, Iz = np.diag(ax.m), np.diag(ay.m), np.diag(az.m)
    return (np.kron(Iz, np.kron(Iy, ax.A)) + np.kron(Iz, np.kron(ay.A, Ix))
            + np.kron(az.A, np.kron(Iy, Ix)))


def rhs(axes, f, faces):
    """b = 4 pi M f + sum over the six faces of (lift (x) M1 (x) M1) g.

    ``f`` is the source sampled at the nodes, array [Z, Y, X]; ``faces`` is the
    list [gxm, gxp, gym, gyp, gzm, gzp] of Dirichlet values at the face points
    (``face_points``: the boundary nodes for GLL; for GL the tangential nodes on
    the boundary plane), x faces indexed [Z, Y], y faces [Z, X], z faces [Y, X].
    With GLL, edge and corner nodes receive one term from each face they lie on.
    """
    ax, ay, az = axes
    b = 4.0 * np.pi * mass(axes) * np.asarray(f, dtype=np.float64)
    gxm, gxp, gym, gyp, gzm, gzp = [np.asarray(g, dtype=np.float64) for g in faces]
    mzy = az.m[:, None] * ay.m[None, :]
    mzx = az.m[:, None] * ax.m[None, :]
    myx = ay.m[:, None] * ax.m[None, :]
    b += ax.liftL[None, None, :] * (mzy * gxm)[:, :, None]
    b += ax.liftR[None, None, :] * (mzy * gxp)[:, :, None]
    b += ay.liftL[None, :, None] * (mzx * gym)[:, None, :]
    b += ay.liftR[None, :, None] * (mzx * gyp)[:, None, :]
    b += az.liftL[:, None, None] * (myx * gzm)[None, :, :]
    b += az.liftR[:, None, None] * (myx * gzp)[None, :, :]
    return b


def node_grid(axes):
    """Coordinate arrays X, Y, Z broadcastable to [Z, Y, X]."""
    ax, ay, az = axes
    return ax.x[None, None, :], ay.x[None, :, None], az.x[:, None, None]


def face_points(axes):
    """Coordinates of the face points where Dirichlet data are given, in face order
    (x-, x+, y-, y+, z-, z+): lists [X, Y, Z] of arrays shaped like the face (x faces [Z, Y],
    y faces [Z, X], z faces [Y, X]).  The tangential coordinates are the nodes of the other two
    axes and the normal coordinate is the boundary plane (for GLL these are the boundary nodes)."""
    ax, ay, az = axes
    out = []
    for d, (lo_, hi_) in enumerate(((ax.a, ax.b), (ay.a, ay.b), (az.a, az.b))):
        for v in (lo_, hi_):
            if d == 0:
                Zg, Yg = np.meshgrid(az.x, ay.x, indexing="ij")
                out.append([np.full(Zg.shape, v), Yg, Zg])
            elif d == 1:
                Zg, Xg = np.meshgrid(az.x, ax.x, indexing="ij")
                out.append([Xg, np.full(Zg.shape, v), Zg])
            else:
                Yg, Xg = np.meshgrid(ay.x, ax.x, indexing="ij")
                out.append([Xg, Yg, np.full(Yg.shape, v)])
    return out
