"""Adaptive octree auxiliary mesh, its SIPDG Poisson problem, and hp + geometric multigrid over
the nested refinement hierarchy (Sec. 6.2 auxiliary mesh, Sec. 6.3 Poisson discretisation,
Sec. 6.4 linear solver).

Mesh (Sec. 6.2).  The refinement starts from a uniform box mesh of Ex x Ey x Ez base elements.
Every element carries degree-q tensor-product Gauss-Legendre nodes, which are also its
quadrature rule (eq. density_approx).  An element of edge lengths (Lx, Ly, Lz), L their
maximum, is halved along every axis d with L_d >= L/2 (not along an axis with L_d < L/2), which
gives 2, 4 or 8 children.  Its indicator compares the GL integral of the density on the element
with the sum of the GL integrals on its children,
    Q = | sum_i rho(x_i) w_i - sum_children sum_i rho(x~_i) w~_i |   (physical weights),
and an element with Q > delta_q is replaced by its children, which are tested in turn.
Readings: elements are tested generation by generation (the outcome does not depend on the
order: each decision uses the element's own samples only); a depth cap ``max_depth`` (halvings
of a base element) bounds the recursion, which the paper leaves unbounded.

Cells live on an integer lattice: per axis a level l_d (halvings along d) and an index i_d in
[0, E_d 2^l_d); along d the cell is lo_d + h_d [i_d, i_d + 1] / 2^l_d, h_d the base width.  A
cell's generation is the number of refinements that produced it.

Element order: depth first over the refinement tree; base elements in (z, y, x) lexicographic
order, x fastest (the uniform mesh's element-major order); the children of an element in (z, y,
x) lexicographic order of their half along each split axis, x fastest.  The (q+1)^3 nodes of an
element are stored [k][j][i], x index i fastest.

Discretisation (Sec. 6.3; eq. sip_bilinear, eq. pen_poly).  The SIPDG form of ``sipdg`` on the
leaves: volume terms grad u . grad v; on every face -[[u]].{grad v} - {grad u}.[[v]] +
sigma [[u]].[[v]]; Nitsche terms on the domain boundary.  Elements of different sizes meet on
hanging faces: the face of an element is tiled by the faces of its neighbours, and every
intersection of two faces ("piece", an axis-aligned rectangle, always the smaller face along
each tangential axis since the cells are dyadic) is integrated by the (q+1) x (q+1) GL rule of
the piece, each side's trace evaluated there by interpolation.  On a conforming face this is the
nodal rule of the common face, so an unrefined mesh gives exactly the Kronecker-sum matrix of
``sipdg`` with GL nodes.  Penalty on a piece: sigma of the smaller width along the normal (the
reading ``sipdg`` states).

Multigrid (Sec. 6.4): degree steps q -> q//2 -> ... -> 1 on the leaves, then mesh steps along the
nested hierarchy: the mesh of generation g is the tree cut at g (cells of generation g and
leaves of lower generation), for g = G-1 down to 0, the uniform base mesh at degree 1, where
the exact fast-diagonalisation solve of ``fdm`` applies.  Every level is rediscretised; the
prolongation interpolates the coarse polynomial at the fine nodes (same element for a degree
step, the parent for a mesh step); R = P^T; the Chebyshev-Jacobi smoother of ``mg`` with its
parameters (``degree_h`` steps on the degree-1 levels below the finest).

Test infrastructure only; see the package docstring.
"""
import itertools

import numpy as np

from . import mg as _mg
from . import nodes as _nodes
from . import sipdg as _sipdg
from .fdm import FDM
from .layout import to_element_major, to_global


class Cell:
    __slots__ = ("lv", "ix", "gen", "children")

    def __init__(self, lv, ix, gen):
        self.lv, self.ix, self.gen = tuple(lv), tuple(ix), gen
        self.children = []


class Octree:
    """The refined auxiliary mesh.  ``rho(x, y, z)`` (arrays) drives the refinement; None keeps
    the base mesh.  ``manual``: optional callable cell -> bool that forces a split (tests)."""

    def __init__(self, E, lo, hi, q, rho=None, delta_q=1e-8, max_depth=3, manual=None):
        self.E = tuple(int(e) for e in E)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.q, self.n = int(q), int(q) + 1
        self.h = [(self.hi[d] - self.lo[d]) / self.E[d] for d in range(3)]
        self.xi, self.w, _ = _nodes.gl(self.q)
        self.roots = [Cell((0, 0, 0), (ex, ey, ez), 0)
                      for ez in range(self.E[2]) for ey in range(self.E[1]) for ex in range(self.E[0])]
        self.tested = 0
        active = list(self.roots)
        while active:
            nxt = []
            for c in active:
                if c.gen >= max_depth:
                    continue
                kids = self.children_of(c)
                if manual is not None:
                    split = manual(c)
                else:
                    self.tested += 1
                    split = rho is not None and self.indicator(c, kids, rho) > delta_q
                if split:
                    c.children = kids
                    nxt.extend(kids)
            active = nxt
        self.max_gen = max(c.gen for c in self.cells())

    # ---- geometry
    def bounds(self, c):
        """(a, b): the cell's lower and upper corner."""
        a = [self.lo[d] + self.h[d] * (c.ix[d] / 2.0 ** c.lv[d]) for d in range(3)]
        b = [a[d] + self.h[d] / 2.0 ** c.lv[d] for d in range(3)]
        return np.array(a), np.array(b)

    def gl_points(self, c):
        """Node coordinates X, Y, Z ([k][j][i], flattened) and physical GL weights of a cell."""
        a, b = self.bounds(c)
        x = [a[d] + 0.5 * (b[d] - a[d]) * (self.xi + 1.0) for d in range(3)]
        wd = [0.5 * (b[d] - a[d]) * self.w for d in range(3)]
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        W = wd[2][:, None, None] * wd[1][None, :, None] * wd[0][None, None, :]
        return X.reshape(-1), Y.reshape(-1), Z.reshape(-1), W.reshape(-1)

    def split_axes(self, c):
        L = [self.h[d] / 2.0 ** c.lv[d] for d in range(3)]
        Lm = max(L)
        return [d for d in range(3) if L[d] >= 0.5 * Lm]

    def children_of(self, c):
        S = self.split_axes(c)
        kids = []
        for oz, oy, ox in itertools.product(*[(0, 1) if d in S else (0,) for d in (2, 1, 0)]):
            o = (ox, oy, oz)
            lv = [c.lv[d] + (1 if d in S else 0) for d in range(3)]
            ix = [2 * c.ix[d] + o[d] if d in S else c.ix[d] for d in range(3)]
            kids.append(Cell(lv, ix, c.gen + 1))
        return kids

    def integral(self, c, rho):
        X, Y, Z, W = self.gl_points(c)
        return float(np.sum(rho(X, Y, Z) * W))

    def indicator(self, c, kids, rho):
        """Q of a cell against the given split."""
        return abs(self.integral(c, rho) - sum(self.integral(k, rho) for k in kids))

    # ---- meshes of the hierarchy
    def cells(self, gen_cut=None):
        """Cells of the mesh cut at generation gen_cut (None: the leaves), in element order."""
        out = []

        def walk(c):
            if not c.children or (gen_cut is not None and c.gen >= gen_cut):
                out.append(c)
            else:
                for k in c.children:
                    walk(k)
        for r in self.roots:
            walk(r)
        return out

    def mesh(self, gen_cut=None, q=None):
        return Mesh(self, self.cells(gen_cut), self.q if q is None else q)


class Mesh:
    """A conforming-or-hanging mesh of cells of one tree, at degree q, with its face pieces.

    pieces: list of (d, A, sA, B, t1, t2) -- normal axis d; cell A on its face sA (-1 lower,
    +1 upper); neighbour cell B (-1 on the domain boundary) on its opposite face; t1, t2 the
    piece's physical intervals along the tangential axes (t1 < t2 in axis order).  Interior pieces
    are listed once, with A the lower cell (sA = +1); boundary pieces in element order, then
    face order x-, x+, y-, y+, z-, z+.
    """

    def __init__(self, tree, cells, q, eps=_sipdg.PENALTY_EPS):
        self.tree, self.cells, self.q, self.n = tree, cells, int(q), int(q) + 1
        self.xi, self.w, self.Dhat = _nodes.gl(self.q)
        self.eps = eps
        nc = len(cells)
        self.a = np.empty((nc, 3))
        self.b = np.empty((nc, 3))
        for e, c in enumerate(cells):
            self.a[e], self.b[e] = tree.bounds(c)
        self.J = 0.5 * (self.b - self.a)
        self.ndof = nc * self.n ** 3
        self._build_pieces()

    def _build_pieces(self):
        cells, E = self.cells, self.tree.E
        Lm = [max(c.lv[d] for c in cells) for d in range(3)]
        lo = np.array([[c.ix[d] << (Lm[d] - c.lv[d]) for d in range(3)] for c in cells])
        hi = np.array([[(c.ix[d] + 1) << (Lm[d] - c.lv[d]) for d in range(3)] for c in cells])
        top = [E[d] << Lm[d] for d in range(3)]
        self.pieces = []
        interior = []
        for d in range(3):
            t1, t2 = [t for t in range(3) if t != d]
            by_lo = {}
            for e in range(len(cells)):
                by_lo.setdefault(lo[e, d], []).append(e)
            for A in range(len(cells)):
                for B in by_lo.get(hi[A, d], []):
                    if (lo[A, t1] < hi[B, t1] and lo[B, t1] < hi[A, t1] and lo[A, t2] < hi[B, t2]
                            and lo[B, t2] < hi[A, t2]):
                        iv = []
                        for t in (t1, t2):   # the smaller of the two nested intervals
                            S = A if hi[A, t] - lo[A, t] <= hi[B, t] - lo[B, t] else B
                            iv.append((self.a[S, t], self.b[S, t]))
                        interior.append((d, A, +1, B, iv[0], iv[1]))
        boundary = []
        for A in range(len(cells)):
            for d in range(3):
                t1, t2 = [t for t in range(3) if t != d]
                for s in (-1, +1):
                    if (s < 0 and lo[A, d] == 0) or (s > 0 and hi[A, d] == top[d]):
                        boundary.append((d, A, s, -1, (self.a[A, t1], self.b[A, t1]),
                                         (self.a[A, t2], self.b[A, t2])))
        self.pieces = interior + boundary
        self.boundary = boundary

    # ---- 1D factors of a cell's traces on a piece
    def _factors(self, e, d, s, t1iv, t2iv):
        """(vn, dn, I1, I2, w1, w2): value and d/dx_d rows of the basis along the normal at the
        face s of cell e, interpolation from the cell's nodes to the piece's GL points along t1
        and t2, and the piece's physical GL weights along t1 and t2."""
        t1, t2 = [t for t in range(3) if t != d]
        vn = _nodes.lagrange_eval(self.xi, float(s))[0]
        dn = _nodes.lagrange_derivative(self.xi, float(s))[0] / self.J[e, d]
        out = []
        for t, (pa, pb) in ((t1, t1iv), (t2, t2iv)):
            xq = pa + 0.5 * (pb - pa) * (self.xi + 1.0)
            r = 2.0 * (xq - self.a[e, t]) / (self.b[e, t] - self.a[e, t]) - 1.0
            out.append((_nodes.lagrange_eval(self.xi, r), 0.5 * (pb - pa) * self.w))
        (I1, w1), (I2, w2) = out
        return vn, dn, I1, I2, w1, w2

    def sigma(self, d, A, B):
        hA = self.b[A, d] - self.a[A, d]
        hF = hA if B < 0 else min(hA, self.b[B, d] - self.a[B, d])
        return _sipdg.penalty(self.q, hF, self.eps)

    @staticmethod
    def _kron3(F, d, Fn):
        """3D operator (points [t2][t1] x nodes [k][j][i]) from the normal row Fn and the
        tangential matrices F = (F1, F2)."""
        Fx = {0: None, 1: None, 2: None}
        t1, t2 = [t for t in range(3) if t != d]
        Fx[d] = Fn[None, :]
        Fx[t1], Fx[t2] = F
        return np.kron(Fx[2], np.kron(Fx[1], Fx[0]))

    # ---- dense assembly (small meshes): the bilinear form piece by piece
    def dense(self, g=None):
        """(A, lift): dense matrix; with g (boundary values, ``boundary_points`` order) also the
        boundary part of the right-hand side."""
        n, N3 = self.n, self.n ** 3
        A = np.zeros((self.ndof, self.ndof))
        lift = np.zeros(self.ndof)
        K1 = self.Dhat.T @ np.diag(self.w) @ self.Dhat
        Wd = np.diag(self.w)
        for e in range(len(self.cells)):
            Jx, Jy, Jz = self.J[e]
            loc = (Jy * Jz / Jx * np.kron(Wd, np.kron(Wd, K1)) + Jx * Jz / Jy * np.kron(Wd, np.kron(K1, Wd))
                   + Jx * Jy / Jz * np.kron(K1, np.kron(Wd, Wd)))
            A[e * N3:(e + 1) * N3, e * N3:(e + 1) * N3] += loc
        goff = 0
        for (d, Ae, sA, Be, t1iv, t2iv) in self.pieces:
            vA, dA, I1, I2, w1, w2 = self._factors(Ae, d, sA, t1iv, t2iv)
            Wq = np.kron(w2, w1)
            TA = self._kron3((I1, I2), d, vA)
            GA = self._kron3((I1, I2), d, dA)
            sig = self.sigma(d, Ae, Be)
            if Be < 0:
                Gn = sA * GA                           # outward normal derivative
                blk = -(TA.T @ (Wq[:, None] * Gn) + Gn.T @ (Wq[:, None] * TA)) + sig * TA.T @ (Wq[:, None] * TA)
                A[Ae * N3:(Ae + 1) * N3, Ae * N3:(Ae + 1) * N3] += blk
                if g is not None:
                    gq = np.asarray(g[goff:goff + n * n])
                    lift[Ae * N3:(Ae + 1) * N3] += sig * TA.T @ (Wq * gq) - Gn.T @ (Wq * gq)
                goff += n * n
                continue
            vB, dB, J1, J2, _, _ = self._factors(Be, d, -1, t1iv, t2iv)
            TB = self._kron3((J1, J2), d, vB)
            GB = self._kron3((J1, J2), d, dB)
            jump = np.hstack([TA, -TB])                # [[u]] along +e_d (A below B)
            avg = 0.5 * np.hstack([GA, GB])            # {d u / d x_d}
            blk = -(jump.T @ (Wq[:, None] * avg) + avg.T @ (Wq[:, None] * jump)) + sig * jump.T @ (Wq[:, None] * jump)
            idx = np.concatenate([np.arange(Ae * N3, (Ae + 1) * N3), np.arange(Be * N3, (Be + 1) * N3)])
            A[np.ix_(idx, idx)] += blk
        return A, lift

    # ---- matrix-free operator, diagonal, mass, right-hand side
    def _nt(self, d):
        """Axes permutation of a cell array [k][j][i] to [normal][t2][t1]."""
        t1, t2 = [t for t in range(3) if t != d]
        return (2 - d, 2 - t2, 2 - t1)

    def _piece_groups(self):
        """Per normal axis and kind (interior / boundary): the pieces' cells and 1D factors as
        stacked arrays (built once)."""
        if getattr(self, "_groups", None) is not None:
            return self._groups
        groups = []
        for d in range(3):
            for interior in (True, False):
                sel = [pc for pc in self.pieces if pc[0] == d and (pc[3] >= 0) == interior]
                if not sel:
                    continue
                G = {"d": d, "interior": interior, "A": np.array([pc[1] for pc in sel]),
                     "sA": np.array([float(pc[2]) for pc in sel]), "B": np.array([pc[3] for pc in sel])}
                fa = [self._factors(pc[1], d, pc[2], pc[4], pc[5]) for pc in sel]
                G["vA"], G["dA"], G["I1A"], G["I2A"] = (np.array([f[i] for f in fa]) for i in range(4))
                G["W"] = np.array([np.outer(f[5], f[4]) for f in fa])
                G["sig"] = np.array([self.sigma(d, pc[1], pc[3]) for pc in sel])
                if interior:
                    fb = [self._factors(pc[3], d, -1, pc[4], pc[5]) for pc in sel]
                    G["vB"], G["dB"], G["I1B"], G["I2B"] = (np.array([f[i] for f in fb]) for i in range(4))
                groups.append(G)
        self._groups = groups
        return groups

    def apply(self, u):
        """y = A u for an element-major vector u."""
        n = self.n
        U = np.asarray(u, dtype=np.float64).reshape(-1, n, n, n)
        K1 = self.Dhat.T @ np.diag(self.w) @ self.Dhat
        w = self.w
        Jx, Jy, Jz = self.J[:, 0], self.J[:, 1], self.J[:, 2]
        Y = ((Jy * Jz / Jx)[:, None, None, None] * np.einsum("ia,ekja->ekji", K1, U) * w[None, None, :, None]
             * w[None, :, None, None]
             + (Jx * Jz / Jy)[:, None, None, None] * np.einsum("jb,ekbi->ekji", K1, U) * w[None, None, None, :]
             * w[None, :, None, None]
             + (Jx * Jy / Jz)[:, None, None, None] * np.einsum("kc,ecji->ekji", K1, U) * w[None, None, None, :]
             * w[None, None, :, None])
        for G in self._piece_groups():
            perm = (0,) + tuple(p + 1 for p in self._nt(G["d"]))
            inv = np.argsort(perm)
            Wq, sig, sA = G["W"], G["sig"][:, None, None], G["sA"][:, None, None]

            def face(V, Dn, I1, I2, cells):
                Ut = np.transpose(U[cells], perm)                       # [piece][normal][t2][t1]
                tr = np.einsum("pqa,pab,prb->pqr", I2, np.einsum("pn,pnab->pab", V, Ut), I1)
                dr = np.einsum("pqa,pab,prb->pqr", I2, np.einsum("pn,pnab->pab", Dn, Ut), I1)
                return tr, dr

            def back(V, Dn, I1, I2, cT, cD, sgn, cells):
                FT = np.einsum("pqa,pqr,prb->pab", I2, cT, I1)
                FD = np.einsum("pqa,pqr,prb->pab", I2, cD, I1)
                c = V[:, :, None, None] * FT[:, None] + sgn * Dn[:, :, None, None] * FD[:, None]
                np.add.at(Y, cells, np.transpose(c, inv))

            trA, drA = face(G["vA"], G["dA"], G["I1A"], G["I2A"], G["A"])
            if G["interior"]:
                trB, drB = face(G["vB"], G["dB"], G["I1B"], G["I2B"], G["B"])
                jmp, davg, half = trA - trB, 0.5 * (drA + drB), 0.5
            else:
                jmp, davg, half = trA, drA, 1.0
            # jmp: u_A - u_B (u_A on the boundary); davg: {du/dx_d}.  Seen from a side with
            # outward normal s e_d, its rows get sum_points W [(sigma [u] - {d_n u}) v - half [u] d_n v]
            # with [u] = +-jmp and {d_n u} = s davg.
            back(G["vA"], G["dA"], G["I1A"], G["I2A"], Wq * (sig * jmp - sA * davg), Wq * (-half * jmp),
                 sA[:, None], G["A"])
            if G["interior"]:
                # B lies above A: outward normal -e_d, [u] = -jmp, {d_n u} = -davg
                back(G["vB"], G["dB"], G["I1B"], G["I2B"], Wq * (-sig * jmp + davg), Wq * (half * jmp),
                     -1.0, G["B"])
        return Y.reshape(-1)

    def diagonal(self):
        n = self.n
        K1d = np.diag(self.Dhat.T @ np.diag(self.w) @ self.Dhat)
        w = self.w
        Jx, Jy, Jz = self.J[:, 0], self.J[:, 1], self.J[:, 2]
        D = ((Jy * Jz / Jx)[:, None, None, None] * (w[:, None, None] * w[None, :, None] * K1d[None, None, :])[None]
             + (Jx * Jz / Jy)[:, None, None, None] * (w[:, None, None] * K1d[None, :, None] * w[None, None, :])[None]
             + (Jx * Jy / Jz)[:, None, None, None] * (K1d[:, None, None] * w[None, :, None] * w[None, None, :])[None])
        D = D.copy()
        for (d, Ae, sA, Be, t1iv, t2iv) in self.pieces:
            perm = self._nt(d)
            inv = np.argsort(perm)
            sig = self.sigma(d, Ae, Be)
            kappa = 2.0 if Be < 0 else 1.0
            sides = [(Ae, sA)] + ([(Be, -1)] if Be >= 0 else [])
            for (e, s) in sides:
                vn, dn, I1, I2, w1, w2 = self._factors(e, d, s, t1iv, t2iv)
                S1 = (w1[:, None] * I1 ** 2).sum(0)
                S2 = (w2[:, None] * I2 ** 2).sum(0)
                nrm = sig * vn ** 2 - kappa * vn * (s * dn)
                D[e] += np.transpose(nrm[:, None, None] * S2[None, :, None] * S1[None, None, :], inv)
        return D.reshape(-1)

    def mass(self):
        w = self.w
        W3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
        return (np.prod(self.J, axis=1)[:, None, None, None] * W3[None]).reshape(-1)

    def nodes(self):
        """X, Y, Z of every node, element-major."""
        n = self.n
        out = np.empty((3, len(self.cells), n, n, n))
        for e in range(len(self.cells)):
            x = [self.a[e, d] + self.J[e, d] * (self.xi + 1.0) for d in range(3)]
            Z, Yg, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
            out[0, e], out[1, e], out[2, e] = X, Yg, Z
        return out[0].reshape(-1), out[1].reshape(-1), out[2].reshape(-1)

    def boundary_points(self):
        """X, Y, Z of the Dirichlet points: boundary pieces in order, each [t2][t1]."""
        pts = []
        for (d, Ae, sA, _, t1iv, t2iv) in self.boundary:
            t1, t2 = [t for t in range(3) if t != d]
            x1 = t1iv[0] + 0.5 * (t1iv[1] - t1iv[0]) * (self.xi + 1.0)
            x2 = t2iv[0] + 0.5 * (t2iv[1] - t2iv[0]) * (self.xi + 1.0)
            G2, G1 = np.meshgrid(x2, x1, indexing="ij")
            P = [None, None, None]
            P[d] = np.full(G1.shape, self.a[Ae, d] if sA < 0 else self.b[Ae, d])
            P[t1], P[t2] = G1, G2
            pts.append(np.stack([p.reshape(-1) for p in P]))
        if not pts:
            return np.zeros(0), np.zeros(0), np.zeros(0)
        allp = np.concatenate(pts, axis=1)
        return allp[0], allp[1], allp[2]

    def boundary_data(self, f, chunk=256):
        """Dirichlet data by quadrature (Sec. 6.3): g(r) = sum_q W_q f(x_q) / |r - x_q| at the
        ``boundary_points``, W_q the physical GL weight of node q (``mass``).  With GL nodes no
        node lies on the boundary, so every term is finite.  f: [..., ndof]; returns [..., nb]."""
        f = np.asarray(f, dtype=np.float64)
        lead = f.shape[:-1]
        F = (self.mass() * f.reshape(-1, self.ndof)).T                 # [ndof, S]
        xq = np.stack(self.nodes(), axis=1)                             # [ndof, 3]
        pts = np.stack(self.boundary_points(), axis=1)                  # [nb, 3]
        out = np.empty((pts.shape[0], F.shape[1]))
        for s in range(0, pts.shape[0], chunk):
            d = np.sqrt(np.sum((pts[s:s + chunk, None, :] - xq[None, :, :]) ** 2, axis=-1))
            out[s:s + chunk] = (1.0 / d) @ F
        return out.T.reshape(lead + (pts.shape[0],))

    def rhs(self, f, g):
        """b = 4 pi M f + boundary lift of g (f at the nodes, g at ``boundary_points``)."""
        n = self.n
        b = 4.0 * np.pi * self.mass() * np.asarray(f, dtype=np.float64)
        B = b.reshape(-1, n, n, n)
        g = np.asarray(g, dtype=np.float64)
        for k, (d, Ae, sA, _, t1iv, t2iv) in enumerate(self.boundary):
            perm = self._nt(d)
            inv = np.argsort(perm)
            vA, dA, I1, I2, w1, w2 = self._factors(Ae, d, sA, t1iv, t2iv)
            cg = np.outer(w2, w1) * g[k * n * n:(k + 1) * n * n].reshape(n, n)
            sig = self.sigma(d, Ae, -1)
            FT = I2.T @ cg @ I1
            B[Ae] += np.transpose((sig * vA - sA * dA)[:, None, None] * FT[None], inv)
        return B.reshape(-1)


def degree_transfer(mf, mc):
    """Per-element interpolation from degree mc.q to mf.q on the same cells (matrix n_f^3 x n_c^3)."""
    I = _nodes.lagrange_eval(mc.xi, mf.xi)
    return np.kron(I, np.kron(I, I))


def mesh_transfer(tree, mf, mc):
    """For each fine cell: (coarse cell index, per-axis interpolation matrices [Ix, Iy, Iz]) --
    the cell itself when it is in both meshes, else its parent (split once between them)."""
    index = {(c.lv, c.ix): e for e, c in enumerate(mc.cells)}
    parent = {}
    for e, cc in enumerate(mc.cells):
        for k in cc.children:
            parent[(k.lv, k.ix)] = e
    out = []
    for c in mf.cells:
        key = (c.lv, c.ix)
        ce = index[key] if key in index else parent[key]
        cc = mc.cells[ce]
        mats = []
        for d in range(3):
            k = c.lv[d] - cc.lv[d]                     # 0: same extent, 1: one half of the parent
            j = c.ix[d] - (cc.ix[d] << k)
            mats.append(_nodes.lagrange_eval(mc.xi, -1.0 + (2.0 * j + 1.0 + mf.xi) / 2.0 ** k))
        out.append((ce, mats))
    return out


class Hierarchy(_mg.Hierarchy):
    """Levels of the octree MG (degree steps on the leaves, then mesh steps) with the
    smoother, Lanczos bounds and V-cycle of ``mg.Hierarchy``."""

    def __init__(self, tree, degree=6, ratio=60.0, safety=1.1, lanczos_steps=30, degree_h=10,
                 eps=_sipdg.PENALTY_EPS):
        self.tree = tree
        specs = [(None, tree.q)]
        while specs[-1][1] > 1:
            specs.append((None, specs[-1][1] // 2))
        for g in range(tree.max_gen - 1, -1, -1):
            specs.append((g, 1))
        self.specs = specs
        self.meshes = [Mesh(tree, tree.cells(g), q, eps) for g, q in specs]
        self.levels = []
        for m in self.meshes:
            lvl = _OctLevel(m)
            self.levels.append(lvl)
        self.transfers = []
        for (gf, qf), (gc, qc), mf, mc in zip(specs[:-1], specs[1:], self.meshes[:-1], self.meshes[1:]):
            if qf != qc:
                self.transfers.append(("deg", degree_transfer(mf, mc)))
            else:
                self.transfers.append(("mesh", mesh_transfer(tree, mf, mc)))
        self.degree = degree
        self.degrees = [degree_h if (l >= 1 and q == 1 and degree_h > 0) else degree
                        for l, (_, q) in enumerate(specs)]
        base = tree.mesh(0, 1)
        assert len(base.cells) == len(tree.roots)
        self.coarse_axes = _sipdg.make_axes(tree.E, 1, tree.lo, tree.hi, eps, "gl")
        self.coarse = _Coarse(FDM(self.coarse_axes), tree.E)
        self.lam = []
        for L in self.levels[:-1]:
            v0 = _mg.hash_vector(L.ndof)
            dm = 1.0 / np.sqrt(L.D)
            lmax = _mg.lanczos_max(lambda v: dm * L.A(dm * v), v0, min(lanczos_steps, L.ndof))
            hi_ = safety * lmax
            self.lam.append((hi_ / ratio, hi_))

    def prolong(self, l, uc):
        kind, T = self.transfers[l]
        mf, mc = self.meshes[l], self.meshes[l + 1]
        nf, nc = mf.n, mc.n
        Uc = np.asarray(uc).reshape(-1, nc ** 3)
        if kind == "deg":
            return (Uc @ T.T).reshape(-1)
        out = np.empty((len(mf.cells), nf ** 3))
        for e, (ce, (Ix, Iy, Iz)) in enumerate(T):
            out[e] = np.kron(Iz, np.kron(Iy, Ix)) @ Uc[ce]
        return out.reshape(-1)

    def restrict(self, l, rf):
        kind, T = self.transfers[l]
        mf, mc = self.meshes[l], self.meshes[l + 1]
        nf, nc = mf.n, mc.n
        Rf = np.asarray(rf).reshape(-1, nf ** 3)
        if kind == "deg":
            return (Rf @ T).reshape(-1)
        out = np.zeros((len(mc.cells), nc ** 3))
        for e, (ce, (Ix, Iy, Iz)) in enumerate(T):
            out[ce] += np.kron(Iz, np.kron(Iy, Ix)).T @ Rf[e]
        return out.reshape(-1)


def exchange(mesh, psi, g_pairs, solve):
    """Exchange on the octree grid (Sec. 6.1 on the auxiliary mesh of Sec. 6.2): for the pair
    densities rho_ij = psi_i psi_j (i <= j, row-major pair order) solve for v_ij with Dirichlet data
    g_pairs[k]; W_k = sum_s psi_s v_ks (pointwise); K_ij = sum_q W_q rho_ij v_ij (the grid's GL
    quadrature); E_X = sum over ordered pairs.  Returns (v, W, K, E_X)."""
    n = len(psi)
    w = mesh.mass()
    pairs = [(i, j) for i in range(n) for j in range(i, n)]

    def idx(i, j):
        i, j = min(i, j), max(i, j)
        return i * n - i * (i - 1) // 2 + (j - i)
    rho = [psi[i] * psi[j] for i, j in pairs]
    v = [solve(mesh.rhs(r, g)) for r, g in zip(rho, g_pairs)]
    K = np.array([float(np.sum(w * r * vv)) for r, vv in zip(rho, v)])
    W = [sum(psi[s] * v[idx(k, s)] for s in range(n)) for k in range(n)]
    EX = float(sum((1.0 if i == j else 2.0) * K[q] for q, (i, j) in enumerate(pairs)))
    return v, W, K, EX


class _Coarse:
    """Exact solve on the uniform base mesh at degree 1 (fast diagonalisation), element-major."""

    def __init__(self, fdm, E):
        self.fdm, self.E = fdm, E

    def solve(self, f):
        return to_element_major(self.fdm.solve(to_global(f, self.E, 2)), self.E, 2)


class _OctLevel:
    def __init__(self, mesh):
        self.mesh = mesh
        self.ndof = mesh.ndof
        self.D = mesh.diagonal()
        self.shape = self.D.shape

    def A(self, u):
        return self.mesh.apply(u)
