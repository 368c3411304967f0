"""Pins of the octree oracle (adaptive auxiliary mesh, hanging-face SIPDG, hp + geometric MG)
against what the paper and the mathematics fix.

* Unrefined: the octree matrix and right-hand side are exactly the Kronecker-sum problem of
  ``sipdg`` with Gauss-Legendre nodes (itself pinned to the element-by-element assembly).
* Hanging faces: SIPDG is consistent, so a polynomial of the element degree that solves the PDE
  is reproduced exactly by the discrete solve, whatever the mesh; the matrix is symmetric
  positive definite; the solution error falls at high order on a refined mesh.
* The matrix-free operator, its diagonal and the boundary lift equal the dense assembly.
* Refinement (Sec. 6.2): the aspect-ratio rule gives 2, 4 or 8 children; a density the GL rule
  integrates exactly is never refined; a sharp density is refined where it is sharp; every
  split had Q > delta_q and every leaf below the depth cap has Q <= delta_q (brute force);
  the leaves tile the box.
* Multigrid (Sec. 6.4): transfers reproduce polynomials of the coarse space exactly; MG-PCG
  converges to the dense solution in few iterations.
"""
import numpy as np
import pytest

from oracle import layout, octree, pcg, sipdg


def _poly(x, y, z):
    """A polynomial of degree <= 3 in each variable, and minus its Laplacian over 4 pi."""
    u = 1.0 + x * x * y - 0.5 * z ** 3 + x * y * z + 0.3 * y ** 3 - x
    lap = 2.0 * y - 3.0 * z + 1.8 * y
    return u, -lap / (4.0 * np.pi)


def _hanging_tree(q=3, E=(2, 2, 1), lo=(-1.0, -1.0, -0.5), hi=(1.0, 1.0, 0.5)):
    """Base cells of aspect 2:2:1 (isotropic split into 8); one refined twice (a 2-level jump
    against its neighbours), one refined once."""
    def manual(c):
        return (c.gen == 0 and c.ix in ((0, 0, 0), (1, 1, 0))) or (c.gen == 1 and c.ix == (1, 1, 1))
    return octree.Octree(E, lo, hi, q, manual=manual, max_depth=2)


def test_unrefined_mesh_is_the_kronecker_sum_with_gl_nodes():
    E, q, lo, hi = (2, 3, 2), 3, (-1.0, 0.0, -2.0), (1.5, 2.0, 1.0)
    tree = octree.Octree(E, lo, hi, q)
    m = tree.mesh()
    assert len(m.cells) == 12 and all(c.gen == 0 for c in m.cells)
    A, _ = m.dense()
    axes = sipdg.make_axes(E, q, lo, hi, family="gl")
    K = sipdg.dense_matrix(axes)
    em_at = layout.to_global(np.arange(m.ndof), E, q + 1).reshape(-1)   # global position -> em index
    P = np.zeros((m.ndof, m.ndof))
    P[np.arange(m.ndof), em_at] = 1.0                                    # u_global = P u_em
    Kem = P.T @ K @ P
    assert np.abs(A - Kem).max() <= 1e-12 * np.abs(K).max()
    # right-hand side with a smooth source and boundary data
    X, Y, Z = m.nodes()
    f = np.cos(X) * np.exp(0.3 * Y) + Z
    gx, gy, gz = m.boundary_points()
    g = np.sin(gx + 2 * gy) - gz
    b = m.rhs(f, g)
    Xg, Yg, Zg = np.broadcast_arrays(*sipdg.node_grid(axes))
    faces = [np.sin(fp[0] + 2 * fp[1]) - fp[2] for fp in sipdg.face_points(axes)]
    bk = sipdg.rhs(axes, np.cos(Xg) * np.exp(0.3 * Yg) + Zg, faces)
    assert np.abs(b - layout.to_element_major(bk, E, q + 1)).max() <= 1e-12 * np.abs(bk).max()


def test_hanging_mesh_structure():
    tree = _hanging_tree()
    m = tree.mesh()
    gens = [c.gen for c in m.cells]
    assert gens.count(0) == 2 and gens.count(1) == 15 and gens.count(2) == 8
    # the leaves tile the box
    vol = np.prod(m.b - m.a, axis=1).sum()
    assert abs(vol - 2.0 * 2.0 * 1.0) < 1e-13
    # every face of every cell is covered exactly by its pieces
    area = np.zeros((len(m.cells), 6))
    for (d, A, sA, B, t1, t2) in m.pieces:
        ar = (t1[1] - t1[0]) * (t2[1] - t2[0])
        area[A, 2 * d + (sA > 0)] += ar
        if B >= 0:
            area[B, 2 * d] += ar
    for e in range(len(m.cells)):
        ext = m.b[e] - m.a[e]
        for d in range(3):
            t = [ext[t] for t in range(3) if t != d]
            assert np.allclose(area[e, 2 * d:2 * d + 2], t[0] * t[1], rtol=1e-13)
    # a 2-level jump exists (a generation-2 cell against a generation-0 cell)
    jumps = [abs(m.cells[A].gen - m.cells[B].gen) for (_, A, _, B, _, _) in m.pieces if B >= 0]
    assert max(jumps) == 2


@pytest.mark.parametrize("q", [1, 2, 3])
def test_matrix_free_operator_diagonal_and_lift_equal_the_dense_assembly(q):
    tree = _hanging_tree(q=q)
    m = tree.mesh()
    A, lift = m.dense(g=np.cos(np.arange(len(m.boundary) * (q + 1) ** 2)))
    rng = np.random.default_rng(3)
    u = rng.standard_normal(m.ndof)
    assert np.abs(m.apply(u) - A @ u).max() <= 1e-12 * np.abs(A @ u).max()
    assert np.abs(m.diagonal() - np.diag(A)).max() <= 1e-12 * np.abs(np.diag(A)).max()
    g = np.cos(np.arange(len(m.boundary) * (q + 1) ** 2))
    f = rng.standard_normal(m.ndof)
    b = m.rhs(f, g)
    assert np.abs(b - (4 * np.pi * m.mass() * f + lift)).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("q", [3, 4])
def test_hanging_faces_reproduce_a_polynomial_solution(q):
    tree = _hanging_tree(q=q)
    m = tree.mesh()
    A, _ = m.dense()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0.0
    X, Y, Z = m.nodes()
    u, f = _poly(X, Y, Z)
    gx, gy, gz = m.boundary_points()
    g, _ = _poly(gx, gy, gz)
    v = np.linalg.solve(A, m.rhs(f, g))
    assert np.abs(v - u).max() <= 1e-9 * np.abs(u).max()


def test_a_wrong_hanging_face_term_breaks_reproduction():
    """Dropping the penalty's hanging-face factor (sigma of the larger cell) still reproduces the
    polynomial (consistency does not depend on sigma), but dropping the interpolation of the
    coarse side (using its nodal trace as if conforming) does not: the pin sees such a slip."""
    tree = _hanging_tree(q=3)
    m = tree.mesh()
    X, Y, Z = m.nodes()
    u, f = _poly(X, Y, Z)
    gx, gy, gz = m.boundary_points()
    g, _ = _poly(gx, gy, gz)
    b = m.rhs(f, g)
    good = m.apply(u) - b
    assert np.abs(good).max() <= 1e-10 * np.abs(b).max()
    orig = m._factors

    def conforming_only(e, d, s, t1iv, t2iv):
        vn, dn, I1, I2, w1, w2 = orig(e, d, s, t1iv, t2iv)
        return vn, dn, np.eye(len(vn)), np.eye(len(vn)), w1, w2
    m._factors = conforming_only
    m._groups = None
    bad = m.apply(u) - b
    assert np.abs(bad).max() > 1e-3 * np.abs(b).max()


def test_aspect_ratio_rule_gives_2_4_or_8_children():
    tree = octree.Octree((1, 1, 1), (0, 0, 0), (1, 1, 1), 2)
    c = tree.roots[0]
    assert len(tree.children_of(c)) == 8
    t2 = octree.Octree((1, 1, 1), (0, 0, 0), (4, 1, 1), 2)      # Ly, Lz < L/2: only x
    assert t2.split_axes(t2.roots[0]) == [0] and len(t2.children_of(t2.roots[0])) == 2
    t3 = octree.Octree((1, 1, 1), (0, 0, 0), (3, 3, 1), 2)      # Lz < L/2: x and y
    assert t3.split_axes(t3.roots[0]) == [0, 1] and len(t3.children_of(t3.roots[0])) == 4
    t4 = octree.Octree((1, 1, 1), (0, 0, 0), (2, 1, 1), 2)      # Ly = L/2 is not below L/2
    assert len(t4.children_of(t4.roots[0])) == 8
    # after one x split of the 4:1:1 cell the children are 2:1:1 and split into 8
    k = t2.children_of(t2.roots[0])[0]
    assert len(t2.children_of(k)) == 8


def test_exactly_integrated_density_is_not_refined():
    q = 4
    tree = octree.Octree((2, 2, 2), (-1, -1, -1), (1, 1, 1), q,
                         rho=lambda x, y, z: (1 + 0.3 * x) ** 9 * (1 - 0.2 * y) ** 9 + 0.5 * z ** 9, delta_q=1e-10)
    assert tree.max_gen == 0 and tree.tested == 8


def _gauss(a, c):
    return lambda x, y, z: np.exp(-a * ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2))


def test_refinement_follows_the_indicator_brute_force():
    q, delta, depth = 2, 1e-5, 4
    rho = _gauss(40.0, (0.3, -0.2, 0.1))
    tree = octree.Octree((2, 2, 2), (-1.5, -1.5, -1.5), (1.5, 1.5, 1.5), q, rho=rho, delta_q=delta, max_depth=depth)
    assert tree.max_gen >= 2
    leaves = tree.cells()

    def walk(c):
        yield c
        for k in c.children:
            yield from walk(k)
    for r in tree.roots:
        for c in walk(r):
            Q = tree.indicator(c, tree.children_of(c), rho)
            if c.children:
                assert Q > delta
            elif c.gen < depth:
                assert Q <= delta
    # refined where the density is sharp: the deepest leaves hold the centre
    a = np.array([tree.bounds(c)[0] for c in leaves])
    b = np.array([tree.bounds(c)[1] for c in leaves])
    deep = [i for i, c in enumerate(leaves) if c.gen == tree.max_gen]
    ctr = np.array([0.3, -0.2, 0.1])
    assert min(np.linalg.norm(0.5 * (a[i] + b[i]) - ctr) for i in deep) < 0.5
    far = [i for i, c in enumerate(leaves) if np.linalg.norm(0.5 * (a[i] + b[i]) - ctr) > 1.6]
    assert far and all(leaves[i].gen <= 1 for i in far)
    # the leaves tile the box
    assert abs(np.prod(b - a, axis=1).sum() - 27.0) < 1e-12
    # the GL rule on the leaves integrates the density to about delta per refined cell
    exact = (np.pi / 40.0) ** 1.5   # the Gaussian lies well inside the box
    tot = sum(tree.integral(c, rho) for c in leaves)
    assert abs(tot - exact) < 50 * delta


def test_transfers_reproduce_coarse_polynomials():
    tree = _hanging_tree(q=4)
    H = octree.Hierarchy(tree)
    assert [s for s in H.specs] == [(None, 4), (None, 2), (None, 1), (1, 1), (0, 1)]
    for l in range(len(H.meshes) - 1):
        mf, mc = H.meshes[l], H.meshes[l + 1]
        pc = mc.q

        def poly(x, y, z):
            return (1 + x ** pc) * (2 - y) ** pc + z ** pc * x
        Xc, Yc, Zc = mc.nodes()
        Xf, Yf, Zf = mf.nodes()
        got = H.prolong(l, poly(Xc, Yc, Zc))
        assert np.abs(got - poly(Xf, Yf, Zf)).max() <= 1e-12, l
        # R = P^T
        rng = np.random.default_rng(l)
        a, bb = rng.standard_normal(mc.ndof), rng.standard_normal(mf.ndof)
        assert abs(H.prolong(l, a) @ bb - a @ H.restrict(l, bb)) <= 1e-12 * np.abs(a).sum() * np.abs(bb).max() * 10


def test_octree_mg_pcg_converges_to_the_dense_solution():
    tree = octree.Octree((2, 2, 2), (-2, -2, -2), (2, 2, 2), 4, rho=_gauss(10.0, (0.4, 0.2, -0.3)),
                         delta_q=1e-4, max_depth=2)
    assert tree.max_gen == 2
    H = octree.Hierarchy(tree)
    m = H.meshes[0]
    X, Y, Z = m.nodes()
    f = _gauss(10.0, (0.4, 0.2, -0.3))(X, Y, Z)
    gx, gy, gz = m.boundary_points()
    b = m.rhs(f, 0.1 * np.cos(gx) * gy)
    x, it, rel, _ = pcg.pcg(H.levels[0].A, b, H.vcycle, rtol=1e-10)
    assert rel <= 1e-10 and it <= 60
    if m.ndof <= 6000:
        A, _ = m.dense()
        ref = np.linalg.solve(A, b)
        assert np.abs(x - ref).max() <= 1e-8 * np.abs(ref).max()


def test_error_falls_at_high_order_on_a_hanging_mesh():
    """A smooth non-polynomial solution u = exp(-a r^2) (f = -Lap u / 4 pi, g = u): on the same
    hanging mesh the nodal error at degree 4 is far below the one at degree 2."""
    a = 1.5

    def exact(x, y, z):
        r2 = x * x + y * y + z * z
        u = np.exp(-a * r2)
        return u, -(4 * a * a * r2 - 6 * a) * u / (4 * np.pi)
    errs = []
    for q in (2, 4):
        m = _hanging_tree(q=q).mesh()
        X, Y, Z = m.nodes()
        u, f = exact(X, Y, Z)
        gx, gy, gz = m.boundary_points()
        g, _ = exact(gx, gy, gz)
        A, _ = m.dense()
        errs.append(np.abs(np.linalg.solve(A, m.rhs(f, g)) - u).max())
    assert errs[0] < 0.1 and errs[1] < errs[0] / 10   # measured 4.9e-2 and 2.2e-3


def test_boundary_data_by_quadrature_brute_force_and_closed_form():
    """Sec. 6.3's Dirichlet data on the octree grid: the vectorised sum equals explicit loops over
    every boundary point and node with weights built here from the GL rule; for a Gaussian well
    inside the box the data approach the closed-form potential erf(sqrt(a) r)/r, and refining
    the mesh around the Gaussian (the octree's purpose) brings them closer."""
    from scipy.special import erf
    from oracle import nodes
    a, c = 8.0, np.array([0.2, -0.1, 0.15])

    def rho(x, y, z):
        return (a / np.pi) ** 1.5 * np.exp(-a * ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2))
    tree = octree.Octree((2, 1, 1), (-2.0, -1.0, -1.0), (2.0, 1.0, 1.0), 2, manual=lambda cl: cl.gen == 0 and
                         cl.ix == (1, 0, 0), max_depth=1)
    m = tree.mesh()
    f = rho(*m.nodes())
    g = m.boundary_data(f)
    xi, w = nodes.gl(2)[:2]
    bx, by, bz = m.boundary_points()
    ref = np.zeros_like(g)
    for e in range(len(m.cells)):
        lo, hi = m.a[e], m.b[e]
        for k in range(3):
            for j in range(3):
                for i in range(3):
                    x = [lo[d] + 0.5 * (hi[d] - lo[d]) * (xi[(i, j, k)[d]] + 1.0) for d in range(3)]
                    W = np.prod([0.5 * (hi[d] - lo[d]) * w[(i, j, k)[d]] for d in range(3)])
                    fq = rho(*x)
                    for p in range(len(bx)):
                        ref[p] += W * fq / np.sqrt((bx[p] - x[0]) ** 2 + (by[p] - x[1]) ** 2 + (bz[p] - x[2]) ** 2)
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()
    # against the closed form, coarse and refined around the Gaussian
    errs = []
    for depth in (0, 3):
        t = octree.Octree((2, 2, 2), (-3.0,) * 3, (3.0,) * 3, 4, rho=rho, delta_q=1e-6, max_depth=depth)
        mm = t.mesh()
        gg = mm.boundary_data(rho(*mm.nodes()))
        px, py, pz = mm.boundary_points()
        r = np.sqrt((px - c[0]) ** 2 + (py - c[1]) ** 2 + (pz - c[2]) ** 2)
        exact = erf(np.sqrt(a) * r) / r
        errs.append(np.abs(gg - exact).max() / np.abs(exact).max())
    assert errs[1] < 3e-6 and errs[1] < errs[0] / 1e4     # measured 0.10 (8 cells) and 1.2e-6 (155 cells)


def test_exchange_on_an_unrefined_octree_equals_the_uniform_gl_exchange():
    """W_k, K_ij and E_x on the octree grid: with no refinement the problem is the uniform GL
    mesh's, so they equal the uniform exchange oracle's (exact solves on both sides)."""
    from oracle import exchange as uex, fdm, layout
    from workloads import gaussians
    E, q, lo, hi = (3, 2, 2), 3, (-3.0, -2.5, -2.0), (3.0, 2.5, 2.0)
    prims = gaussians.Primitives([0.9, 1.6, 0.7], [[0.3, 0.1, 0.0], [-0.4, 0.0, 0.2], [0.1, -0.3, -0.1]])
    orb = gaussians.Orbitals(prims, gaussians.lowdin(np.array([[1.0, 0.3], [0.2, -1.0], [0.5, 0.4]]),
                                                     prims.overlap()))
    m = octree.Octree(E, lo, hi, q).mesh()
    A, _ = m.dense()
    X, Y, Z = m.nodes()
    psi = list(orb.values(X, Y, Z))
    bx, by, bz = m.boundary_points()
    g = orb.pair_potentials(bx, by, bz)
    v, W, K, EX = octree.exchange(m, psi, list(g), lambda b: np.linalg.solve(A, b))
    axes = sipdg.make_axes(E, q, lo, hi, family="gl")
    Xg, Yg, Zg = np.broadcast_arrays(*sipdg.node_grid(axes))
    psig = list(orb.values(Xg, Yg, Zg))
    fp = sipdg.face_points(axes)
    gp = [[orb.pair_potentials(*fp[f])[k] for f in range(6)] for k in range(len(g))]
    vu, Wu, Ku, EXu = uex.exchange(axes, psig, gp, fdm.FDM(axes).solve)
    assert np.abs(K - Ku).max() <= 1e-11 * np.abs(Ku).max()
    assert abs(EX - EXu) <= 1e-11 * abs(EXu)
    for k in range(len(W)):
        Wg = layout.to_element_major(Wu[k], E, q + 1)
        assert np.abs(W[k] - Wg).max() <= 1e-10 * np.abs(Wg).max()
