"""The five synthetic workloads, as closed-form sources on a uniform auxiliary mesh.

Every workload is a mesh description plus closed-form sources.  Callers sample
them at their own node and boundary-face coordinates, so the GPU library and
the CPU oracle each use coordinates they computed themselves.

Workloads (all seeded with numpy.random.default_rng):

* ``single``      4x4x4 elements, p=3, box [-5,5]^3; rho = normalised Gaussian
                  of exponent 2.0 at the origin plus one of exponent 0.5 at
                  (1,0,0); 2 multigrid levels; tolerance 1e-10.
* ``exchange8``   16x16x16 elements, p=4, box [-8,8]^3; 8 atoms uniform in
                  [-4,4]^3, 3 s primitives per atom with exponents log-uniform
                  in [0.3,10], 8 orbitals from N(0,1) coefficients,
                  Loewdin-orthonormalised with the analytic overlap; all 36 pair
                  densities; 4 levels; tolerance 1e-8.  (seed 2)
* ``exchange16``  same mesh and atoms, 16 orbitals, 136 pairs.  (seed 3)
* ``uneven``      256 densities split 86/85/85 over 8^3, 12^3, 16^3 element
                  meshes (p=4, box [-E/2, E/2]^3); each density a sum of 2..12
                  normalised Gaussians (exponents log-uniform in [0.3,10],
                  weights U[0.5,1.5], centres uniform in [-E/4, E/4]^3).  (seed 4)
* ``octree``      the exchange8 molecule on an adaptive octree auxiliary mesh:
                  8x8x8 base elements on [-8,8]^3, degree q=4 Gauss-Legendre,
                  refined on the electron density sum_k psi_k^2 with
                  delta_q = 1e-8 (the paper's tolerance) and at most 3
                  refinements per base element; all 36 pair densities as
                  right-hand sides, Dirichlet data from their closed-form
                  potentials; tolerance 1e-8.  (seed 2)
* ``large``       32x32x32 elements, p=4, box [-16,16]^3; molecules of 16..32
                  atoms in [-8,8]^3 with the exchange8 primitive recipe,
                  8 orbitals, 36 pairs per molecule.  (seed 50000+i train,
                  90000+i held out)
"""
import numpy as np

from .gaussians import GaussianDensity, Orbitals, Primitives, lowdin

ALPHA_LO, ALPHA_HI = 0.3, 10.0


class Mesh:
    def __init__(self, E, p, lo, hi):
        self.E = tuple(int(e) for e in E)
        self.p = int(p)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)

    def __repr__(self):
        return f"Mesh(E={self.E}, p={self.p}, lo={self.lo}, hi={self.hi})"


def cube(E, p, half):
    return Mesh((E, E, E), p, (-half,) * 3, (half,) * 3)


class DensityBatch:
    """Independent densities with closed-form potentials (one Poisson RHS each)."""

    def __init__(self, densities, mesh_ids=None):
        self.densities = list(densities)
        self.mesh_ids = list(mesh_ids) if mesh_ids is not None else [0] * len(self.densities)

    def __len__(self):
        return len(self.densities)

    def rho(self, k, X, Y, Z):
        return self.densities[k].density(X, Y, Z)

    def potential(self, k, X, Y, Z):
        return self.densities[k].potential(X, Y, Z)


class Workload:
    def __init__(self, name, meshes, n_levels, rtol, batch=None, orbitals=None):
        self.name = name
        self.meshes = meshes
        self.n_levels = n_levels
        self.rtol = rtol
        self.batch = batch
        self.orbitals = orbitals


def _log_uniform(rng, n):
    return np.exp(rng.uniform(np.log(ALPHA_LO), np.log(ALPHA_HI), size=n))


def _atoms_and_pool(rng, n_atoms, box_half, per_atom=3):
    atoms = rng.uniform(-box_half, box_half, size=(n_atoms, 3))
    alpha = _log_uniform(rng, n_atoms * per_atom)
    centres = np.repeat(atoms, per_atom, axis=0)
    return atoms, Primitives(alpha, centres)


def _orbitals(rng, prims, norb):
    C = rng.standard_normal((len(prims), norb))
    return Orbitals(prims, lowdin(C, prims.overlap()))


def single():
    dens = GaussianDensity([1.0, 1.0], [2.0, 0.5], [[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    return Workload("single", [cube(4, 3, 5.0)], 2, 1e-10, batch=DensityBatch([dens]))


def exchange8(norb=8, seed=2):
    rng = np.random.default_rng(2)
    _, prims = _atoms_and_pool(rng, 8, 4.0)
    orng = rng if seed == 2 else np.random.default_rng(seed)
    return Workload(f"exchange{norb}", [cube(16, 4, 8.0)], 4, 1e-8,
                    orbitals=_orbitals(orng, prims, norb))


def exchange16():
    return exchange8(norb=16, seed=3)


def uneven(n_rhs=256, seed=4):
    rng = np.random.default_rng(seed)
    Es = (8, 12, 16)
    meshes = [cube(E, 4, E / 2.0) for E in Es]
    perm = rng.permutation(n_rhs)
    counts = [n_rhs - 2 * (n_rhs // 3), n_rhs // 3, n_rhs // 3]
    mesh_of = np.empty(n_rhs, dtype=int)
    start = 0
    for m, c in enumerate(counts):
        mesh_of[perm[start:start + c]] = m
        start += c
    dens = []
    for k in range(n_rhs):
        E = Es[mesh_of[k]]
        K = int(rng.integers(2, 13))
        dens.append(GaussianDensity(rng.uniform(0.5, 1.5, K), _log_uniform(rng, K),
                                    rng.uniform(-E / 4.0, E / 4.0, size=(K, 3))))
    return Workload("uneven", meshes, 4, 1e-8, batch=DensityBatch(dens, mesh_of))


def octree():
    """The octree workload: base mesh, refinement parameters and the molecule's orbitals; the
    refinement density is ``density`` (the electron density of the occupied orbitals)."""
    wl = exchange8()
    wl.name = "octree"
    wl.meshes = [cube(8, 4, 8.0)]
    wl.n_levels = None
    wl.delta_q, wl.max_depth = 1e-8, 3
    orb = wl.orbitals

    def density(x, y, z):
        v = np.asarray(orb.values(x, y, z))
        return (v * v).sum(axis=0)
    wl.density = density
    return wl


def large_molecule(index, held_out=False, norb=8):
    seed = (90000 if held_out else 50000) + index
    rng = np.random.default_rng(seed)
    n_atoms = int(rng.integers(16, 33))
    _, prims = _atoms_and_pool(rng, n_atoms, 8.0)
    return Workload("large", [cube(32, 4, 16.0)], 5, 1e-8, orbitals=_orbitals(rng, prims, norb))


def scaled(E, p, n_rhs, seed=7, n_levels=None, rtol=1e-8):
    """A density batch on an arbitrary cube mesh with h = 1 (tests and sweeps)."""
    rng = np.random.default_rng(seed)
    dens = []
    for _ in range(n_rhs):
        K = int(rng.integers(2, 6))
        dens.append(GaussianDensity(rng.uniform(0.5, 1.5, K), _log_uniform(rng, K),
                                    rng.uniform(-E / 4.0, E / 4.0, size=(K, 3))))
    return Workload(f"scaled{E}p{p}", [cube(E, p, E / 2.0)], n_levels, rtol, batch=DensityBatch(dens))


BY_NAME = {"single": single, "exchange8": exchange8, "exchange16": exchange16, "uneven": uneven}
