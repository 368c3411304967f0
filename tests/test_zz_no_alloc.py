"""The entry point that allocates nothing (dg_boundary_data_noalloc) against dg_boundary_data.

Both compute the Dirichlet data by quadrature of the same sources; the fixed
work space makes the no-allocation entry take narrower source tiles and fewer
split parts, so the two differ only by the order of the partial sums (FP64
rounding).  Two calls in a row share the GPU's fixed array: the second, on a
smaller mesh with fewer sources, must not see the first one's leftovers.
"""
import numpy as np
import pytest

from workloads import configs

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b, nsrc):
    a, b = a.reshape(nsrc, -1), b.reshape(nsrc, -1)
    return max(float(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()) for k in range(nsrc))


def test_no_alloc_entry_matches_boundary_data_on_two_calls(gpu_lib):
    import torch
    wl = configs.exchange8()
    big = wl.meshes[0]                                           # 16^3 elements, p = 4: 512,000 nodes
    small = configs.Mesh((5, 4, 6), 3, (-2.5, -2.0, -3.0), (2.5, 2.0, 3.0))
    ctx = gpu_lib.Context([(m.E, m.p, m.lo, m.hi) for m in (big, small)])
    # call 1: the 36 pair densities of the exchange workload (the records of all 36 do not fit
    # the fixed array at once, so the entry takes several passes)
    xyz, _ = ctx.mesh_coords(0)
    phi = wl.orbitals.values_torch(*xyz, device="cuda").reshape(-1).contiguous()
    f1 = gpu_lib.pair_densities(phi, wl.orbitals.norb)
    ref1 = ctx.boundary_data(f1, mesh_id=0)
    g1 = torch.full_like(ref1, np.nan)
    ctx.boundary_data_noalloc(f1, g1, mesh_id=0)
    torch.cuda.synchronize()
    assert _rel(g1.cpu().numpy(), ref1.cpu().numpy(), 36) <= 1e-12
    # call 2: three signed sources on a small ragged mesh of degree 3
    xyz2, _ = ctx.mesh_coords(1)
    rng = np.random.default_rng(91)
    dens = [configs.GaussianDensity(rng.uniform(0.5, 1.5, 2), rng.uniform(0.4, 1.2, 2),
                                    rng.uniform(-1.0, 1.0, (2, 3))) for _ in range(3)]
    f2 = _t(np.concatenate([d.density(*xyz2) * np.cos(0.7 * xyz2[0] + 0.3 * k) for k, d in enumerate(dens)]))
    ref2 = ctx.boundary_data(f2, mesh_id=1)
    g2 = torch.full_like(ref2, np.nan)
    ctx.boundary_data_noalloc(f2, g2, mesh_id=1)
    torch.cuda.synchronize()
    assert _rel(g2.cpu().numpy(), ref2.cpu().numpy(), 3) <= 1e-12
    # an empty call does nothing
    ctx.boundary_data_noalloc(f2[:0], g2[:0], mesh_id=1)


def test_no_alloc_entry_rejects_a_mesh_beyond_its_work_space(gpu_lib):
    """A mesh of 11,520,000 nodes: one source's records exceed the 8,388,608-value array."""
    import torch
    m = configs.Mesh((48, 48, 40), 4, (-24.0, -24.0, -20.0), (24.0, 24.0, 20.0))
    ctx = gpu_lib.Context([(m.E, m.p, m.lo, m.hi)], lanes=1)
    nd, nf = ctx.info[0]["n_dofs"], ctx.info[0]["n_face"]
    assert nd > 8 * 1024 * 1024
    f = torch.zeros(nd, dtype=torch.float64, device="cuda")
    g = torch.zeros(nf, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.DgError, match="too large"):
        ctx.boundary_data_noalloc(f, g)
