"""Python binding of libdgpoisson.so (argument marshalling only).

Every computation runs in the HIP library; this module only converts
arguments: torch tensors on the GPU provide device memory, the current torch
stream provides the HIP stream.  If the library is missing the import fails
loudly -- there is no fallback path.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# DG_POISSON_LIB selects another build of the same library (for example one
# compiled with different tile parameters); the default is the in-tree build.
LIB_PATH = os.environ.get("DG_POISSON_LIB", os.path.join(_HERE, "libdgpoisson.so"))

DG_OK, DG_WARN_NOT_CONVERGED = 0, 1
DG_PREC_FP64, DG_PREC_FP32_IR, DG_PREC_FP32_PC, DG_PREC_BF16_PC, DG_PREC_BF16F_PC = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": DG_PREC_FP64, "fp32_ir": DG_PREC_FP32_IR, "fp32_pc": DG_PREC_FP32_PC,
              "bf16_pc": DG_PREC_BF16_PC, "bf16f_pc": DG_PREC_BF16F_PC}
NODE_FAMILIES = {"gll": 0, "gl": 1}   # dg_opts.node_family


class DgMesh(ctypes.Structure):
    _fields_ = [("ne", ctypes.c_int * 3), ("p", ctypes.c_int),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class DgOpts(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("cheb_degree", ctypes.c_int), ("cheb_ratio", ctypes.c_double),
                ("cheb_safety", ctypes.c_double), ("lanczos_steps", ctypes.c_int),
                ("penalty_eps", ctypes.c_double), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("check_every", ctypes.c_int), ("use_graph", ctypes.c_int), ("lanes", ctypes.c_int),
                ("cheb_degree_h", ctypes.c_int), ("fused", ctypes.c_int), ("fused_wgs", ctypes.c_int),
                ("fused_spin", ctypes.c_longlong), ("node_family", ctypes.c_int), ("learned_cgc", ctypes.c_int)]


class DgRhsStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("status", ctypes.c_int),
                ("guess_used", ctypes.c_int), ("rel_residual", ctypes.c_double)]


class DgError(RuntimeError):
    pass


class DgOctreeDesc(ctypes.Structure):
    _fields_ = [("ne", ctypes.c_int * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("q", ctypes.c_int), ("delta_q", ctypes.c_double), ("max_depth", ctypes.c_int),
                ("max_elements", ctypes.c_longlong)]


DENSITY_FN = ctypes.CFUNCTYPE(None, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2510_21213_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sigs = {
        "dg_opts_default": (None, [ctypes.POINTER(DgOpts)]),
        "dg_poisson_setup": (I, [ctypes.POINTER(DgMesh), I, ctypes.POINTER(DgOpts), ctypes.POINTER(P)]),
        "dg_poisson_destroy": (None, [P]),
        "dg_status_string": (ctypes.c_char_p, [I]),
        "dg_last_error": (ctypes.c_char_p, []),
        "dg_mesh_info": (I, [P, I, ctypes.POINTER(LL), ctypes.POINTER(LL), ctypes.POINTER(I)]),
        "dg_mesh_coords": (I, [P, I, P, P]),
        "dg_poisson_solve_batch": (I, [P, I, P, P, P, P, P, P, P]),
        "dg_exchange_apply": (I, [P, I, I, P, P, P, P, P, P, P, P]),
        "dg_operator_apply": (I, [P, I, I, I, P, P, P]),
        "dg_operator_apply_f32": (I, [P, I, I, I, P, P, P]),
        "dg_operator_apply_mfma": (I, [P, I, I, I, P, P, P]),
        "dg_vcycle_apply_f32": (I, [P, I, I, I, P, P, P]),
        "dg_rhs_assemble": (I, [P, I, I, P, P, P, P]),
        "dg_boundary_data": (I, [P, I, I, P, P, P]),
        "dg_pair_densities": (I, [LL, I, I, I, P, P, P]),
        "dg_boundary_data_noalloc": (I, [P, I, I, P, P, P]),
        "dg_tile_set": (I, [I, I, I, I, I, I]),
        "dg_tile_get": (I, [I, I, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "dg_vcycle_apply": (I, [P, I, I, I, P, P, P]),
        "dg_coarse_solve": (I, [P, I, I, P, P, P]),
        "dg_restrict": (I, [P, I, I, I, P, P, P]),
        "dg_prolong_add": (I, [P, I, I, I, P, P, P]),
        "dg_level_info": (I, [P, I, I, P, P, P, P]),
        "dg_profile_enable": (I, [P, I]),
        "dg_fused_fallbacks": (I, [P, ctypes.POINTER(LL)]),
        "dg_hartree_action": (I, [P, I, I, P, I, P, P, P, P]),
        "dg_exchange_action": (I, [P, I, I, P, I, P, I, P, P, P, P, P, P]),
        "dg_ace_build": (I, [P, I, I, P, P, P, P]),
        "dg_ace_action": (I, [P, I, I, P, I, P, I, P, P, P]),
        "dg_net_create": (I, [P, ctypes.POINTER(P)]),
        "dg_net_destroy": (None, [P]),
        "dg_net_last_error": (ctypes.c_char_p, []),
        "dg_net_num_params": (LL, [P]),
        "dg_net_set_params": (I, [P, P, LL]),
        "dg_net_get_params": (I, [P, P, LL]),
        "dg_net_forward": (I, [P, I, P, P, P, P]),
        "dg_net_backward": (I, [P, P, P, P]),
        "dg_net_infer": (I, [P, I, P, P, P, P]),
        "dg_net_adam": (I, [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P]),
        "dg_net_prepare_input": (I, [P, I, LL, P, P, P, P]),
        "dg_net_train_step": (I, [P, P, I, I, P, P, ctypes.c_float, I, ctypes.POINTER(D), P]),
        "dg_net_guess": (I, [P, P, I, I, P, P, P]),
        "dg_net_save": (I, [P, ctypes.c_char_p]),
        "dg_net_set_bf16": (I, [P, I]),
        "dg_net_load": (I, [P, ctypes.c_char_p]),
        "dg_poisson_attach_guess": (I, [P, P]),
        "dg_profile_read": (I, [P, ctypes.POINTER(LL), ctypes.POINTER(D), ctypes.POINTER(D)]),
        "dg_octree_create": (I, [ctypes.POINTER(DgOctreeDesc), DENSITY_FN, P, ctypes.POINTER(DgOpts),
                                 ctypes.POINTER(P)]),
        "dg_octree_destroy": (None, [P]),
        "dg_octree_info": (I, [P, ctypes.POINTER(LL), ctypes.POINTER(LL), ctypes.POINTER(LL), ctypes.POINTER(I),
                               ctypes.POINTER(I)]),
        "dg_octree_level_info": (I, [P, I, ctypes.POINTER(LL), ctypes.POINTER(I), ctypes.POINTER(D),
                                     ctypes.POINTER(D)]),
        "dg_octree_elements": (I, [P, P, P]),
        "dg_octree_nodes": (I, [P, P, P, P]),
        "dg_octree_boundary_points": (I, [P, P, P, P]),
        "dg_octree_rhs": (I, [P, I, P, P, P, P]),
        "dg_octree_apply": (I, [P, I, I, P, P, P]),
        "dg_octree_vcycle": (I, [P, I, P, P, P]),
        "dg_octree_solve": (I, [P, I, P, P, P, P]),
        "dg_octree_set_rhs_per_block": (I, [P, I]),
        "dg_octree_boundary_data": (I, [P, I, P, P, P]),
        "dg_octree_apply_f32": (I, [P, I, I, P, P, P]),
        "dg_octree_exchange": (I, [P, I, P, P, P, P, P, ctypes.POINTER(D), P, P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()

STEPS = {"APPLY": 0, "RESID": 1, "CHEB": 2, "CHEBDOT": 3, "PQ": 4, "RESIDDOT": 5, "RESTRICT": 6}
TILE_TABLE = os.path.join(_HERE, "tiles_gfx950.json")


def tile_set(fp_bytes, n, step, tx, ty, zlen):
    """Work-group tile of one operator step for contexts set up afterwards (dg_tile_set)."""
    code = lib.dg_tile_set(int(fp_bytes), int(n), STEPS[step] if isinstance(step, str) else int(step),
                           int(tx), int(ty), int(zlen))
    if code != 0:
        raise DgError(f"tile_set: {lib.dg_last_error().decode()}")


def tile_get(fp_bytes, n, step):
    tx, ty, z = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    code = lib.dg_tile_get(int(fp_bytes), int(n), STEPS[step] if isinstance(step, str) else int(step),
                           ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(z))
    if code != 0:
        raise DgError(f"tile_get: {lib.dg_last_error().decode()}")
    return tx.value, ty.value, z.value


def apply_tile_table(path=TILE_TABLE):
    """Apply a tile table written by tune_tiles.py (a list of {fp_bytes, n, step, tx, ty, zlen})."""
    import json
    with open(path) as f:
        for t in json.load(f)["tiles"]:
            tile_set(t["fp_bytes"], t["n"], t["step"], t["tx"], t["ty"], t["zlen"])


if os.path.exists(TILE_TABLE) and not os.environ.get("DG_POISSON_NO_TILE_TABLE"):
    apply_tile_table()


def pair_densities(phi, norb, first=0, count=None):
    """rho_ij = phi_i phi_j for the pairs first .. first+count-1 (row-major i <= j order) of the
    packed orbitals phi (float64 CUDA tensor [norb * n_dofs]); returns [count * n_dofs]."""
    nd = phi.numel() // norb
    total = norb * (norb + 1) // 2
    count = total - first if count is None else count
    rho = torch.empty(count * nd, dtype=torch.float64, device=phi.device)
    _check(lib.dg_pair_densities(nd, norb, first, count, _ptr(phi), _ptr(rho), _stream()), "pair_densities")
    return rho


def status_string(code):
    return lib.dg_status_string(code).decode()


def default_opts(**kw):
    o = DgOpts()
    lib.dg_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "node_family" and isinstance(v, str):
            v = NODE_FAMILIES[v]
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _check(code, what, allow_warn=False):
    if code == DG_OK or (allow_warn and code == DG_WARN_NOT_CONVERGED):
        return code
    raise DgError(f"{what}: {status_string(code)} ({lib.dg_last_error().decode()})")


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _ptr_t(t, dtype):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A set-up DG Poisson solver for one or more uniform meshes.

    meshes: list of (ne, p, lo, hi) with ne, lo, hi 3-sequences.
    options: fields of dg_opts (precision may be "fp64", "fp32_ir", "fp32_pc" or "bf16_pc").
    """

    def __init__(self, meshes, **options):
        arr = (DgMesh * len(meshes))()
        for k, (ne, p, lo, hi) in enumerate(meshes):
            arr[k].ne[:] = [int(v) for v in ne]
            arr[k].p = int(p)
            arr[k].lo[:] = [float(v) for v in lo]
            arr[k].hi[:] = [float(v) for v in hi]
        self.opts = default_opts(**options)
        h = ctypes.c_void_p()
        _check(lib.dg_poisson_setup(arr, len(meshes), ctypes.byref(self.opts), ctypes.byref(h)), "setup")
        self._h = h
        self.n_meshes = len(meshes)
        self.info = [self.mesh_info(m) for m in range(self.n_meshes)]

    def close(self):
        if getattr(self, "_h", None):
            lib.dg_poisson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- description
    def mesh_info(self, mesh_id):
        nd, nf, nl = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
        _check(lib.dg_mesh_info(self._h, mesh_id, ctypes.byref(nd), ctypes.byref(nf), ctypes.byref(nl)), "mesh_info")
        return {"n_dofs": nd.value, "n_face": nf.value, "n_levels": nl.value}

    def level_info(self, mesh_id, level):
        ne = (ctypes.c_int * 3)()
        p, lo, hi = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(lib.dg_level_info(self._h, mesh_id, level, ne, ctypes.byref(p), ctypes.byref(lo), ctypes.byref(hi)),
               "level_info")
        return {"ne": tuple(ne), "p": p.value, "lam_lo": lo.value, "lam_hi": hi.value}

    def mesh_coords(self, mesh_id):
        """(xyz [3, n_dofs], fxyz [3, n_face]) as numpy arrays."""
        inf = self.info[mesh_id]
        xyz = np.empty((3, inf["n_dofs"]))
        fxyz = np.empty((3, inf["n_face"]))
        _check(lib.dg_mesh_coords(self._h, mesh_id, xyz.ctypes.data_as(ctypes.c_void_p),
                                  fxyz.ctypes.data_as(ctypes.c_void_p)), "mesh_coords")
        return xyz, fxyz

    # ---- solves
    def solve_batch(self, rho, g, mesh_ids=None, x0=None, out=None):
        """Solve the packed batch; returns (v, stats list of dicts).  g None: Dirichlet data by quadrature."""
        nrhs = len(mesh_ids) if mesh_ids is not None else (rho.numel() // self.info[0]["n_dofs"] if rho.numel() else 0)
        if mesh_ids is None:
            mesh_ids = [0] * nrhs
        ids = (ctypes.c_int * max(1, nrhs))(*mesh_ids)
        nd = sum(self.info[m]["n_dofs"] for m in mesh_ids)
        nf = sum(self.info[m]["n_face"] for m in mesh_ids)
        if rho.numel() != nd or (g is not None and g.numel() != nf):
            raise ValueError("rho/g sizes do not match the meshes")
        if out is None:
            out = torch.empty(nd, dtype=torch.float64, device=rho.device)
        stats = (DgRhsStats * max(1, nrhs))()
        code = lib.dg_poisson_solve_batch(self._h, nrhs, ids, _ptr(rho), _ptr(g), _ptr(x0), _ptr(out),
                                          stats, _stream())
        _check(code, "solve_batch", allow_warn=True)
        return out, [_stats(stats[i]) for i in range(nrhs)]

    def exchange(self, phi, g_pairs, mesh_id=0, keep_potentials=False):
        """Returns (W, K, E_x, stats, v or None).  g_pairs None: Dirichlet data by quadrature."""
        nd = self.info[mesh_id]["n_dofs"]
        norb = phi.numel() // nd
        npairs = norb * (norb + 1) // 2
        if g_pairs is not None and g_pairs.numel() != npairs * self.info[mesh_id]["n_face"]:
            raise ValueError("g_pairs has the wrong size")
        W = torch.empty(norb * nd, dtype=torch.float64, device=phi.device)
        K = torch.empty(npairs, dtype=torch.float64, device=phi.device)
        v = torch.empty(npairs * nd, dtype=torch.float64, device=phi.device) if keep_potentials else None
        ex = ctypes.c_double()
        stats = (DgRhsStats * npairs)()
        code = lib.dg_exchange_apply(self._h, mesh_id, norb, _ptr(phi), _ptr(g_pairs), _ptr(W), _ptr(K),
                                     ctypes.byref(ex), _ptr(v), stats, _stream())
        _check(code, "exchange_apply", allow_warn=True)
        return W, K, ex.value, [_stats(stats[i]) for i in range(npairs)], v

    # ---- consumers: actions projected on a basis, compressed exchange
    def _count(self, t, mesh_id):
        nd = self.info[mesh_id]["n_dofs"]
        if t.numel() % nd:
            raise ValueError("field stack is not a whole number of fields")
        return t.numel() // nd

    def hartree_action(self, phi, u, vH, mesh_id=0):
        """[nbasis, nu] matrix of (phi_i, u_a vH) by the grid's quadrature (dg_hartree_action)."""
        nb, nu = self._count(phi, mesh_id), self._count(u, mesh_id)
        out = torch.empty(nb * nu, dtype=torch.float64, device=phi.device)
        _check(lib.dg_hartree_action(self._h, mesh_id, nb, _ptr(phi), nu, _ptr(u), _ptr(vH), _ptr(out), _stream()),
               "hartree_action")
        return out.view(nb, nu)

    def exchange_action(self, phi, u, psi, g_pairs=None, mesh_id=0, keep_w=False):
        """([nbasis, nu] matrix of (phi_i, K u_a), W or None, stats) (dg_exchange_action)."""
        nb, nu, no = self._count(phi, mesh_id), self._count(u, mesh_id), self._count(psi, mesh_id)
        out = torch.empty(nb * nu, dtype=torch.float64, device=phi.device)
        W = torch.empty(nu * self.info[mesh_id]["n_dofs"], dtype=torch.float64, device=phi.device) if keep_w else None
        stats = (DgRhsStats * (nu * no))()
        code = lib.dg_exchange_action(self._h, mesh_id, nb, _ptr(phi), nu, _ptr(u), no, _ptr(psi), _ptr(g_pairs),
                                      _ptr(out), _ptr(W), stats, _stream())
        _check(code, "exchange_action", allow_warn=True)
        return out.view(nb, nu), W, [_stats(stats[i]) for i in range(nu * no)]

    def ace_build(self, psi, W, mesh_id=0):
        """The compressed exchange vectors xi [nocc * n_dofs] (dg_ace_build)."""
        no = self._count(psi, mesh_id)
        xi = torch.empty_like(psi)
        _check(lib.dg_ace_build(self._h, mesh_id, no, _ptr(psi), _ptr(W), _ptr(xi), _stream()), "ace_build")
        return xi

    def ace_action(self, phi, u, xi, mesh_id=0):
        """[nbasis, nu] matrix of sum_k (phi_i, xi_k)(xi_k, u_a) (dg_ace_action)."""
        nb, nu, no = self._count(phi, mesh_id), self._count(u, mesh_id), self._count(xi, mesh_id)
        out = torch.empty(nb * nu, dtype=torch.float64, device=phi.device)
        _check(lib.dg_ace_action(self._h, mesh_id, nb, _ptr(phi), nu, _ptr(u), no, _ptr(xi), _ptr(out), _stream()),
               "ace_action")
        return out.view(nb, nu)

    def attach_guess(self, net):
        """Use a trained Net for the initial guess of later solves (None to stop)."""
        _check(lib.dg_poisson_attach_guess(self._h, net._h if net is not None else None), "attach_guess")
        self._guess = net

    def fused_fallbacks(self):
        """Group-persistent solves (fused=2) that fell back to the level kernels."""
        n = ctypes.c_longlong()
        _check(lib.dg_fused_fallbacks(self._h, ctypes.byref(n)), "fused_fallbacks")
        return n.value

    # ---- timing of the finest-level Chebyshev step
    def profile(self, enable=True):
        _check(lib.dg_profile_enable(self._h, 1 if enable else 0), "profile_enable")

    def profile_read(self):
        n, sec, by = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
        _check(lib.dg_profile_read(self._h, ctypes.byref(n), ctypes.byref(sec), ctypes.byref(by)), "profile_read")
        return {"launches": n.value, "seconds": sec.value, "bytes": by.value}

    # ---- single steps
    def operator_apply(self, u, mesh_id=0, level=0):
        nrhs = u.numel() // self._level_dofs(mesh_id, level)
        y = torch.empty_like(u)
        f32 = u.dtype == torch.float32
        fn = lib.dg_operator_apply_f32 if f32 else lib.dg_operator_apply
        pt = (lambda t: _ptr_t(t, torch.float32)) if f32 else _ptr
        _check(fn(self._h, mesh_id, level, nrhs, pt(u), pt(y), _stream()), "operator_apply")
        return y

    def operator_apply_mfma(self, u, mesh_id=0, level=0):
        """y = A u (FP32 fields) with the x and y contractions on the matrix cores (BF16 operands)."""
        nrhs = u.numel() // self._level_dofs(mesh_id, level)
        y = torch.empty_like(u)
        _check(lib.dg_operator_apply_mfma(self._h, mesh_id, level, nrhs, _ptr_t(u, torch.float32),
                                          _ptr_t(y, torch.float32), _stream()), "operator_apply_mfma")
        return y

    def rhs_assemble(self, rho, g, mesh_id=0):
        nrhs = rho.numel() // self.info[mesh_id]["n_dofs"]
        b = torch.empty_like(rho)
        _check(lib.dg_rhs_assemble(self._h, mesh_id, nrhs, _ptr(rho), _ptr(g), _ptr(b), _stream()), "rhs_assemble")
        return b

    def boundary_data(self, f, mesh_id=0):
        """Dirichlet data g (packed face vectors) of the packed sources f by quadrature."""
        nd, nf = self.info[mesh_id]["n_dofs"], self.info[mesh_id]["n_face"]
        if f.numel() % nd:
            raise ValueError("f is not a whole number of fields")
        nsrc = f.numel() // nd
        g = torch.empty(nsrc * nf, dtype=torch.float64, device=f.device)
        _check(lib.dg_boundary_data(self._h, mesh_id, nsrc, _ptr(f), _ptr(g), _stream()), "boundary_data")
        return g

    def boundary_data_noalloc(self, f, g, mesh_id=0):
        """dg_boundary_data_noalloc into the caller's g (packed face vectors): nothing is
        allocated on either side of the call."""
        nd, nf = self.info[mesh_id]["n_dofs"], self.info[mesh_id]["n_face"]
        if f.numel() % nd or g.numel() != (f.numel() // nd) * nf:
            raise ValueError("f / g sizes do not match the mesh")
        _check(lib.dg_boundary_data_noalloc(self._h, mesh_id, f.numel() // nd, _ptr(f), _ptr(g), _stream()),
               "boundary_data_noalloc")
        return g

    def vcycle(self, r, mesh_id=0, level=0):
        nrhs = r.numel() // self._level_dofs(mesh_id, level)
        z = torch.empty_like(r)
        f32 = r.dtype == torch.float32
        fn = lib.dg_vcycle_apply_f32 if f32 else lib.dg_vcycle_apply
        pt = (lambda t: _ptr_t(t, torch.float32)) if f32 else _ptr
        _check(fn(self._h, mesh_id, level, nrhs, pt(r), pt(z), _stream()), "vcycle_apply")
        return z

    def coarse_solve(self, r, mesh_id=0):
        L = self.info[mesh_id]["n_levels"] - 1
        nrhs = r.numel() // self._level_dofs(mesh_id, L)
        z = torch.empty_like(r)
        _check(lib.dg_coarse_solve(self._h, mesh_id, nrhs, _ptr(r), _ptr(z), _stream()), "coarse_solve")
        return z

    def restrict(self, r, mesh_id=0, level=0):
        nrhs = r.numel() // self._level_dofs(mesh_id, level)
        rc = torch.empty(nrhs * self._level_dofs(mesh_id, level + 1), dtype=torch.float64, device=r.device)
        _check(lib.dg_restrict(self._h, mesh_id, level, nrhs, _ptr(r), _ptr(rc), _stream()), "restrict")
        return rc

    def prolong_add(self, zc, zf, mesh_id=0, level=0):
        nrhs = zf.numel() // self._level_dofs(mesh_id, level)
        _check(lib.dg_prolong_add(self._h, mesh_id, level, nrhs, _ptr(zc), _ptr(zf), _stream()), "prolong_add")
        return zf

    def _level_dofs(self, mesh_id, level):
        li = self.level_info(mesh_id, level)
        n = li["p"] + 1
        return li["ne"][0] * li["ne"][1] * li["ne"][2] * n ** 3


class Octree:
    """Adaptive octree auxiliary mesh with its MG-PCG Poisson solver (dg_octree_*).

    rho: callable rho(x, y, z) on numpy arrays (or None: the base mesh, unrefined); options:
    fields of dg_opts (FP64 precision only).
    """

    def __init__(self, ne, lo, hi, q=4, rho=None, delta_q=1e-8, max_depth=3, max_elements=1 << 20, **options):
        d = DgOctreeDesc()
        d.ne[:] = [int(v) for v in ne]
        d.lo[:] = [float(v) for v in lo]
        d.hi[:] = [float(v) for v in hi]
        d.q, d.delta_q, d.max_depth, d.max_elements = int(q), float(delta_q), int(max_depth), int(max_elements)
        self.opts = default_opts(**options)
        self._err = None

        def cb(n, x, y, z, out, user):
            try:
                xa, ya, za = (np.ctypeslib.as_array(a, shape=(n,)) for a in (x, y, z))
                np.ctypeslib.as_array(out, shape=(n,))[:] = np.asarray(rho(xa, ya, za), dtype=np.float64)
            except Exception as e:   # a failing density: NaN makes the library reject the mesh
                self._err = e
                np.ctypeslib.as_array(out, shape=(n,))[:] = np.nan
        self._cb = DENSITY_FN(cb) if rho is not None else DENSITY_FN()
        h = ctypes.c_void_p()
        code = lib.dg_octree_create(ctypes.byref(d), self._cb, None, ctypes.byref(self.opts), ctypes.byref(h))
        if self._err is not None:
            raise self._err
        _check(code, "octree_create")
        self._h = h
        ne_, nd, nb, nl, mg = (ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int(),
                               ctypes.c_int())
        _check(lib.dg_octree_info(h, ctypes.byref(ne_), ctypes.byref(nd), ctypes.byref(nb), ctypes.byref(nl),
                                  ctypes.byref(mg)), "octree_info")
        self.n_elements, self.n_dofs, self.n_boundary = ne_.value, nd.value, nb.value
        self.n_levels, self.max_generation = nl.value, mg.value
        self.q = int(q)

    def close(self):
        if getattr(self, "_h", None):
            lib.dg_octree_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level):
        ne, q, lo, hi = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(lib.dg_octree_level_info(self._h, level, ctypes.byref(ne), ctypes.byref(q), ctypes.byref(lo),
                                        ctypes.byref(hi)), "octree_level_info")
        return {"n_elements": ne.value, "q": q.value, "lam_lo": lo.value, "lam_hi": hi.value,
                "n_dofs": ne.value * (q.value + 1) ** 3}

    def set_rhs_per_block(self, rb):
        _check(lib.dg_octree_set_rhs_per_block(self._h, int(rb)), "octree_set_rhs_per_block")

    def elements(self):
        """(lohi [n_elements, 6], generation [n_elements])."""
        lohi = np.empty((self.n_elements, 6))
        gen = np.empty(self.n_elements, dtype=np.int32)
        _check(lib.dg_octree_elements(self._h, lohi.ctypes.data_as(ctypes.c_void_p),
                                      gen.ctypes.data_as(ctypes.c_void_p)), "octree_elements")
        return lohi, gen

    def nodes(self):
        xyz = np.empty((3, self.n_dofs))
        _check(lib.dg_octree_nodes(self._h, *(xyz[i].ctypes.data_as(ctypes.c_void_p) for i in range(3))),
               "octree_nodes")
        return xyz

    def boundary_points(self):
        xyz = np.empty((3, max(self.n_boundary, 1)))
        _check(lib.dg_octree_boundary_points(self._h, *(xyz[i].ctypes.data_as(ctypes.c_void_p) for i in range(3))),
               "octree_boundary_points")
        return xyz[:, :self.n_boundary]

    def boundary_data(self, f):
        """Dirichlet data by quadrature of the sources f [nsrc, n_dofs]: [nsrc, n_boundary]."""
        nsrc = f.numel() // self.n_dofs
        g = torch.empty((nsrc, self.n_boundary), dtype=torch.float64, device=f.device)
        _check(lib.dg_octree_boundary_data(self._h, nsrc, _ptr(f), _ptr(g), _stream()), "octree_boundary_data")
        return g

    def rhs(self, f, g=None):
        """b = 4 pi M f + lift(g); g None: the Dirichlet data by quadrature of f."""
        nrhs = f.numel() // self.n_dofs
        b = torch.empty_like(f)
        _check(lib.dg_octree_rhs(self._h, nrhs, _ptr(f), _ptr(g), _ptr(b), _stream()), "octree_rhs")
        return b

    def apply(self, u, level=0):
        n = self.level_info(level)["n_dofs"]
        y = torch.empty_like(u)
        _check(lib.dg_octree_apply(self._h, level, u.numel() // n, _ptr(u), _ptr(y), _stream()), "octree_apply")
        return y

    def apply_f32(self, u, level=0):
        """FP32 operator (float32 CUDA tensor)."""
        n = self.level_info(level)["n_dofs"]
        y = torch.empty_like(u)
        _check(lib.dg_octree_apply_f32(self._h, level, u.numel() // n, _ptr_t(u, torch.float32),
                                       _ptr_t(y, torch.float32), _stream()), "octree_apply_f32")
        return y

    def vcycle(self, r):
        z = torch.empty_like(r)
        _check(lib.dg_octree_vcycle(self._h, r.numel() // self.n_dofs, _ptr(r), _ptr(z), _stream()),
               "octree_vcycle")
        return z

    def exchange(self, phi, g_pairs=None, keep_potentials=False):
        """(W [norb, n_dofs], K [npairs], E_x, stats, v or None) for orbitals phi [norb, n_dofs];
        g_pairs None: Dirichlet data by quadrature."""
        norb = phi.numel() // self.n_dofs
        npairs = norb * (norb + 1) // 2
        W = torch.empty((norb, self.n_dofs), dtype=torch.float64, device=phi.device)
        v = torch.empty((npairs, self.n_dofs), dtype=torch.float64, device=phi.device) if keep_potentials else None
        K = np.empty(npairs)
        ex = ctypes.c_double()
        st = (DgRhsStats * npairs)()
        code = lib.dg_octree_exchange(self._h, norb, _ptr(phi), _ptr(g_pairs), _ptr(v), _ptr(W),
                                      K.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ex), st, _stream())
        _check(code, "octree_exchange", allow_warn=True)
        return W, K, ex.value, [_stats(st[i]) for i in range(npairs)], v

    def solve(self, b):
        """x = A^-1 b (MG-PCG); returns (x, stats list)."""
        nrhs = b.numel() // self.n_dofs
        x = torch.empty_like(b)
        st = (DgRhsStats * max(nrhs, 1))()
        code = lib.dg_octree_solve(self._h, nrhs, _ptr(b), _ptr(x), st, _stream())
        _check(code, "octree_solve", allow_warn=True)
        return x, [_stats(st[i]) for i in range(nrhs)]


def _stats(s):
    return {"iters": s.iters, "outer_iters": s.outer_iters, "status": s.status, "guess_used": s.guess_used,
            "rel_residual": s.rel_residual}


class DgNetConfig(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("channels", ctypes.c_int), ("in_channels", ctypes.c_int),
                ("out_channels", ctypes.c_int)]


def _ncheck(code, what):
    if code != DG_OK:
        raise DgError(f"{what}: {status_string(code)} ({lib.dg_net_last_error().decode()})")


class Net:
    """The learned-initial-guess U-Net (include/dg_poisson.h, dg_net_*)."""

    def __init__(self, levels=4, channels=32, in_channels=125, out_channels=27):
        cfg = DgNetConfig(levels, channels, in_channels, out_channels)
        h = ctypes.c_void_p()
        _ncheck(lib.dg_net_create(ctypes.byref(cfg), ctypes.byref(h)), "net_create")
        self._h = h
        self.levels, self.channels = levels, channels
        self.in_channels, self.out_channels = in_channels, out_channels
        self.num_params = lib.dg_net_num_params(h)

    def close(self):
        if getattr(self, "_h", None):
            lib.dg_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_bf16(self, enable=True):
        """Forward convolutions on the matrix cores (BF16 operands, FP32 accumulation) or in FP32."""
        _ncheck(lib.dg_net_set_bf16(self._h, 1 if enable else 0), "net_set_bf16")

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _ncheck(lib.dg_net_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size), "net_set_params")

    def get_params(self):
        p = np.empty(self.num_params, dtype=np.float32)
        _ncheck(lib.dg_net_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size), "net_get_params")
        return p

    def forward(self, x, ne, batch):
        ne_c = (ctypes.c_int * 3)(*ne)
        y = torch.empty(batch * ne[0] * ne[1] * ne[2] * self.out_channels, dtype=torch.float32, device=x.device)
        _ncheck(lib.dg_net_forward(self._h, batch, ne_c, _ptr_t(x, torch.float32), _ptr_t(y, torch.float32),
                                   _stream()), "net_forward")
        return y

    def infer(self, x, ne, batch):
        """The guess's forward: matrix cores with BF16 activations (dg_net_infer)."""
        ne_c = (ctypes.c_int * 3)(*ne)
        y = torch.empty(batch * ne[0] * ne[1] * ne[2] * self.out_channels, dtype=torch.float32, device=x.device)
        _ncheck(lib.dg_net_infer(self._h, batch, ne_c, _ptr_t(x, torch.float32), _ptr_t(y, torch.float32),
                                 _stream()), "net_infer")
        return y

    def backward(self, dy):
        g = torch.empty(self.num_params, dtype=torch.float32, device=dy.device)
        _ncheck(lib.dg_net_backward(self._h, _ptr_t(dy, torch.float32), _ptr_t(g, torch.float32), _stream()),
                "net_backward")
        return g

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        _ncheck(lib.dg_net_adam(self._h, lr, b1, b2, eps, _stream()), "net_adam")

    def prepare_input(self, rho, batch, n_dofs):
        x = torch.empty(batch * n_dofs, dtype=torch.float32, device=rho.device)
        s = torch.empty(batch, dtype=torch.float64, device=rho.device)
        _ncheck(lib.dg_net_prepare_input(self._h, batch, n_dofs, _ptr(rho), _ptr_t(x, torch.float32), _ptr(s),
                                         _stream()), "net_prepare_input")
        return x, s

    def train_step(self, ctx, x, t, batch, lr, mesh_id=0, mode=0):
        """mode 0: A-norm gradient; 1: nodal L2 gradient; 2: V-cycle preconditioned A-norm gradient."""
        loss = ctypes.c_double()
        _ncheck(lib.dg_net_train_step(self._h, ctx._h, mesh_id, batch, _ptr_t(x, torch.float32), _ptr(t), lr,
                                      mode, ctypes.byref(loss), _stream()), "net_train_step")
        return loss.value

    def guess(self, ctx, rho, batch, mesh_id=0):
        v0 = torch.empty_like(rho)
        _ncheck(lib.dg_net_guess(self._h, ctx._h, mesh_id, batch, _ptr(rho), _ptr(v0), _stream()), "net_guess")
        return v0

    def save(self, path):
        _ncheck(lib.dg_net_save(self._h, str(path).encode()), "net_save")

    def load(self, path):
        _ncheck(lib.dg_net_load(self._h, str(path).encode()), "net_load")
