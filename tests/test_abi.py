"""The C-ABI library loads and exports every function include/dg_poisson.h declares.

Runs on the CPU: only host-only entry points are called.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg_poisson.h")
LIB = os.path.join(ROOT, "paper_2510_21213_amd", "libdgpoisson.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdgpoisson.so is not built (run paper_2510_21213_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["dg_poisson_setup", "dg_poisson_solve_batch", "dg_exchange_apply", "dg_poisson_destroy",
                     "dg_status_string", "dg_operator_apply", "dg_vcycle_apply", "dg_coarse_solve"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_only_entry_points(lib):
    lib.dg_status_string.restype = ctypes.c_char_p
    assert lib.dg_status_string(0) == b"ok"
    assert lib.dg_status_string(-1) == b"invalid argument"
    from paper_2510_21213_amd import binding
    o = binding.default_opts()
    assert o.cheb_degree == 6 and o.cheb_degree_h == 10 and o.cheb_ratio == 60.0 and abs(o.penalty_eps - 0.125) < 1e-15 and o.rtol == 1e-8
    assert o.node_family == 0 and binding.default_opts(node_family="gl").node_family == 1
    with pytest.raises(KeyError):
        binding.default_opts(nonexistent=1)


def test_setup_rejects_bad_arguments_without_touching_the_gpu(lib):
    from paper_2510_21213_amd import binding
    h = ctypes.c_void_p()
    opts = binding.default_opts()
    # null mesh array -> DG_ERR_ARG before any device call
    rc = binding.lib.dg_poisson_setup(None, 0, ctypes.byref(opts), ctypes.byref(h))
    assert rc == -1
    assert b"mesh" in binding.lib.dg_last_error()


def test_tile_table_host_calls(lib):
    """dg_tile_set / dg_tile_get need no GPU: a compiled tile round-trips, shapes without a
    kernel and bad arguments are rejected, and degrees without slab kernels report tx = 0."""
    from paper_2510_21213_amd import binding
    orig = binding.tile_get(4, 5, "CHEB")
    assert orig[0] in (2, 4) and 1 <= orig[2] <= 4
    try:
        binding.tile_set(4, 5, "CHEB", 2, 2, 3)
        assert binding.tile_get(4, 5, "CHEB") == (2, 2, 3)
    finally:
        binding.tile_set(4, 5, "CHEB", *orig)
    for bad in [(4, 5, "CHEB", 8, 8, 2), (4, 3, "PQ", 4, 4, 5), (2, 5, "PQ", 4, 4, 2), (8, 2, "APPLY", 8, 8, 3),
                (8, 4, "APPLY", 4, 4, 2)]:
        with pytest.raises(binding.DgError):
            binding.tile_set(*bad)
    assert binding.tile_get(8, 4, "APPLY")[0] == 0
