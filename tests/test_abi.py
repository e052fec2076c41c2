"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, validates
arguments before touching the device, and its host-side 1D tables and node coordinates agree with
the oracle's independently computed ones."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2109_04996_amd import hexpa as hx
from paper_2109_04996_amd.inputs import lattice_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hexpa.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hx_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    return hx.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    bound = {n for n, _, _ in hx.SIGNATURES}
    for n in names:
        assert hasattr(lib, n), f"{n} declared in hexpa.h but not exported"
        assert n in bound, f"{n} has no binding"


def test_version(lib):
    assert "hexpa" in hx.hx_version()


@pytest.mark.parametrize("p,q,rule", [(0, 2, hx.HX_GAUSS), (9, 11, hx.HX_GAUSS), (3, 7, hx.HX_GAUSS),
                                      (3, 5, hx.HX_GLL), (3, 4, 7)])
def test_basis_rejects(lib, p, q, rule):
    with pytest.raises(hx.HexpaError) as e:
        hx.hx_basis_create(p, q, rule)
    assert e.value.code == hx.HX_EINVAL
    assert hx.hx_last_error()


def test_mesh_rejects_before_device(lib):
    m = lattice_mesh(2, 2, warp=None)
    xyz = np.zeros((m["nnodes"], 3))
    with pytest.raises(hx.HexpaError) as e:
        hx.hx_mesh_create(0, m["elem_nodes"], xyz, None)
    assert e.value.code == hx.HX_EINVAL
    bad = m["elem_nodes"].copy()
    bad[3, 5] = m["nnodes"]  # out of range
    with pytest.raises(hx.HexpaError) as e:
        hx.hx_mesh_create(2, bad, xyz, None)
    assert e.value.code == hx.HX_ERANGE
    bad[3, 5] = -1
    with pytest.raises(hx.HexpaError) as e:
        hx.hx_mesh_create(2, bad, xyz, None)
    assert e.value.code == hx.HX_ERANGE
    h = C.c_void_p()
    assert lib.hx_mesh_create(2, 1, 10, None, None, None, C.byref(h)) == hx.HX_EINVAL
    assert lib.hx_mesh_create(2, 1, 10, None, None, None, None) == hx.HX_EINVAL


def test_null_handles(lib):
    assert lib.hx_op_apply(None, None, None, None) == hx.HX_EINVAL
    assert lib.hx_op_diagonal(None, None, None) == hx.HX_EINVAL
    assert lib.hx_pcg_solve(None, None, None, None, None, None) == hx.HX_EINVAL
    assert lib.hx_pcg_solve_noalloc(None, None, None, None, None, None) == hx.HX_EINVAL
    h = C.c_void_p()
    assert lib.hx_op_create_lor(None, None, None, C.byref(h)) == hx.HX_EINVAL
    assert lib.hx_op_create_lor(None, None, None, None) == hx.HX_EINVAL
    assert lib.hx_op_lor_matrix(None, None, None, None) == hx.HX_EINVAL
    o = hx.hx_pmg_opts_default()
    h = C.c_void_p()
    assert lib.hx_pmg_create(None, 2, C.byref(o), None, C.byref(h)) == hx.HX_EINVAL
    ops = (C.c_void_p * 2)(None, None)
    assert lib.hx_pmg_create(ops, 1, C.byref(o), None, C.byref(h)) == hx.HX_EINVAL  # nlevels < 2
    assert lib.hx_pmg_create(ops, 2, C.byref(o), None, C.byref(h)) == hx.HX_EINVAL  # null operators
    assert lib.hx_pmg_vcycle(None, None, None, None) == hx.HX_EINVAL
    assert lib.hx_pmg_prolong(None, 0, None, None, None) == hx.HX_EINVAL
    assert lib.hx_pmg_restrict(None, 0, None, None, None) == hx.HX_EINVAL
    assert lib.hx_pmg_levels(None) == 0
    lib.hx_pmg_destroy(None)
    lib.hx_op_destroy(None)
    lib.hx_mesh_destroy(None)
    lib.hx_basis_destroy(None)


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("rule,dq", [(hx.HX_GAUSS, 2), (hx.HX_GAUSS, 1), (hx.HX_GLL, 1)])
def test_basis_tables_match_oracle(lib, p, rule, dq):
    from oracle.fem import reference_tables
    q = p + dq
    b = hx.hx_basis_create(p, q, rule)
    try:
        t = hx.hx_basis_get_tables(b, p, q)
    finally:
        hx.hx_basis_destroy(b)
    xn, xq, wq, phi, dphi = reference_tables(p, q, "gauss" if rule == hx.HX_GAUSS else "gll")
    np.testing.assert_allclose(t["nodes"], xn, atol=1e-15)
    np.testing.assert_allclose(t["qpts"], xq, atol=1e-15)
    np.testing.assert_allclose(t["qweights"], wq, rtol=1e-14)
    np.testing.assert_allclose(t["interp"], phi, atol=1e-14)
    np.testing.assert_allclose(t["grad"], dphi, atol=1e-12 * max(1, p * p))


@pytest.mark.parametrize("p", [1, 3, 7])
def test_node_coordinates_match_oracle(lib, p):
    from oracle.fem import node_coordinates
    m = lattice_mesh(3, p, warp="B", shuffle_seed=4)
    xyz = hx.hx_mesh_nodes_trilinear(p, m["elem_verts"], m["verts"], m["elem_nodes"], m["nnodes"])
    np.testing.assert_allclose(xyz, node_coordinates(m, p), atol=2e-16 * 4)


def test_solve_opts_defaults(lib):
    o = hx.hx_solve_opts_default()
    assert o.rtol == 1e-8 and o.precond == hx.HX_PC_JACOBI and o.cheb_degree == 4
    with pytest.raises(AttributeError):
        hx.hx_solve_opts_default(not_a_field=1)


def test_pmg_opts_defaults(lib):
    o = hx.hx_pmg_opts_default()
    assert (o.smooth_degree, o.smooth_ratio, o.lanczos_steps, o.coarse_maxit, o.coarse_rtol, o.prec) == \
        (3, 15.0, 20, 30, 0.1, hx.HX_FP64)
    assert hx.hx_solve_opts_default().pmg is None
    with pytest.raises(AttributeError):
        hx.hx_pmg_opts_default(not_a_field=1)


def test_product_path_does_not_import_oracle():
    # the binding and the problem builder never reach the oracle
    import ast
    pkg = os.path.join(ROOT, "paper_2109_04996_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, f)).read())
            for node in ast.walk(tree):
                if isinstance(node, (ast.Import, ast.ImportFrom)):
                    mod = node.module if isinstance(node, ast.ImportFrom) else node.names[0].name
                    assert not (mod or "").startswith("oracle"), f"{f} imports {mod}"
