"""GPU tests of the fused Helmholtz operator alpha A + beta B (the bake-off systems (alpha A + beta B) u = B f).

Every kernel family (collocated strip and element kernels with the diagonal mass term, the line-per-
thread Gauss kernels, their strip form, the point-per-thread kernel) against the oracle's
assembled alpha A + beta B at 1e-12, for degrees 1..8, GLL-collocated and Gauss rules, one and three
components; E-vectors, the diagonal, FP32, and solves.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fem, solvers  # noqa: E402
from paper_2109_04996_amd import hexpa as hx  # noqa: E402
from paper_2109_04996_amd.inputs import kappa_field_params, lattice_mesh, rotate_elements, uniform_vector  # noqa: E402
from paper_2109_04996_amd.problem import Hierarchy, Problem  # noqa: E402

ALPHA, BETA = 0.8, 3.5


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _rules(p):
    out = [("gll", p + 1), ("gauss", p + 1), ("gauss", p + 2)]
    return [(r, q) for r, q in out if q <= 10]


CASES = [(p, r, q) for p in range(1, 9) for r, q in _rules(p)]


@pytest.mark.parametrize("p,rule,q", CASES)
@pytest.mark.parametrize("ncomp", [1, 3])
def test_helmholtz_apply_matches_oracle(p, rule, q, ncomp):
    N = 3 if p <= 6 else 2
    print(f"\n[case] helmholtz N={N} p={p} q={q} {rule} ncomp={ncomp}", flush=True)
    mesh = rotate_elements(lattice_mesh(N, p, warp="B", shuffle_seed=2), p, 0.2, seed=p)
    H = fem.assemble_helmholtz(mesh, p, q, rule, ALPHA, BETA)
    with Problem(N, p, q, rule, "helmholtz", ncomp=ncomp, mesh=mesh, helmholtz=(ALPHA, BETA)) as pr:
        x = uniform_vector(mesh["nnodes"], 1, ncomp)
        yr = fem.apply(H, x, ncomp)
        y = pr.apply(pr.to_dev(x)).cpu().numpy()
        assert rel(y, yr) <= 1e-12, rel(y, yr)
        assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()
        st = hx.hx_op_get_stats(pr.h_op)
        assert st["kind"] == hx.HX_HELMHOLTZ
        if ncomp == 1:
            np.testing.assert_allclose(pr.diagonal().cpu().numpy(), fem.diagonal(H), rtol=1e-12)


@pytest.mark.parametrize("p,q", [(7, 9), (5, 7)])
def test_helmholtz_vector_fp32(p, q):
    # three components in FP32 (the joint-component Gauss kernel): FP64 and FP32 geometric factors,
    # against the oracle at the FP32 bound of the diffusion parity tests
    N = 2 if p == 7 else 3
    mesh = rotate_elements(lattice_mesh(N, p, warp="B", shuffle_seed=3), p, 0.2, seed=p)
    H = fem.assemble_helmholtz(mesh, p, q, "gauss", ALPHA, BETA)
    with Problem(N, p, q, "gauss", "helmholtz", ncomp=3, mesh=mesh, helmholtz=(ALPHA, BETA)) as pr:
        x = uniform_vector(mesh["nnodes"], 4, 3)
        yr = fem.apply(H, x.astype(np.float32).astype(np.float64), 3)
        for qprec in (hx.HX_FP64, hx.HX_FP32):
            y32 = pr.apply_f32(pr.to_dev(x, torch.float32), qdata_prec=qprec).double().cpu().numpy()
            assert rel(y32, yr) <= 6e-6, (qprec, rel(y32, yr))


@pytest.mark.parametrize("p,rule,q,N", [(7, "gll", 8, 3), (7, "gauss", 8, 3), (6, "gauss", 8, 3),
                                        (4, "gll", 5, 3), (7, "gauss", 9, 2)])
def test_helmholtz_lattice_paths(p, rule, q, N):
    # unrotated lattice meshes: the strip kernels (degree 7 and the Gauss q = 8 strips) on the affine
    # node numbering, and the E-vector output of every family, element by element
    mesh = lattice_mesh(N, p, warp="B", shuffle_seed=4)
    H = fem.assemble_helmholtz(mesh, p, q, rule, ALPHA, BETA)
    with Problem(N, p, q, rule, "helmholtz", mesh=mesh, helmholtz=(ALPHA, BETA)) as pr:
        assert pr.stats["index_mode"] == 2
        x = uniform_vector(mesh["nnodes"], 2)
        y = pr.apply(pr.to_dev(x)).cpu().numpy()
        assert rel(y, H @ x) <= 1e-12
        ye = pr.apply_elem(pr.to_dev(x)).cpu().numpy()
        Ae = fem.element_matrices(mesh, p, q, rule, "diffusion")
        Be = fem.element_matrices(mesh, p, q, rule, "mass")
        xe = x[mesh["elem_nodes"]]
        ref = np.einsum("eij,ej->ei", ALPHA * Ae + BETA * Be, xe)
        assert rel(ye[:, 0, :], ref) <= 1e-12
        # FP32 vectors with FP32 geometric factors (the FP32 bound of the diffusion parity tests)
        y32 = pr.apply_f32(pr.to_dev(x, torch.float32), qdata_prec=hx.HX_FP32).double().cpu().numpy()
        assert rel(y32, H @ x.astype(np.float32).astype(np.float64)) <= 6e-6


def test_helmholtz_kappa_and_limits():
    # a coefficient multiplies the diffusion part only; beta = 0 is the diffusion operator and alpha = 0
    # the mass operator, both through the Helmholtz kernels
    p, q, N = 5, 7, 3
    kp = kappa_field_params(102, M=64)
    mesh = lattice_mesh(N, p, warp="B", shuffle_seed=7)
    x = uniform_vector(mesh["nnodes"], 3)
    for a, b in ((ALPHA, BETA), (1.0, 0.0), (0.0, 2.0)):
        H = fem.assemble_helmholtz(mesh, p, q, "gauss", a, b, kappa=kp)
        with Problem(N, p, q, "gauss", "helmholtz", mesh=mesh, kappa=kp, helmholtz=(a, b)) as pr:
            assert rel(pr.apply(pr.to_dev(x)).cpu().numpy(), H @ x) <= 1e-12, (a, b)


def test_helmholtz_rejects_bad_coefficients():
    mesh = lattice_mesh(2, 2)
    for a, b in ((0.0, 0.0), (-1.0, 1.0), (1.0, float("nan"))):
        with pytest.raises(hx.HexpaError):
            Problem(2, 2, 3, "gll", "helmholtz", mesh=mesh, helmholtz=(a, b))
    with Problem(2, 2, 3, "gll", "helmholtz", mesh=mesh) as pr:
        with pytest.raises(hx.HexpaError):
            pr.apply_bf16(pr.zeros(torch.float32))


@pytest.mark.parametrize("p,rule,q,ncomp", [(4, "gll", 5, 1), (3, "gauss", 5, 3), (7, "gll", 8, 1)])
def test_helmholtz_solve_matches_direct(p, rule, q, ncomp):
    # (alpha A + beta B) u = B f with homogeneous Dirichlet conditions: Jacobi-PCG and the FP32-operator
    # Chebyshev form to 1e-12 against the oracle's direct solve
    N = 3
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=5)
    H = solvers.expand(fem.assemble_helmholtz(mesh, p, q, rule, ALPHA, BETA), ncomp)
    free = solvers.free_mask(mesh["boundary"], ncomp)
    b = uniform_vector(mesh["nnodes"], 6, ncomp) * free
    xd = solvers.direct_solve(H, b, free)
    with Problem(N, p, q, rule, "helmholtz", ncomp=ncomp, mesh=mesh, helmholtz=(ALPHA, BETA)) as pr:
        x, info = pr.solve(pr.to_dev(b), rtol=1e-12)
        assert rel(x.cpu().numpy(), xd) <= 1e-9, info
        x, info = pr.solve(pr.to_dev(b), rtol=1e-12, precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP32)
        assert rel(x.cpu().numpy(), xd) <= 1e-9, info


def test_helmholtz_pmultigrid():
    # a V-cycle hierarchy of Helmholtz operators (every level alpha A_l + beta B_l): FCG to 1e-10 matches
    # the direct solve in far fewer iterations than Jacobi-PCG
    N = 4
    mesh7 = lattice_mesh(N, 7, warp="A", shuffle_seed=0)
    H = fem.assemble_helmholtz(mesh7, 7, 8, "gll", ALPHA, BETA)
    free = solvers.free_mask(mesh7["boundary"])
    b = uniform_vector(mesh7["nnodes"], 7) * free
    xd = solvers.direct_solve(H, b, free)
    with Hierarchy(N, [7, 3, 1], "gll", "helmholtz", helmholtz=(ALPHA, BETA)) as mg:
        x, info = mg.solve(mg.fine.to_dev(b), rtol=1e-10)
        xj, ij = mg.fine.solve(mg.fine.to_dev(b), rtol=1e-10)
        assert rel(x.cpu().numpy(), xd) <= 1e-7, info
        assert info["iterations"] * 4 < ij["iterations"], (info, ij)
