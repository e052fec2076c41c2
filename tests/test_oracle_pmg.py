"""Pins of the p-multigrid oracle (CPU only).

The transfer is fixed by what interpolation must reproduce: every function of
the coarse space exactly (polynomials in the physical coordinates on the
affine mesh A, the coordinate functions on the trilinear mesh B), and, with
quadrature exact for both bilinear forms, the Galerkin identity P^T A_f P =
A_c. The V-cycle is fixed by its algebra: with an identity transfer and an
exact coarse solve it is the exact inverse; with an exact coarse solve it is
symmetric positive definite and its error propagation contracts.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, pmg, solvers
from paper_2109_04996_amd.inputs import lattice_mesh


def _poly(X, deg):
    """A fixed polynomial of degree <= deg in each coordinate."""
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    return 0.7 + x ** deg * y ** max(deg - 1, 0) * z ** deg - 1.3 * y ** deg + 0.4 * x * z - 0.2 * z ** deg


@pytest.mark.parametrize("pf,pc", [(2, 1), (4, 2), (7, 3), (5, 5)])
def test_interpolation_1d(pf, pc):
    I = pmg.interpolation_1d(pf, pc)
    xf = np.polynomial.legendre.Legendre.basis(pf).deriv().roots() if pf > 1 else np.array([])
    xf = np.concatenate([[-1.0], np.sort(xf), [1.0]])
    from oracle.quadrature import gll_rule
    xc, _ = gll_rule(pc)
    for d in range(pc + 1):  # polynomials of degree <= pc are reproduced
        assert np.allclose(I @ xc ** d, xf ** d, atol=1e-13, rtol=0)
    assert np.allclose(I.sum(axis=1), 1.0, atol=1e-14)
    if pf == pc:
        assert np.allclose(I, np.eye(pf + 1), atol=1e-14)


@pytest.mark.parametrize("N,pf,pc", [(3, 4, 2), (2, 7, 3), (2, 3, 1)])
def test_prolongation_reproduces_coarse_space(N, pf, pc):
    mf = lattice_mesh(N, pf, warp="A", shuffle_seed=1)
    mc = lattice_mesh(N, pc, warp="A", shuffle_seed=1)
    P = pmg.prolongation(mf, mc, pf, pc)
    Xf, Xc = fem.node_coordinates(mf, pf), fem.node_coordinates(mc, pc)
    assert P.shape == (mf["nnodes"], mc["nnodes"])
    # mesh A: axis-aligned boxes, so polynomials of degree <= pc per coordinate are coarse functions
    u = _poly(Xc, pc)
    assert np.max(np.abs(P @ u - _poly(Xf, pc))) <= 1e-12 * np.max(np.abs(u))
    # mesh B (trilinear, not affine): the coordinate functions lie in every Q_p space
    mf, mc = lattice_mesh(N, pf, warp="B", shuffle_seed=2), lattice_mesh(N, pc, warp="B", shuffle_seed=2)
    P = pmg.prolongation(mf, mc, pf, pc)
    Xf, Xc = fem.node_coordinates(mf, pf), fem.node_coordinates(mc, pc)
    assert np.max(np.abs(P @ Xc - Xf)) <= 1e-13
    # a coarse function that vanishes on the boundary interpolates to one that does
    uc = np.random.default_rng(0).uniform(-1, 1, mc["nnodes"]) * (mc["boundary"] == 0)
    assert np.all((P @ uc)[mf["boundary"] != 0] == 0)


@pytest.mark.parametrize("kind", ["diffusion", "mass"])
@pytest.mark.parametrize("pf,pc", [(4, 2), (3, 1)])
def test_galerkin_identity(kind, pf, pc):
    # mesh A with Gauss q = p + 2 integrates both forms exactly on both levels; the coarse space lies
    # in the fine one, so the coarse matrix is the fine one restricted to it
    N = 2
    mf, mc = lattice_mesh(N, pf, warp="A", shuffle_seed=3), lattice_mesh(N, pc, warp="A", shuffle_seed=3)
    Af = fem.assemble(mf, pf, pf + 2, "gauss", kind)
    Ac = fem.assemble(mc, pc, pc + 2, "gauss", kind)
    P = pmg.prolongation(mf, mc, pf, pc)
    G = (P.T @ Af @ P).toarray()
    assert np.max(np.abs(G - Ac.toarray())) <= 1e-12 * np.max(np.abs(Ac.toarray()))


def _levels(N, degrees, warp="B", rule="gll"):
    meshes = [lattice_mesh(N, p, warp=warp, shuffle_seed=4) for p in degrees]
    out = []
    for l, (m, p) in enumerate(zip(meshes, degrees)):
        q = p + 1 if rule == "gll" else p + 2
        A = fem.assemble(m, p, q, rule, "diffusion")
        free = solvers.free_mask(m["boundary"])
        P = pmg.prolongation(m, meshes[l + 1], p, degrees[l + 1]) if l + 1 < len(degrees) else None
        out.append(pmg.Level(A, free, solvers.jacobi_lambda_max(A, free), P))
    return meshes, out


def test_identity_transfer_and_exact_coarse_solve_give_the_inverse():
    mesh = lattice_mesh(2, 3, warp="B", shuffle_seed=4)
    A = fem.assemble(mesh, 3, 4, "gll", "diffusion")
    free = solvers.free_mask(mesh["boundary"])
    lam = solvers.jacobi_lambda_max(A, free)
    levels = [pmg.Level(A, free, lam, sp.identity(A.shape[0], format="csr")), pmg.Level(A, free)]
    r = np.random.default_rng(0).uniform(-1, 1, A.shape[0]) * free
    z = pmg.vcycle(levels, r, degree=3, ratio=8.0, coarse="direct")
    assert np.linalg.norm(z - solvers.direct_solve(A, r, free)) <= 1e-11 * np.linalg.norm(z)


def _dense_vcycle(levels, n, free, **kw):
    idx = np.flatnonzero(free)
    V = np.zeros((idx.size, idx.size))
    for j, c in enumerate(idx):
        e = np.zeros(n)
        e[c] = 1.0
        V[:, j] = pmg.vcycle(levels, e, **kw)[idx]
    return V


@pytest.mark.parametrize("degrees", [(4, 2), (4, 2, 1)])
def test_vcycle_symmetric_and_contracting(degrees):
    meshes, levels = _levels(2, degrees)
    A0, free = levels[0].A, levels[0].free
    V = _dense_vcycle(levels, A0.shape[0], free, degree=2, ratio=10.0, coarse="direct")
    assert np.max(np.abs(V - V.T)) <= 1e-10 * np.max(np.abs(V))
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
    Aii = A0[free][:, free].toarray()
    lam = np.sort(np.linalg.eigvals(V @ Aii).real)
    # error propagation I - V A contracts, and V A is far better conditioned than D^-1 A
    assert 0 < lam[0] and lam[-1] < 2
    assert np.max(np.abs(1 - lam)) < 0.6
    d = Aii.diagonal()
    lj = np.linalg.eigvalsh(Aii / np.sqrt(np.outer(d, d)))
    assert lam[-1] / lam[0] < 0.2 * lj[-1] / lj[0]


def test_flexible_pcg_with_vcycle():
    meshes, levels = _levels(3, (4, 2, 1))
    m = meshes[0]
    X = fem.node_coordinates(m, 4)
    B = fem.assemble(m, 4, 5, "gll", "mass")
    f = 3 * np.pi ** 2 * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    b = B @ f
    A, free = fem.assemble(m, 4, 5, "gll", "diffusion"), levels[0].free
    x, it, res = pmg.flexible_pcg(A, b, free, lambda r: pmg.vcycle(levels, r, degree=2, ratio=10.0,
                                                                    coarse_rtol=0.0, coarse_maxit=10))
    assert res <= 1e-8
    xr = solvers.direct_solve(A, b, free)
    assert np.linalg.norm(x - xr) <= 1e-7 * np.linalg.norm(xr)
    _, it_j, _ = solvers.jacobi_pcg(A, b, free, tol=1e-8)
    assert it < it_j / 3


def test_vector_vcycle_is_three_scalar_vcycles():
    # the vector operator is the scalar one on each interleaved component (index 3 node + c); with an
    # exact coarse solve nothing couples the components, so the expanded V-cycle is three scalar ones
    meshes, levels = _levels(2, (4, 2, 1))
    vec = []
    for lv in levels:
        P3 = None if lv.P is None else sp.kron(lv.P, sp.identity(3), format="csr")
        vec.append(pmg.Level(solvers.expand(lv.A_full, 3), np.repeat(lv.free, 3), lv.lam_max, P3))
    n = levels[0].A.shape[0]
    r = np.random.default_rng(1).uniform(-1, 1, 3 * n)
    z = pmg.vcycle(vec, r, degree=3, ratio=15.0, coarse="direct")
    for c in range(3):
        zc = pmg.vcycle(levels, r[c::3], degree=3, ratio=15.0, coarse="direct")
        assert np.max(np.abs(z[c::3] - zc)) <= 1e-13 * np.max(np.abs(zc))
