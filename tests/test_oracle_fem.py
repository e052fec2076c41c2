"""Pins of the oracle's element matrices and assembled operators.

Each check is fixed by mathematics independent of the oracle's code path:
volumes, integrals of polynomials in closed form, invariants of the
stiffness matrix, exact reproduction of polynomial solutions, convergence
order, hand assembly on two elements, re-integration with more points, and
the closed form of the diagonal of the collocated operator.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, solvers
from oracle.quadrature import gll_rule, lagrange_deriv_table
from paper_2109_04996_amd.inputs import lattice_mesh

RULES = [("gauss", 2), ("gll", 1)]  # (rule, q - p)


def test_meshes_are_warped():
    # with N = 2 the warps vanish at every vertex (sin at 0, 1/2, 1); the pins use N >= 3
    u = lattice_mesh(3, 1, warp=None)["verts"]
    for w in ("A", "B"):
        v = lattice_mesh(3, 1, warp=w)["verts"]
        assert np.abs(v - u).max() > 0.03
    vb = lattice_mesh(3, 1, warp="B")["verts"]
    assert np.abs(vb[:, 0] - u[:, 0]).max() > 0.03  # x moves with y: non-affine bricks


def _ops(N, p, warp, rule, dq, kind, seed=0):
    mesh = lattice_mesh(N, p, warp=warp, shuffle_seed=seed)
    return mesh, fem.assemble(mesh, p, p + dq, rule, kind)


@pytest.mark.parametrize("warp", [None, "A", "B"])
@pytest.mark.parametrize("rule,dq", RULES)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_mass_integrates_volume(warp, rule, dq, p):
    mesh, B = _ops(3, p, warp, rule, dq, "mass")
    one = np.ones(mesh["nnodes"])
    assert abs(one @ (B @ one) - 1.0) < 1e-13


@pytest.mark.parametrize("warp", ["A", "B"])
@pytest.mark.parametrize("rule,dq", RULES)
@pytest.mark.parametrize("p", [1, 2, 4])
def test_diffusion_invariants(warp, rule, dq, p):
    mesh, A = _ops(3 if p < 4 else 2, p, warp, rule, dq, "diffusion")
    one = np.ones(mesh["nnodes"])
    assert np.abs(A @ one).max() < 1e-12 * abs(A).max()
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    if mesh["nnodes"] <= 800:
        ev = np.linalg.eigvalsh(A.toarray())
        assert abs(ev[0]) < 1e-11 * ev[-1]
        assert ev[1] > 1e-6 * ev[-1]  # exactly one zero eigenvalue: the constants
        free = solvers.free_mask(mesh["boundary"])
        evi = np.linalg.eigvalsh(A[free][:, free].toarray())
        assert evi[0] > 0


@pytest.mark.parametrize("warp", ["A", "B"])
@pytest.mark.parametrize("rule,dq,p", [("gauss", 2, 1), ("gauss", 2, 3), ("gll", 1, 3), ("gll", 1, 5)])
def test_coordinate_function_forms(warp, rule, dq, p):
    # x is in V_h on any trilinear mesh: int |grad x|^2 = vol = 1 and int x^2 = 1/3 over the unit cube.
    mesh = lattice_mesh(3, p, warp=warp, shuffle_seed=3)
    X = fem.node_coordinates(mesh, p)
    A = fem.assemble(mesh, p, p + dq, rule, "diffusion")
    B = fem.assemble(mesh, p, p + dq, rule, "mass")
    for a in range(3):
        xa = X[:, a]
        assert abs(xa @ (A @ xa) - 1.0) < 1e-12
        assert abs(xa @ (B @ xa) - 1.0 / 3.0) < 1e-13


@pytest.mark.parametrize("rule,dq,p", [("gauss", 2, 2), ("gauss", 2, 4), ("gll", 1, 3), ("gll", 1, 5)])
def test_quadratic_forms_mesh_a(rule, dq, p):
    # on the axis-aligned mesh A, u = v = x^2 is in V_h: u'Au = int (2x)^2 = 4/3, u'Bu = int x^4 = 1/5
    mesh = lattice_mesh(3, p, warp="A", shuffle_seed=1)
    X = fem.node_coordinates(mesh, p)
    A = fem.assemble(mesh, p, p + dq, rule, "diffusion")
    B = fem.assemble(mesh, p, p + dq, rule, "mass")
    u = X[:, 1] ** 2
    assert abs(u @ (A @ u) - 4.0 / 3.0) < 1e-12
    assert abs(u @ (B @ u) - 0.2) < 1e-13
    # mixed form: u = x^2, v = y z: int grad u . grad v = 0, int u v = 1/3 * 1/4
    v = X[:, 0] * X[:, 2]
    w = X[:, 1] ** 2
    assert abs(v @ (A @ w)) < 1e-13
    assert abs(v @ (B @ w) - 1.0 / 12.0) < 1e-13


def _manufactured(X):
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    u = x * (1 - x) * y * (1 - y) * z * (1 - z)
    f = 2 * (y * (1 - y) * z * (1 - z) + x * (1 - x) * z * (1 - z) + x * (1 - x) * y * (1 - y))
    return u, f


@pytest.mark.parametrize("p", [2, 3])
def test_manufactured_polynomial_reproduced(p):
    # u in Q_2 on mesh A with f = -lap u in Q_2: the Galerkin solution is u itself (Gauss q = p+2 exact).
    mesh = lattice_mesh(3, p, warp="A", shuffle_seed=2)
    X = fem.node_coordinates(mesh, p)
    A = fem.assemble(mesh, p, p + 2, "gauss", "diffusion")
    B = fem.assemble(mesh, p, p + 2, "gauss", "mass")
    u, f = _manufactured(X)
    free = solvers.free_mask(mesh["boundary"])
    uh = solvers.direct_solve(A, B @ f, free)
    assert np.abs(uh - u).max() < 1e-13


@pytest.mark.parametrize("p", [3, 4])
def test_manufactured_polynomial_gll(p):
    # collocated GLL stiffness (exact to degree 2p-1 >= p+2 for p >= 3) with an exact Gauss load vector
    mesh = lattice_mesh(3, p, warp="A", shuffle_seed=2)
    X = fem.node_coordinates(mesh, p)
    A = fem.assemble(mesh, p, p + 1, "gll", "diffusion")
    B = fem.assemble(mesh, p, p + 2, "gauss", "mass")
    u, f = _manufactured(X)
    free = solvers.free_mask(mesh["boundary"])
    uh = solvers.direct_solve(A, B @ f, free)
    assert np.abs(uh - u).max() < 1e-13


@pytest.mark.slow
def test_convergence_order_sine():
    # u = sin(pi x) sin(pi y) sin(pi z), f = 3 pi^2 u; L2 error ~ h^(p+1) (textbook a priori estimate)
    p = 2
    errs = []
    for N in (2, 4, 8):
        mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
        X = fem.node_coordinates(mesh, p)
        A = fem.assemble(mesh, p, p + 2, "gauss", "diffusion")
        B = fem.assemble(mesh, p, p + 2, "gauss", "mass")
        u = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
        free = solvers.free_mask(mesh["boundary"])
        uh = solvers.direct_solve(A, B @ (3 * np.pi ** 2 * u), free)
        e = uh - u
        errs.append(np.sqrt(e @ (B @ e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 0.6, rates


@pytest.mark.parametrize("kind", ["mass", "diffusion"])
def test_two_element_hand_assembly(kind):
    # N=3 lattice restricted to its first two elements along x: assemble by hand and compare
    p = 2
    mesh = lattice_mesh(3, p, warp="B", shuffle_seed=None)
    sub = dict(mesh)
    sub["elem_verts"] = mesh["elem_verts"][:2]
    sub["elem_nodes"] = mesh["elem_nodes"][:2]
    sub["nelem"] = 2
    Ae = fem.element_matrices(sub, p, p + 2, "gauss", kind)
    dense = np.zeros((mesh["nnodes"], mesh["nnodes"]))
    for e in range(2):
        idx = sub["elem_nodes"][e]
        for a in range(len(idx)):
            for b in range(len(idx)):
                dense[idx[a], idx[b]] += Ae[e, a, b]
    A = fem.assemble(sub, p, p + 2, "gauss", kind).toarray()
    assert np.abs(A - dense).max() < 1e-15 * np.abs(dense).max() + 1e-300
    # the shared face: 9 nodes belong to both elements
    shared = np.intersect1d(sub["elem_nodes"][0], sub["elem_nodes"][1])
    assert shared.size == (p + 1) ** 2


@pytest.mark.parametrize("kind", ["mass", "diffusion"])
@pytest.mark.parametrize("p", [2, 5])
def test_reintegration_more_points(kind, p):
    # mesh A: integrands are polynomials of degree <= 2p per direction, exact with q = p+2 Gauss points
    mesh = lattice_mesh(3, p, warp="A", shuffle_seed=4)
    a = fem.element_matrices(mesh, p, p + 2, "gauss", kind, elems=[0, 5])
    b = fem.element_matrices(mesh, p, p + 6, "gauss", kind, elems=[0, 5])
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("warp", ["A", "B"])
@pytest.mark.parametrize("p", [2, 4])
def test_collocated_diagonal_closed_form(warp, p):
    # With q = p+1 GLL points collocated with the nodes, phi_i(x_j) = delta_ij, so the element diagonal is
    # sum_l D_li^2 G11(l,j,k) + sum_m D_mj^2 G22(i,m,k) + sum_n D_nk^2 G33(i,j,n)
    #   + 2 (D_ii D_jj G12 + D_ii D_kk G13 + D_jj D_kk G23)(i,j,k),
    # G = w detJ J^-1 J^-T at the points, D the 1D derivative matrix at the GLL nodes.
    mesh = lattice_mesh(3, p, warp=warp, shuffle_seed=5)
    A = fem.assemble(mesh, p, p + 1, "gll", "diffusion")
    P = p + 1
    xn, wn = gll_rule(p)
    D = lagrange_deriv_table(xn, xn)  # D[a, i] = l_i'(x_a)
    r3 = fem.reference_points3(xn)
    w3 = np.einsum("c,b,a->cba", wn, wn, wn).ravel()
    diag = np.zeros(mesh["nnodes"])
    V = mesh["verts"][mesh["elem_verts"]]
    for e in range(mesh["nelem"]):
        _, J = fem.trilinear_map(V[e], r3)
        det, inv = fem.det_and_inverse(J)
        G = (w3 * det)[:, None, None] * np.einsum("nai,nbi->nab", inv, inv)
        G = G.reshape(P, P, P, 3, 3)  # [k, j, i]
        de = np.zeros((P, P, P))
        for k in range(P):
            for j in range(P):
                for i in range(P):
                    s = sum(D[l, i] ** 2 * G[k, j, l, 0, 0] for l in range(P))
                    s += sum(D[m, j] ** 2 * G[k, m, i, 1, 1] for m in range(P))
                    s += sum(D[n, k] ** 2 * G[n, j, i, 2, 2] for n in range(P))
                    s += 2 * (D[i, i] * D[j, j] * G[k, j, i, 0, 1] + D[i, i] * D[k, k] * G[k, j, i, 0, 2]
                              + D[j, j] * D[k, k] * G[k, j, i, 1, 2])
                    de[k, j, i] = s
        np.add.at(diag, mesh["elem_nodes"][e], de.ravel())
    np.testing.assert_allclose(fem.diagonal(A), diag, rtol=1e-12)


def test_shuffle_invariance():
    # the element order is a relabelling of a sum: the assembled operator does not depend on it
    a = fem.assemble(lattice_mesh(3, 3, warp="B", shuffle_seed=0), 3, 5, "gauss", "diffusion")
    b = fem.assemble(lattice_mesh(3, 3, warp="B", shuffle_seed=9), 3, 5, "gauss", "diffusion")
    assert abs(a - b).max() < 1e-14 * abs(a).max()


def test_vector_operator_is_blockwise():
    mesh = lattice_mesh(3, 2, warp="B", shuffle_seed=0)
    A = fem.assemble(mesh, 2, 4, "gauss", "diffusion")
    x = np.random.default_rng(0).standard_normal(3 * mesh["nnodes"])
    y = fem.apply(A, x, ncomp=3)
    for c in range(3):
        np.testing.assert_allclose(y[c::3], A @ x[c::3], rtol=1e-14, atol=1e-14)
    K = solvers.expand(A, 3)
    np.testing.assert_allclose(K @ x, y, rtol=1e-13, atol=1e-13)


def test_element_apply_matches_assembly():
    mesh = lattice_mesh(3, 3, warp="B", shuffle_seed=1)
    x = np.random.default_rng(1).uniform(-1, 1, mesh["nnodes"])
    ye = fem.element_apply(mesh, 3, 5, "gauss", "diffusion", x, np.arange(mesh["nelem"]))
    y = np.zeros(mesh["nnodes"])
    np.add.at(y, mesh["elem_nodes"], ye[:, 0, :])
    A = fem.assemble(mesh, 3, 5, "gauss", "diffusion")
    np.testing.assert_allclose(y, A @ x, rtol=1e-12, atol=1e-13)


def test_kappa_field_contrast():
    from paper_2109_04996_amd.inputs import kappa_field_params
    kp = kappa_field_params(100)
    g = np.random.default_rng(0).uniform(0, 1, (20000, 3))
    k = fem.kappa_eval(kp, g)
    assert 0.07 < k.min() and k.max() < 14.0
    assert k.max() / k.min() > 30
    # kappa = 1 where the field is constant: scale 0 gives exp(shift)
    kp0 = dict(kp, scale=0.0, shift=0.0)
    assert np.all(fem.kappa_eval(kp0, g) == 1.0)
    # a coefficient scales the stiffness: kappa == 2 everywhere doubles A
    mesh = lattice_mesh(3, 2, warp="B")
    A1 = fem.assemble(mesh, 2, 4, "gauss", "diffusion")
    A2 = fem.assemble(mesh, 2, 4, "gauss", "diffusion", kappa=dict(kp, scale=0.0, shift=np.log(2.0)))
    assert abs(A2 - 2 * A1).max() < 1e-14 * abs(A1).max()


@pytest.mark.parametrize("N,p,q,tol", [(4, 5, 7, 1e-12), (4, 3, 5, 1e-9)])
def test_kappa_location_closed_form(N, p, q, tol):
    # where kappa is evaluated: a coefficient that varies along x alone (one feature, omega = (w, 0, 0),
    # phase -pi/2, so g = sqrt(2) sin(w x)). On mesh A (axis-aligned bricks) the coordinate functions
    # and their squares lie in V_h, so for u in {y, x^2, y^2}
    #   u^T A u = int kappa |grad u|^2 = int_0^1 kappa(x) dx, 4 int_0^1 kappa(x) x^2 dx, (4/3) int_0^1 kappa(x) dx,
    # up to the element rule's quadrature error. The 1D integrals come from a 200-point Gauss rule on
    # [0, 1] that does not use the mesh. Evaluating kappa at reference coordinates, at another axis or
    # at the element's nodes instead of its physical quadrature points breaks one of the three.
    w, sc, sh = 3.0, 0.5, 0.1
    kp = dict(omega=np.array([[w, 0.0, 0.0]]), phase=np.array([-np.pi / 2]), scale=sc, shift=sh, M=1)
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=2)
    A = fem.assemble(mesh, p, q, "gauss", "diffusion", kappa=kp)
    X = fem.node_coordinates(mesh, p)
    t, wt = np.polynomial.legendre.leggauss(200)
    t, wt = 0.5 * (t + 1.0), 0.5 * wt
    kap = np.exp(sc * np.sqrt(2.0) * np.sin(w * t) + sh)
    I0, I2 = float(wt @ kap), float(wt @ (kap * t * t))
    y, x2, y2 = X[:, 1], X[:, 0] ** 2, X[:, 1] ** 2
    assert abs(y @ (A @ y) / I0 - 1.0) <= tol
    assert abs(x2 @ (A @ x2) / (4.0 * I2) - 1.0) <= tol
    assert abs(y2 @ (A @ y2) / (4.0 / 3.0 * I0) - 1.0) <= tol


@pytest.mark.parametrize("rule,p,q", [("gauss", 3, 5), ("gll", 3, 4), ("gauss", 2, 3)])
def test_helmholtz_forms(rule, p, q):
    # alpha A + beta B: with u = x (the coordinate function, in V_h on any trilinear mesh)
    # u^T (alpha A + beta B) u = alpha int |grad x|^2 + beta int x^2 = alpha + beta / 3 (exact for these rules);
    # beta = 0 annihilates constants, alpha = 0 integrates 1 to beta times the volume; symmetric; positive
    # definite for beta > 0 even without boundary conditions
    mesh = lattice_mesh(3, p, warp="B", shuffle_seed=1)
    X = fem.node_coordinates(mesh, p)
    a, b = 0.7, 2.5
    H = fem.assemble_helmholtz(mesh, p, q, rule, a, b)
    x = X[:, 0]
    assert abs(x @ (H @ x) - (a + b / 3.0)) <= 1e-12
    one = np.ones(mesh["nnodes"])
    assert np.abs(fem.assemble_helmholtz(mesh, p, q, rule, a, 0.0) @ one).max() <= 1e-12
    assert abs(one @ (fem.assemble_helmholtz(mesh, p, q, rule, 0.0, b) @ one) - b) <= 1e-12
    assert abs(H - H.T).max() <= 1e-14 * abs(H).max()
    if mesh["nnodes"] <= 400:
        assert np.linalg.eigvalsh(H.toarray())[0] > 0.0


def test_lor_degree_one_is_the_q1_operator():
    # at p = 1 the refinement is trivial: the LOR matrix is the Q1 operator with the same vertex rule
    from paper_2109_04996_amd.inputs import kappa_field_params
    m = lattice_mesh(3, 1, warp="B", shuffle_seed=2)
    kp = kappa_field_params(7, M=32)
    L = fem.assemble_lor(m, 1, kp)
    A = fem.assemble(m, 1, 2, "gll", "diffusion", kp)
    assert abs(L - A).max() <= 1e-15 * abs(A).max()


@pytest.mark.parametrize("p", [2, 3, 5])
def test_lor_invariants_and_coordinate_function(p):
    # constants in the kernel, symmetric; on mesh A (affine sub-hexes, constant detJ: the vertex rule is
    # exact for grad x . grad x detJ) the coordinate functions give x'Lx = vol = 1 and x'Ly = 0; the
    # sub-hexes fill the elements (their volumes add up to 1 on either mesh)
    for warp in ("A", "B"):
        m = lattice_mesh(3, p, warp=warp, shuffle_seed=1)
        L = fem.assemble_lor(m, p)
        assert abs(L - L.T).max() <= 1e-14 * abs(L).max()
        assert np.abs(L @ np.ones(L.shape[0])).max() <= 1e-12 * abs(L).max()
        lm = fem.lor_mesh(m, p)
        assert lm["nelem"] == m["nelem"] * p ** 3
        vol = fem.assemble(lm, 1, 3, "gauss", "mass").sum()
        assert abs(vol - 1.0) <= 1e-13
        if warp == "A":
            X = fem.node_coordinates(m, p)
            for d in range(3):
                assert abs(X[:, d] @ L @ X[:, d] - 1.0) <= 1e-12
            assert abs(X[:, 0] @ L @ X[:, 1]) <= 1e-12


def test_lor_spectral_equivalence():
    # FEM-SEM equivalence (Preconditioning section): the generalized eigenvalues of (A, L) on the free
    # nodes stay in a band independent of p, for the GLL-collocated operator, while those of (A, D)
    # spread with p. Mesh A, 2^3 (3^3 at p <= 3) elements.
    import scipy.linalg as sl
    kd = []
    for p in (2, 3, 4, 6, 8):
        N = 2 if p > 3 else 3
        m = lattice_mesh(N, p, warp="A", shuffle_seed=1)
        free = m["boundary"] == 0
        A = fem.assemble(m, p, p + 1, "gll", "diffusion")[free][:, free].toarray()
        L = fem.assemble_lor(m, p)[free][:, free].toarray()
        ev = sl.eigh(A, L, eigvals_only=True)
        assert 0.35 <= ev.min() and ev.max() <= 2.4, (p, ev.min(), ev.max())
        d = np.diag(A)
        evd = np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))
        kd.append(evd.max() / evd.min())
    assert kd[-1] > 8 * kd[0], kd  # 23.6 at p = 2, 244 at p = 8
