"""Pins of the oracle's solves, Chebyshev preconditioner and MLP."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import fem, mlp, solvers
from paper_2109_04996_amd.inputs import lattice_mesh


def _problem(N=3, p=3, warp="B"):
    mesh = lattice_mesh(N, p, warp=warp, shuffle_seed=0)
    A = fem.assemble(mesh, p, p + 2, "gauss", "diffusion")
    B = fem.assemble(mesh, p, p + 2, "gauss", "mass")
    X = fem.node_coordinates(mesh, p)
    f = 3 * np.pi ** 2 * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    free = solvers.free_mask(mesh["boundary"])
    return mesh, A, B @ f, free


def test_jacobi_pcg_matches_direct():
    mesh, A, b, free = _problem()
    x_ref = solvers.direct_solve(A, b, free)
    x, it, res = solvers.jacobi_pcg(A, b, free, tol=1e-12)
    assert res <= 1e-12
    assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    assert np.all(x[~free] == 0)
    # CG converges in at most n_free steps in exact arithmetic; here far fewer
    assert 5 < it < free.sum()


def test_pcg_residual_criterion():
    mesh, A, b, free = _problem()
    x, it, res = solvers.jacobi_pcg(A, b, free, tol=1e-8)
    r = (b - A @ x) * free
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b * free) * (1 + 1e-6)
    assert abs(res - np.linalg.norm(r) / np.linalg.norm(b * free)) < 1e-15


def _chebyshev_by_eigen(A, dinv, r, lo, hi, k, free):
    # z = D^-1/2 V s(Lambda) V^T D^-1/2 r with s(l) = (1 - T_k(theta(l))/T_k(theta(0))) / l
    Aii = A[free][:, free].toarray()
    d = 1.0 / dinv[free]
    S = Aii / np.sqrt(np.outer(d, d))
    lam, V = np.linalg.eigh(S)
    th = lambda l: (hi + lo - 2 * l) / (hi - lo)
    Tk = lambda t: C.chebval(t, [0] * k + [1])
    s = (1 - Tk(th(lam)) / Tk(th(0.0))) / lam
    z = np.zeros_like(r)
    rs = r[free] / np.sqrt(d)
    z[free] = (V @ (s * (V.T @ rs))) / np.sqrt(d)
    return z


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_chebyshev_recurrence_equals_polynomial(k):
    mesh, A, b, free = _problem(N=3, p=2)
    f = free.astype(float)
    Am = (A.multiply(np.outer(f, f))).tocsr()
    dinv = np.where(free, 1.0 / A.diagonal(), 0.0)
    lmax = solvers.jacobi_lambda_max(A, free)
    lo, hi = lmax * 1.1 / 30, lmax * 1.1
    r = np.random.default_rng(3).standard_normal(b.size) * f
    z = solvers.chebyshev_apply(Am, dinv, r, lo, hi, k)
    zr = _chebyshev_by_eigen(A, dinv, r, lo, hi, k, free)
    np.testing.assert_allclose(z, zr, rtol=1e-10, atol=1e-12 * np.abs(zr).max())


def test_chebyshev_general_base_map():
    # the recurrence with a base map v -> M v in place of D^-1 (the learned smoother's form):
    # (a) M = D^-1 as a map gives the array path bit for bit;
    # (b) M a general SPD matrix on the free nodes (not diagonal): z = M^1/2 V s(L) V^T M^1/2 r with
    #     (L, V) the eigenpairs of M^1/2 A M^1/2, s(l) = (1 - T_k(theta(l)) / T_k(theta(0))) / l;
    # (c) M = A^-1 on the free nodes: z = s(1) A^-1 r.
    mesh, A, b, free = _problem(N=3, p=2)
    f = free.astype(float)
    Am = (A.multiply(np.outer(f, f))).tocsr()
    dinv = np.where(free, 1.0 / A.diagonal(), 0.0)
    r = np.random.default_rng(4).standard_normal(b.size) * f
    lmax = solvers.jacobi_lambda_max(A, free)
    lo, hi = lmax * 1.1 / 30, lmax * 1.1
    k = 4
    np.testing.assert_array_equal(solvers.chebyshev_apply(Am, lambda v: dinv * v, r, lo, hi, k),
                                  solvers.chebyshev_apply(Am, dinv, r, lo, hi, k))
    nf = int(free.sum())
    Aii = A[free][:, free].toarray()
    G = np.random.default_rng(5).standard_normal((nf, nf)) / np.sqrt(nf)
    Mf = np.diag(dinv[free]) + 0.02 * (G @ G.T) * dinv[free].mean()  # SPD, far from diagonal
    M = lambda v: _embed(Mf @ v[free], free)
    w, U = np.linalg.eigh(Mf)
    Mh = (U * np.sqrt(w)) @ U.T
    lam, V = np.linalg.eigh(Mh @ Aii @ Mh)
    lo2, hi2 = lam.max() * 1.1 / 30, lam.max() * 1.1
    th = lambda l: (hi2 + lo2 - 2 * l) / (hi2 - lo2)
    Tk = lambda t: C.chebval(t, [0] * k + [1])
    sv = (1 - Tk(th(lam)) / Tk(th(0.0))) / lam
    zr = _embed(Mh @ (V @ (sv * (V.T @ (Mh @ r[free])))), free)
    z = solvers.chebyshev_apply(Am, M, r, lo2, hi2, k)
    np.testing.assert_allclose(z, zr, rtol=1e-9, atol=1e-11 * np.abs(zr).max())
    Ainv = np.linalg.inv(Aii)
    z = solvers.chebyshev_apply(Am, lambda v: _embed(Ainv @ v[free], free), r, lo, hi, k)
    s1 = 1 - Tk((hi + lo - 2.0) / (hi - lo)) / Tk((hi + lo) / (hi - lo))
    np.testing.assert_allclose(z, s1 * _embed(Ainv @ r[free], free), rtol=1e-10, atol=1e-12 * np.abs(z).max())


def _embed(vf, free):
    out = np.zeros(free.size)
    out[free] = vf
    return out


def test_chebyshev_is_spd_and_pcg_converges():
    mesh, A, b, free = _problem(N=3, p=3)
    lmax = solvers.jacobi_lambda_max(A, free)
    x_ref = solvers.direct_solve(A, b, free)
    x, it, res = solvers.chebyshev_pcg(A, b, free, lmax * 1.1 / 30, lmax * 1.1, 4, tol=1e-10)
    assert res <= 1e-10
    _, itj, _ = solvers.jacobi_pcg(A, b, free, tol=1e-10)
    assert it < itj  # 3 extra applies per iteration buy fewer iterations
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


def test_lambda_max_dense():
    mesh, A, b, free = _problem(N=3, p=1)
    Aii = A[free][:, free].toarray()
    d = np.diag(Aii)
    ev = np.linalg.eigvals(Aii / d[:, None])
    assert abs(solvers.jacobi_lambda_max(A, free) - ev.real.max()) < 1e-10


def test_lambda_max_lanczos_branch():
    # more than 64 free nodes (N = 3, p = 2: 125): the sparse Lanczos branch, against the dense
    # eigenvalues of the non-symmetric D^-1 A_II computed without the symmetric scaling
    mesh, A, b, free = _problem(N=3, p=2)
    assert int(free.sum()) > 64
    Aii = A[free][:, free].toarray()
    ev = np.linalg.eigvals(Aii / np.diag(Aii)[:, None])
    assert abs(ev.imag).max() < 1e-10
    assert abs(solvers.jacobi_lambda_max(A, free) - ev.real.max()) < 1e-9 * ev.real.max()


def test_mlp_gradients_finite_differences():
    rng = np.random.default_rng(0)
    params = mlp.init_params(10, 7, 4, seed=7)
    params["b1"] = rng.standard_normal(7) * 0.1
    params["b2"] = rng.standard_normal(4) * 0.1
    X = rng.standard_normal((5, 10))
    T = rng.standard_normal((5, 4))
    _, g = mlp.loss_and_grads(params, X, T)
    h = 1e-6
    for k, v in params.items():
        num = np.zeros_like(v)
        for idx in np.ndindex(v.shape):
            old = v[idx]
            v[idx] = old + h
            lp = mlp.loss(params, X, T)
            v[idx] = old - h
            lm = mlp.loss(params, X, T)
            v[idx] = old
            num[idx] = (lp - lm) / (2 * h)
        assert np.linalg.norm(num - g[k]) <= 1e-7 * np.linalg.norm(g[k]), k


def test_mlp_zero_loss_and_linear_limit():
    # targets equal to the outputs: zero loss and zero gradient
    params = mlp.init_params(6, 5, 3, seed=1)
    X = np.random.default_rng(2).standard_normal((4, 6))
    Y, _ = mlp.forward(params, X)
    L, g = mlp.loss_and_grads(params, X, Y)
    assert L == 0.0 and all(np.all(v == 0) for v in g.values())
    # tiny inputs: tanh is the identity to first order, so y ~= W2 W1 x + b2
    Xs = 1e-6 * X
    Ys, _ = mlp.forward(params, Xs)
    lin = Xs @ (params["W2"] @ params["W1"]).T + params["b2"]
    assert np.abs(Ys - lin).max() < 1e-16 + 1e-12 * np.abs(lin).max()


def test_adam_first_step_closed_form():
    # after one step from zero moments, m_hat = g and v_hat = g^2: the update is lr * g / (|g| + eps)
    params = dict(w=np.array([1.0, -2.0, 3.0]))
    g = dict(w=np.array([0.5, -1e-3, 0.0]))
    st = {}
    mlp.adam_step(params, g, st, lr=0.1, eps=1e-8)
    exp = np.array([1.0, -2.0, 3.0]) - 0.1 * g["w"] / (np.abs(g["w"]) + 1e-8)
    np.testing.assert_allclose(params["w"], exp, rtol=1e-14)
