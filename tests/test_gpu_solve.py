"""GPU PCG solves against the oracle: iteration counts, residuals, and solutions vs a direct solve."""
import numpy as np
import scipy.sparse as sp
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fem, solvers  # noqa: E402
from paper_2109_04996_amd import hexpa as hx  # noqa: E402
from paper_2109_04996_amd.inputs import lattice_mesh  # noqa: E402
from paper_2109_04996_amd.problem import Problem  # noqa: E402


def _sine(X):
    return np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])


def _setup(N, p, q, rule, ncomp=1, warp="A", seed=0):
    """GPU operator + GPU RHS b = B f^ (mass with q = p+2 Gauss), and the oracle's matrices."""
    print(f"\n[case] solve N={N} p={p} q={q} rule={rule} ncomp={ncomp} warp={warp}", flush=True)
    mesh = lattice_mesh(N, p, warp=warp, shuffle_seed=seed)
    pr = Problem(N, p, q, rule, "diffusion", ncomp=ncomp, mesh=mesh)
    mass = Problem(N, p, p + 2, "gauss", "mass", ncomp=ncomp, mesh=mesh)
    s = np.array([1.0, -1.0, 0.5])[:ncomp]
    f = (3 * np.pi ** 2 * _sine(pr.xyz))[:, None] * s[None, :]
    b = mass.apply(pr.to_dev(f.ravel()))
    mass.close()
    A = fem.assemble(mesh, p, q, rule, "diffusion")
    B = fem.assemble(mesh, p, p + 2, "gauss", "mass")
    X = fem.node_coordinates(mesh, p)
    fo = ((3 * np.pi ** 2 * _sine(X))[:, None] * s[None, :]).ravel()
    Ak = solvers.expand(A, ncomp)
    bo = solvers.expand(B, ncomp) @ fo
    free = solvers.free_mask(mesh["boundary"], ncomp)
    return mesh, pr, b, Ak, bo, free


@pytest.mark.parametrize("N,p,q,rule", [(4, 3, 5, "gauss"), (4, 4, 5, "gll"), (3, 7, 8, "gll")])
def test_jacobi_pcg_matches_oracle(N, p, q, rule):
    mesh, pr, b, A, bo, free = _setup(N, p, q, rule)
    with pr:
        np.testing.assert_allclose(b.cpu().numpy(), bo, rtol=1e-12, atol=1e-14 * np.abs(bo).max())
        x, info = pr.solve(b, rtol=1e-8, check_every=1)
        xo, ito, reso = solvers.jacobi_pcg(A, bo, free, tol=1e-8)
        assert info["true_rel_residual"] <= 1.05e-8, info
        assert abs(info["iterations"] - ito) <= 2, (info["iterations"], ito)
        xd = solvers.direct_solve(A, bo, free)
        x = x.cpu().numpy()
        assert np.all(x[~free] == 0)
        # both stop at a 1e-8 residual: their solutions agree to the oracle's own distance from x*
        tol = 3 * np.linalg.norm(xo - xd) + 1e-12 * np.linalg.norm(xd)
        assert np.linalg.norm(x - xd) <= tol
        # tight solve: agree with the direct solve
        x2, info2 = pr.solve(b, rtol=1e-13, check_every=5)
        assert np.linalg.norm(x2.cpu().numpy() - xd) <= 1e-10 * np.linalg.norm(xd), info2


def test_vector_pcg_matches_oracle():
    mesh, pr, b, A, bo, free = _setup(3, 5, 7, "gauss", ncomp=3)
    with pr:
        x, info = pr.solve(b, rtol=1e-12)
        xd = solvers.direct_solve(A, bo, free)
        assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-9 * np.linalg.norm(xd)
        for c, sc in enumerate([1.0, -1.0, 0.5]):
            xc = x.cpu().numpy()[c::3]
            np.testing.assert_allclose(xc, sc * x.cpu().numpy()[0::3], rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("cheb_prec", [hx.HX_FP64, hx.HX_FP32])
def test_chebyshev_pcg(cheb_prec):
    mesh, pr, b, A, bo, free = _setup(4, 4, 6, "gauss", warp="B")
    with pr:
        xj, ij = pr.solve(b, rtol=1e-10)
        x, info = pr.solve(b, rtol=1e-10, precond=hx.HX_PC_CHEBYSHEV, cheb_prec=cheb_prec)
        assert info["true_rel_residual"] <= 1.05e-10
        assert info["iterations"] < ij["iterations"]
        lmax = solvers.jacobi_lambda_max(A, free)
        assert 0.8 * lmax <= info["lam_max"] <= 1.0001 * lmax, (info["lam_max"], lmax)
        xd = solvers.direct_solve(A, bo, free)
        assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-8 * np.linalg.norm(xd)


@pytest.mark.parametrize("precond,qd", [(hx.HX_PC_JACOBI, hx.HX_FP64), (hx.HX_PC_JACOBI, hx.HX_FP32),
                                        (hx.HX_PC_CHEBYSHEV, hx.HX_FP32)])
def test_iterative_refinement(precond, qd):
    mesh, pr, b, A, bo, free = _setup(4, 5, 7, "gauss", warp="B")
    with pr:
        x, info = pr.solve(b, mode=hx.HX_SOLVE_IR, precond=precond, inner_qdata=qd, rtol=1e-8)
        assert info["true_rel_residual"] <= 1.05e-8, info
        assert info["outer_iterations"] >= 2
        xd = solvers.direct_solve(A, bo, free)
        xo, _, _ = solvers.jacobi_pcg(A, bo, free, tol=1e-8)
        # error of the mixed solve is of the size of the plain FP64 solve's at the same residual
        assert np.linalg.norm(x.cpu().numpy() - xd) <= 10 * np.linalg.norm(xo - xd) + 1e-12


@pytest.mark.parametrize("ncomp,precond,qd,check", [(1, hx.HX_PC_JACOBI, hx.HX_FP64, 5), (1, hx.HX_PC_JACOBI, hx.HX_FP32, 1),
                                                    (3, hx.HX_PC_JACOBI, hx.HX_FP32, 10),
                                                    (1, hx.HX_PC_CHEBYSHEV, hx.HX_FP32, 2)])
def test_mixed_reliable_updates(ncomp, precond, qd, check):
    """FP32 PCG with FP64 residual replacement: meets the FP64 true residual, keeps the Krylov space
    (iterations close to FP64 PCG's, not the restart count of refinement), and its error is that of a
    plain FP64 solve at the same residual."""
    mesh, pr, b, A, bo, free = _setup(4, 5, 7, "gauss", ncomp=ncomp, warp="B")
    with pr:
        opts = dict(precond=precond, cheb_prec=hx.HX_FP32, rtol=1e-8, check_every=check)
        x64, i64 = pr.solve(b, **opts)
        x, info = pr.solve(b, mode=hx.HX_SOLVE_MIXED, inner_qdata=qd, **opts)
        assert info["true_rel_residual"] <= 1.05e-8, info
        # one replacement per decade of residual (reliable_delta 0.1), at least
        assert info["outer_iterations"] >= 4, info
        assert info["iterations"] <= 1.15 * i64["iterations"] + 2 * check, (info, i64)
        xd = solvers.direct_solve(A, bo, free)
        xo, _, _ = solvers.jacobi_pcg(A, bo, free, tol=1e-8)
        assert np.linalg.norm(x.cpu().numpy() - xd) <= 10 * np.linalg.norm(xo - xd) + 1e-12
        assert np.all(x.cpu().numpy()[~free] == 0)
        # a tight solve reaches the direct solution: the replacement leaves no FP32 floor
        x2, info2 = pr.solve(b, mode=hx.HX_SOLVE_MIXED, inner_qdata=qd, **dict(opts, rtol=1e-12))
        assert info2["true_rel_residual"] <= 1.05e-12, info2
        assert np.linalg.norm(x2.cpu().numpy() - xd) <= 1e-9 * np.linalg.norm(xd)
        with pytest.raises(hx.HexpaError):
            pr.solve(b, mode=hx.HX_SOLVE_MIXED, reliable_delta=1.0)


def test_failures_reported():
    mesh, pr, b, A, bo, free = _setup(3, 3, 5, "gauss")
    with pr:
        x, info = pr.solve(b, maxit=2, check_every=1, raise_on_error=False)
        assert info["status"] == "HX_ENOCONV" and info["iterations"] == 2
        bn = b.clone()
        bn[int(np.flatnonzero(free)[3])] = float("nan")
        x, info = pr.solve(bn, raise_on_error=False)
        assert info["status"] == "HX_EBREAKDOWN"
        # warm start from the converged solution: done at once
        x0, _ = pr.solve(b, rtol=1e-10)
        x1, info = pr.solve(b, x=x0.clone(), use_x0=1, rtol=1e-9, check_every=1)
        assert info["iterations"] <= 1
        zero = torch.zeros_like(b)
        x2, info = pr.solve(zero)
        assert torch.count_nonzero(x2) == 0


@pytest.mark.parametrize("mode", [hx.HX_SOLVE_FP64, hx.HX_SOLVE_IR])
@pytest.mark.parametrize("prec", [hx.HX_BF16, hx.HX_BF16_SPLIT])
def test_chebyshev_bf16_flexible(mode, prec):
    mesh, pr, b, A, bo, free = _setup(4, 6, 8, "gauss", warp="B")
    with pr:
        _, ij = pr.solve(b, rtol=1e-8)
        x, info = pr.solve(b, rtol=1e-8, mode=mode, precond=hx.HX_PC_CHEBYSHEV, cheb_prec=prec, flexible=1)
        assert info["true_rel_residual"] <= 1.05e-8, info
        assert info["iterations"] < ij["iterations"], (info, ij)
        xd = solvers.direct_solve(A, bo, free)
        xo, _, _ = solvers.jacobi_pcg(A, bo, free, tol=1e-8)
        assert np.linalg.norm(x.cpu().numpy() - xd) <= 10 * np.linalg.norm(xo - xd) + 1e-12


@pytest.mark.parametrize("form", [dict(), dict(precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP32),
                                  dict(mode=hx.HX_SOLVE_IR),
                                  dict(precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_BF16_SPLIT, flexible=1)])
def test_graph_replay_matches_eager(form):
    # the same kernels in the same order: the replayed iterations give the eager solve bit for bit,
    # in a first solve (capture + replays) and in a second one (a new capture on the same operator),
    # with the host's convergence checks and reads between the replays
    mesh, pr, b, A, bo, free = _setup(4, 6, 8, "gauss", warp="B")
    with pr:
        x0, i0 = pr.solve(b, rtol=1e-8, check_every=3, graph=0, **form)
        x1, i1 = pr.solve(b, rtol=1e-8, check_every=3, graph=1, **form)
        x2, i2 = pr.solve(b, rtol=1e-8, check_every=3, graph=1, **form)
        assert i0["iterations"] == i1["iterations"] == i2["iterations"] > 3
        assert i0["operator_applies"] == i1["operator_applies"]
        assert torch.equal(x0, x1) and torch.equal(x1, x2)
        assert i1["true_rel_residual"] <= 1.05e-8


@pytest.mark.parametrize("cheb_prec,tol", [(hx.HX_FP64, 1e-12), (hx.HX_FP32, 3e-5), (hx.HX_BF16_SPLIT, 1.2e-2),
                                           (hx.HX_BF16, 6e-2)])
def test_chebyshev_action_matches_oracle(cheb_prec, tol):
    # The preconditioner's action itself: one CG iteration from x = 0 leaves x = alpha M b (p_0 = z_0 =
    # M b), so x / |x| is the direction of the Chebyshev action M b. It is compared with the oracle's
    # recurrence (degree 4, the masked operator) on the interval the library used: lam_hi = 1.1 lam_max
    # with the library's estimate, lam_lo = lam_hi / 30. Bounds: FP64 round-off; FP32 and bf16 three
    # times the single-apply bounds of the FP32 and bf16 parity tests (degree 4 = three operator applies
    # whose terms are of the size of the result).
    mesh, pr, b, A, bo, free = _setup(4, 4, 6, "gauss", warp="B")
    with pr:
        x, info = pr.solve(b, rtol=1e-30, maxit=1, check_every=1, precond=hx.HX_PC_CHEBYSHEV, cheb_prec=cheb_prec,
                           raise_on_error=False)
        assert info["status"] == "HX_ENOCONV" and info["iterations"] == 1, info
        lam = info["lam_max"]
        lmax = solvers.jacobi_lambda_max(A, free)
        assert 0.8 * lmax <= lam <= 1.0001 * lmax
        f = free.astype(float)
        Am = sp.diags(f) @ A @ sp.diags(f)
        dinv = np.where(free, 1.0 / A.diagonal(), 0.0)
        z = solvers.chebyshev_apply(Am, dinv, bo * f, 1.1 * lam / 30.0, 1.1 * lam, 4)
        xv = x.cpu().numpy()
        d = xv / np.linalg.norm(xv) - z / np.linalg.norm(z)
        assert np.linalg.norm(d) <= tol, np.linalg.norm(d)
        assert np.all(xv[~free] == 0)


@pytest.mark.parametrize("N,p,q,rule,ncomp", [(4, 7, 8, "gll", 1), (4, 3, 5, "gauss", 1), (3, 5, 7, "gauss", 3),
                                              (3, 6, 8, "gauss", 1)])
def test_node_gather_cg_matches_colored(N, p, q, rule, ncomp):
    # The CG operator as one E-vector launch plus a node gather with p'Ap fused (HX_SCATTER_GATHER):
    # the same iteration as the colored scatter up to summation order -- iterations within 2, the same
    # solution to the solve's own accuracy, deterministic bits, and the oracle's direct solution at 1e-12
    mesh, pr, b, A, bo, free = _setup(N, p, q, rule, ncomp=ncomp, warp="B")
    with pr:
        x0, i0 = pr.solve(b, rtol=1e-10, check_every=1)
        x1, i1 = pr.solve(b, rtol=1e-10, check_every=1, scatter=hx.HX_SCATTER_GATHER)
        x2, i2 = pr.solve(b, rtol=1e-10, check_every=1, scatter=hx.HX_SCATTER_GATHER)
        assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]
        assert abs(i1["iterations"] - i0["iterations"]) <= 2, (i0, i1)
        assert i1["true_rel_residual"] <= 1.05e-10
        xd = solvers.direct_solve(A, bo, free)
        x3, _ = pr.solve(b, rtol=1e-13, check_every=5, scatter=hx.HX_SCATTER_GATHER)
        assert np.linalg.norm(x3.cpu().numpy() - xd) <= 1e-10 * np.linalg.norm(xd)
        # graph replay of the gather iteration: bit for bit the eager one
        x4, i4 = pr.solve(b, rtol=1e-10, check_every=1, scatter=hx.HX_SCATTER_GATHER, graph=1)
        assert torch.equal(x1, x4) and i4["iterations"] == i1["iterations"]
