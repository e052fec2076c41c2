"""GPU p-multigrid against the oracle: transfers, one V-cycle, and flexible-CG solves.

Transfers are compared element by element with the oracle's assembled
interpolation matrix P and its transpose, on meshes with randomly rotated
elements (the same rotations on every level) and element counts that leave a
ragged last workgroup. The V-cycle is compared with the oracle's V-cycle given
the same lam_max per level (the library's Lanczos estimates) and a coarse
Jacobi-PCG of a fixed iteration count, so both compute the same map.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fem, pmg, solvers  # noqa: E402
from paper_2109_04996_amd import hexpa as hx  # noqa: E402
from paper_2109_04996_amd.inputs import lattice_mesh, rotate_elements, uniform_vector  # noqa: E402
from paper_2109_04996_amd.problem import Hierarchy  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _meshes(N, degrees, warp, frac, seed=0):
    ms = [lattice_mesh(N, p, warp=warp, shuffle_seed=seed) for p in degrees]
    if frac > 0:
        ms = [rotate_elements(m, p, frac, seed=3) for m, p in zip(ms, degrees)]
    return ms


@pytest.mark.parametrize("N,degrees,warp,frac", [(5, (4, 2), "B", 0.2), (4, (7, 3, 1), "A", 0.0),
                                                 (3, (8, 4), "B", 0.3), (9, (2, 1), "B", 0.2),
                                                 (3, (6, 5), "A", 0.0), (1, (4, 2), "A", 0.0),
                                                 (2, (3, 1), "B", 0.0)])
def test_transfers_match_oracle(N, degrees, warp, frac):
    print(f"\n[case] pmg transfers N={N} degrees={degrees} warp={warp} rotated={frac}", flush=True)
    ms = _meshes(N, degrees, warp, frac)
    with Hierarchy(N, degrees, meshes=ms) as H:
        for l in range(len(degrees) - 1):
            P = pmg.prolongation(ms[l], ms[l + 1], degrees[l], degrees[l + 1])
            xc = uniform_vector(ms[l + 1]["nnodes"], 10 + l)
            rf = uniform_vector(ms[l]["nnodes"], 20 + l)
            y = H.prolong(l, H.levels[l + 1].to_dev(xc)).cpu().numpy()
            yr = P @ xc
            assert np.max(np.abs(y - yr)) <= 1e-14 * (np.abs(P) @ np.abs(xc)).max()
            assert rel(y, yr) <= 1e-14
            z = H.restrict(l, H.levels[l].to_dev(rf)).cpu().numpy()
            zr = P.T @ rf
            assert rel(z, zr) <= 1e-13
            assert np.max(np.abs(z - zr)) <= 1e-13 * (np.abs(P).T @ np.abs(rf)).max()
            # deterministic: the same bits twice
            assert torch.equal(H.restrict(l, H.levels[l].to_dev(rf)), H.restrict(l, H.levels[l].to_dev(rf)))


@pytest.mark.parametrize("N,degrees,rule,kind,warp,frac", [(4, (4, 2, 1), "gll", "diffusion", "B", 0.2),
                                                           (3, (7, 3), "gll", "diffusion", "A", 0.0),
                                                           # one element: the coarsest level has no free node
                                                           (1, (4, 2, 1), "gll", "diffusion", "A", 0.0),
                                                           (3, (5, 2, 1), "gauss", "diffusion", "B", 0.0),
                                                           (4, (3, 1), "gauss", "mass", "B", 0.0)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vcycle_matches_oracle(N, degrees, rule, kind, warp, frac, prec):
    print(f"\n[case] pmg V-cycle N={N} degrees={degrees} {rule} {kind} warp={warp} {prec}", flush=True)
    ms = _meshes(N, degrees, warp, frac)
    opts = dict(smooth_degree=3, smooth_ratio=15.0, coarse_maxit=8, coarse_rtol=0.0,
                prec=hx.HX_FP64 if prec == "fp64" else hx.HX_FP32)
    with Hierarchy(N, degrees, rule=rule, kind=kind, meshes=ms, **opts) as H:
        levels = []
        for l, (m, p) in enumerate(zip(ms, degrees)):
            q = p + 1 if rule == "gll" else p + 2
            A = fem.assemble(m, p, q, rule, kind)
            free = solvers.free_mask(m["boundary"])
            P = pmg.prolongation(m, ms[l + 1], p, degrees[l + 1]) if l + 1 < len(degrees) else None
            lam = H.lambda_max(l) if P is not None else 0.0
            if P is not None:  # the library's estimate is a Lanczos value from below
                lam_ref = solvers.jacobi_lambda_max(A, free)
                assert 0.9 * lam_ref <= lam <= lam_ref * (1 + 1e-12), (lam, lam_ref)
            levels.append(pmg.Level(A, free, lam, P))
        r = uniform_vector(ms[0]["nnodes"], 5) * levels[0].f
        zd = H.vcycle(H.fine.to_dev(r))
        assert torch.equal(zd, H.vcycle(H.fine.to_dev(r)))  # the same bits twice
        z = zd.cpu().numpy()
        zr = pmg.vcycle(levels, r, degree=3, ratio=15.0, coarse_rtol=0.0, coarse_maxit=8)
        assert np.all(z[~levels[0].free] == 0)
        # FP32: single-precision smoothers and an 8-step FP32 coarse CG (FP64 reductions and transfers)
        tol = 1e-10 if prec == "fp64" else 1e-4
        assert rel(z, zr) <= tol, rel(z, zr)


def _rhs(H):
    """b = B f^ with f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z), through the library's mass operator."""
    from paper_2109_04996_amd.problem import Problem
    fine = H.fine
    X = fine.xyz
    f = 3 * np.pi ** 2 * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    with Problem(fine.N, fine.p, fine.p + 2, "gauss", "mass", mesh=fine.mesh) as M:
        return M.apply(fine.to_dev(f))


@pytest.mark.parametrize("N,degrees,rule", [(6, (4, 2, 1), "gll"), (4, (7, 3, 1), "gll"), (4, (5, 2, 1), "gauss")])
@pytest.mark.parametrize("coarse_rtol,prec", [(0.0, "fp64"), (1e-2, "fp64"), (1e-1, "fp32")])
def test_pmg_solve(N, degrees, rule, coarse_rtol, prec):
    print(f"\n[case] pmg solve N={N} degrees={degrees} {rule} coarse_rtol={coarse_rtol} {prec}", flush=True)
    with Hierarchy(N, degrees, rule=rule, warp="B", coarse_maxit=20, coarse_rtol=coarse_rtol,
                   prec=hx.HX_FP64 if prec == "fp64" else hx.HX_FP32) as H:
        b = _rhs(H)
        x, info = H.solve(b, rtol=1e-8, check_every=1)
        assert info["true_rel_residual"] <= 1.05e-8, info
        _, info_j = H.fine.solve(b, rtol=1e-8, check_every=1)
        assert info["iterations"] * 3 < info_j["iterations"], (info["iterations"], info_j["iterations"])
        m, p = H.fine.mesh, degrees[0]
        q = p + 1 if rule == "gll" else p + 2
        A = fem.assemble(m, p, q, rule, "diffusion")
        free = solvers.free_mask(m["boundary"])
        xd = solvers.direct_solve(A, b.cpu().numpy(), free)
        assert np.all(x.cpu().numpy()[~free] == 0)
        # a tight solve reaches the direct solution
        x2, info2 = H.solve(b, rtol=1e-12, check_every=1)
        assert rel(x2.cpu().numpy(), xd) <= 1e-9, info2


def test_pmg_rejects_bad_hierarchies():
    N = 3
    ms = [lattice_mesh(N, 4, warp="B", shuffle_seed=0), lattice_mesh(N, 2, warp="B", shuffle_seed=1)]
    with pytest.raises(hx.HexpaError, match="geometry"):
        Hierarchy(N, (4, 2), meshes=ms)
    with pytest.raises(hx.HexpaError, match="decrease"):
        Hierarchy(N, (2, 4))
    with pytest.raises(hx.HexpaError, match="smooth_degree"):
        Hierarchy(N, (2, 1), smooth_degree=0)
    with pytest.raises(hx.HexpaError, match="prec must be"):
        Hierarchy(N, (2, 1), prec=7)
    with pytest.raises(hx.HexpaError, match="bf16 p-multigrid needs"):
        Hierarchy(N, (2, 1), rule="gauss", kind="mass", prec=hx.HX_BF16)
    with Hierarchy(N, (2, 1)) as H:
        b = H.fine.zeros()
        with pytest.raises(hx.HexpaError, match="needs opts.pmg"):
            H.fine.solve(b, precond=hx.HX_PC_PMG)
        with pytest.raises(hx.HexpaError, match="HX_SOLVE_FP64"):
            H.solve(b, mode=hx.HX_SOLVE_IR)
        with pytest.raises(hx.HexpaError, match="level out of range"):
            hx.hx_pmg_prolong(H.h, 1, b, b)
        assert hx.hx_pmg_levels(H.h) == 2


def test_pmg_solve_variable_coefficient():
    """Diffusion with the seeded kappa field (contrast ~1e2) on every level, Gauss q = p + 2."""
    from paper_2109_04996_amd.inputs import kappa_field_params
    print("\n[case] pmg solve kappa seed 100 N=8 degrees=(6, 3, 1) gauss", flush=True)
    kp = kappa_field_params(100, M=512)
    for prec in (hx.HX_FP64, hx.HX_FP32):
        with Hierarchy(8, (6, 3, 1), rule="gauss", kappa=kp, prec=prec) as H:
            b = H.fine.to_dev(uniform_vector(H.fine.n, 2) * (H.fine.mesh["boundary"] == 0))
            x, info = H.solve(b, rtol=1e-8, check_every=1)
            assert info["true_rel_residual"] <= 1.05e-8, info
            _, info_j = H.fine.solve(b, rtol=1e-8, check_every=1)
            assert info["iterations"] * 3 < info_j["iterations"], (info["iterations"], info_j["iterations"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vector_hierarchy_matches_oracle(prec):
    """Three interleaved components (index 3 node + c): transfers against kron(P, I_3), one V-cycle against
    the oracle's on the expanded matrices (its coarse CG is one CG over all components, like the library's)."""
    import scipy.sparse as sp
    N, degrees = 3, (4, 2, 1)
    print(f"\n[case] pmg vector N={N} degrees={degrees} {prec}", flush=True)
    ms = _meshes(N, degrees, "B", 0.2)
    opts = dict(smooth_degree=3, smooth_ratio=15.0, coarse_maxit=8, coarse_rtol=0.0,
                prec=hx.HX_FP64 if prec == "fp64" else hx.HX_FP32)
    with Hierarchy(N, degrees, meshes=ms, ncomp=3, **opts) as H:
        levels = []
        for l, (m, p) in enumerate(zip(ms, degrees)):
            A = solvers.expand(fem.assemble(m, p, p + 1, "gll", "diffusion"), 3)
            free = solvers.free_mask(m["boundary"], 3)
            P = None
            if l + 1 < len(degrees):
                P = sp.kron(pmg.prolongation(m, ms[l + 1], p, degrees[l + 1]), sp.identity(3), format="csr")
                xc = uniform_vector(ms[l + 1]["nnodes"], 30 + l, 3)
                rf = uniform_vector(m["nnodes"], 40 + l, 3)
                assert rel(H.prolong(l, H.levels[l + 1].to_dev(xc)).cpu().numpy(), P @ xc) <= 1e-14
                assert rel(H.restrict(l, H.levels[l].to_dev(rf)).cpu().numpy(), P.T @ rf) <= 1e-13
            levels.append(pmg.Level(A, free, H.lambda_max(l) if P is not None else 0.0, P))
        r = uniform_vector(ms[0]["nnodes"], 5, 3) * levels[0].f
        z = H.vcycle(H.fine.to_dev(r)).cpu().numpy()
        zr = pmg.vcycle(levels, r, degree=3, ratio=15.0, coarse_rtol=0.0, coarse_maxit=8)
        assert np.all(z[~levels[0].free] == 0)
        assert rel(z, zr) <= (1e-10 if prec == "fp64" else 1e-4), rel(z, zr)


def test_vector_pmg_solve():
    """BP4-type vector diffusion (Gauss q = p + 2, three components with different right-hand sides)."""
    print("\n[case] pmg vector solve N=4 degrees=(5, 2, 1) gauss", flush=True)
    with Hierarchy(4, (5, 2, 1), rule="gauss", warp="B", ncomp=3) as H:
        b = H.fine.to_dev(uniform_vector(H.fine.mesh["nnodes"], 2, 3)
                          * np.repeat(H.fine.mesh["boundary"] == 0, 3))
        x, info = H.solve(b, rtol=1e-8, check_every=1)
        assert info["true_rel_residual"] <= 1.05e-8, info
        _, info_j = H.fine.solve(b, rtol=1e-8, check_every=1)
        assert info["iterations"] * 3 < info_j["iterations"], (info["iterations"], info_j["iterations"])


@pytest.mark.parametrize("prec", ["bf16", "bf16split"])
@pytest.mark.parametrize("N,degrees,rule", [(4, (7, 3, 1), "gll"), (4, (6, 3, 1), "gauss")])
def test_pmg_bf16_finest_level(N, degrees, rule, prec):
    """An FP32 hierarchy whose finest level smooths on the bf16 matrix cores: the V-cycle stays close to
    the FP64 one (a smoother needs about one digit) and the FP64 flexible CG still reaches 1e-8."""
    pv = hx.HX_BF16 if prec == "bf16" else hx.HX_BF16_SPLIT
    print(f"\n[case] pmg bf16 N={N} degrees={degrees} {rule} {prec}", flush=True)
    opts = dict(rule=rule, warp="B", coarse_maxit=8, coarse_rtol=0.0)
    with Hierarchy(N, degrees, **opts) as H64, Hierarchy(N, degrees, prec=pv, **opts) as Hb:
        r = H64.fine.to_dev(uniform_vector(H64.fine.n, 5) * (H64.fine.mesh["boundary"] == 0))
        z64 = H64.vcycle(r)
        zb = Hb.vcycle(r)
        err = float(torch.linalg.norm(zb - z64) / torch.linalg.norm(z64))
        assert err <= (1e-1 if prec == "bf16" else 3e-2), err
        b = _rhs(Hb)
        _, info = Hb.solve(b, rtol=1e-8, check_every=1)
        assert info["true_rel_residual"] <= 1.05e-8, info
        _, info64 = H64.solve(b, rtol=1e-8, check_every=1)
        assert info["iterations"] <= 2 * info64["iterations"] + 2, (info["iterations"], info64["iterations"])



def test_pmg_solve_from_initial_guess():
    """use_x0: a loose solve, then the tight one started from its result (the outer CG corrects x0)."""
    print("\n[case] pmg warm start N=5 degrees=(4, 2, 1) gll", flush=True)
    with Hierarchy(5, (4, 2, 1), warp="B") as H:
        b = _rhs(H)
        x_full, info_full = H.solve(b, rtol=1e-10, check_every=1)
        x0, info0 = H.solve(b, rtol=1e-4, check_every=1)
        x, info = H.solve(b, x=x0.clone(), rtol=1e-10, check_every=1, use_x0=1)
        assert info["true_rel_residual"] <= 1.05e-10, info
        assert info["iterations"] < info_full["iterations"], (info["iterations"], info_full["iterations"])
        assert float(torch.linalg.norm(x - x_full) / torch.linalg.norm(x_full)) <= 1e-8
