"""The solve that allocates nothing (hx_pcg_solve_noalloc) against hx_pcg_solve, through the C ABI.

Both run the same kernels in the same order on the same inputs, so the solutions, iteration counts
and residuals must agree bit for bit. Two calls in a row share the device's scratch array, the
second on a smaller problem with three components, and a third call goes back to the first problem
once hx_pcg_solve has cached its diagonal.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2109_04996_amd import hexpa as hx  # noqa: E402
from paper_2109_04996_amd.inputs import lattice_mesh, uniform_vector  # noqa: E402
from paper_2109_04996_amd.problem import Problem  # noqa: E402


def _problem(N, p, q, rule, ncomp, warp):
    print(f"\n[case] no-alloc solve N={N} p={p} q={q} rule={rule} ncomp={ncomp} warp={warp}", flush=True)
    mesh = lattice_mesh(N, p, warp=warp, shuffle_seed=0)
    pr = Problem(N, p, q, rule, "diffusion", ncomp=ncomp, mesh=mesh)
    free = np.repeat(~mesh["boundary"].astype(bool), ncomp)
    b = pr.to_dev(uniform_vector(pr.n, 2) * free)
    return pr, b, free


def _both(pr, b, **opts):
    o = hx.hx_solve_opts_default(**opts)
    xa = torch.full((pr.n,), 7.0, dtype=torch.float64, device="cuda")  # stale values: both overwrite x
    ia = hx.hx_pcg_solve_noalloc(pr.h_op, b, xa, o)
    xb = pr.zeros()
    ib = hx.hx_pcg_solve(pr.h_op, b, xb, o)
    return xa.cpu().numpy(), ia, xb.cpu().numpy(), ib


def _same(xa, ia, xb, ib, free, rtol):
    np.testing.assert_array_equal(xa, xb)
    assert np.all(xa[~free] == 0)
    for k in ("iterations", "operator_applies", "rel_residual", "true_rel_residual"):
        assert ia[k] == ib[k], (k, ia, ib)
    assert ia["true_rel_residual"] <= 1.05 * rtol, ia


def test_noalloc_solve_matches_pcg_solve_twice_then_smaller():
    big, b_big, f_big = _problem(8, 5, 6, "gll", 1, "B")       # 68,921 DOFs
    small, b_small, f_small = _problem(3, 4, 6, "gauss", 3, "A")  # 3 x 2,197 DOFs
    with big, small:
        assert big.n <= hx.HX_NOALLOC_MAX_DOFS
        # first call: no cached diagonal, it is computed into the scratch array
        xa, ia, xb, ib = _both(big, b_big, rtol=1e-9, check_every=3)
        _same(xa, ia, xb, ib, f_big, 1e-9)
        # second call, smaller and with three components: the larger call's contents must not leak
        xa, ia, xb, ib = _both(small, b_small, rtol=1e-10, check_every=1)
        _same(xa, ia, xb, ib, f_small, 1e-10)
        # back to the first problem: hx_pcg_solve has cached its diagonal, which is used now
        o = hx.hx_solve_opts_default(rtol=1e-9, check_every=3)
        xc = big.zeros()
        ic = hx.hx_pcg_solve_noalloc(big.h_op, b_big, xc, o)
        xd = big.zeros()
        idd = hx.hx_pcg_solve(big.h_op, b_big, xd, o)
        _same(xc.cpu().numpy(), ic, xd.cpu().numpy(), idd, f_big, 1e-9)


def test_noalloc_unpreconditioned_and_warm_start():
    pr, b, free = _problem(3, 3, 5, "gauss", 1, "B")
    with pr:
        xa, ia, xb, ib = _both(pr, b, precond=hx.HX_PC_NONE, rtol=1e-10, check_every=1)
        _same(xa, ia, xb, ib, free, 1e-10)
        # warm start from a loose solve's iterate
        o = hx.hx_solve_opts_default(rtol=1e-3)
        x0 = pr.zeros()
        hx.hx_pcg_solve(pr.h_op, b, x0, o)
        o2 = hx.hx_solve_opts_default(rtol=1e-10, use_x0=1, check_every=2)
        xa, xb = x0.clone(), x0.clone()
        ia = hx.hx_pcg_solve_noalloc(pr.h_op, b, xa, o2)
        ib = hx.hx_pcg_solve(pr.h_op, b, xb, o2)
        _same(xa.cpu().numpy(), ia, xb.cpu().numpy(), ib, free, 1e-10)


def test_noalloc_rejects_what_it_does_not_serve():
    pr, b, free = _problem(2, 2, 4, "gauss", 1, "A")
    with pr:
        x = pr.zeros()
        for opts, code in [({"precond": hx.HX_PC_CHEBYSHEV}, hx.HX_EUNSUPPORTED),
                           ({"mode": hx.HX_SOLVE_IR}, hx.HX_EUNSUPPORTED),
                           ({"scatter": hx.HX_SCATTER_GATHER}, hx.HX_EUNSUPPORTED),
                           ({"graph": 1}, hx.HX_EUNSUPPORTED),
                           ({"rtol": 0.0}, hx.HX_EINVAL)]:
            with pytest.raises(hx.HexpaError) as e:
                hx.hx_pcg_solve_noalloc(pr.h_op, b, x, hx.hx_solve_opts_default(**opts))
            assert e.value.code == code, opts
    # one node row past the limit: (7 * 15 + 1)^3 = 1,191,016 > 1,048,576
    big = Problem(15, 7, 8, "gll", "diffusion", warp="A")
    with big:
        assert big.n > hx.HX_NOALLOC_MAX_DOFS
        x = big.zeros()
        with pytest.raises(hx.HexpaError) as e:
            hx.hx_pcg_solve_noalloc(big.h_op, x, x, hx.hx_solve_opts_default())
        assert e.value.code == hx.HX_EINVAL
        assert "HX_NOALLOC_MAX_DOFS" in hx.hx_last_error()
