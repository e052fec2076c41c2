"""p-multigrid V-cycle on assembled matrices, FP64 (oracle; test infrastructure only).

Preconditioning section: multigrid over a hierarchy of polynomial degrees on one
mesh (p-multigrid), with matrix-free smoothers, is named as the route to
matrix-free solvers; the paper fixes neither the degree schedule, the smoother
nor the coarse solver. The readings taken here:

* the levels share the mesh and its elements; level l + 1 has a lower degree;
* the prolongation is interpolation: a continuous function of the coarse space,
  given by its values at the coarse GLL nodes, is evaluated at the fine GLL
  nodes (so it is exact on the coarse space, which lies inside the fine one);
  the restriction is its transpose;
* smoother: Chebyshev acceleration of D^-1 A (``solvers.chebyshev_apply``),
  ``degree`` steps, before and after the coarse correction, on the interval
  [lam_hi / ratio, lam_hi]; a level may replace D^-1 by another base map M
  (the learned element map), with lam_max that of M A;
* coarsest level: Jacobi-PCG (``solvers.jacobi_pcg``), to a relative tolerance
  or, with tolerance 0, for exactly ``coarse_maxit`` iterations.

Every level carries homogeneous Dirichlet conditions by masking: residuals,
corrections and smoother outputs are zero at constrained nodes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .quadrature import gll_rule, lagrange_table
from .solvers import chebyshev_apply, direct_solve, jacobi_pcg


def interpolation_1d(p_fine: int, p_coarse: int) -> np.ndarray:
    """I[i, a] = l_a(xi_i): the coarse Lagrange basis (GLL nodes of degree p_coarse) at the fine GLL nodes."""
    xf, _ = gll_rule(p_fine)
    xc, _ = gll_rule(p_coarse)
    return lagrange_table(xc, xf)


def prolongation(mesh_f: dict, mesh_c: dict, p_fine: int, p_coarse: int) -> sp.csr_matrix:
    """The n_fine x n_coarse interpolation matrix.

    Element e holds fine local node (i, j, k) and coarse local node (a, b, c);
    the value at a fine node is sum_abc I[i,a] I[j,b] I[k,c] u_c(a, b, c). A
    fine node shared by several elements takes its row from the first of them
    in element order (every one gives the same function values, since the
    coarse function is continuous).
    """
    I = interpolation_1d(p_fine, p_coarse)
    I3 = np.kron(I, np.kron(I, I))  # row i + Pf (j + Pf k), column a + Pc (b + Pc c)
    nf, nc = mesh_f["nnodes"], mesh_c["nnodes"]
    assert mesh_f["nelem"] == mesh_c["nelem"]
    done = np.zeros(nf, bool)
    rows, cols, vals = [], [], []
    for e in range(mesh_f["nelem"]):
        fn = mesh_f["elem_nodes"][e]
        cn = mesh_c["elem_nodes"][e]
        for loc in range(fn.size):
            g = fn[loc]
            if done[g]:
                continue
            done[g] = True
            rows.append(np.full(cn.size, g))
            cols.append(cn)
            vals.append(I3[loc])
    assert done.all(), "a fine node belongs to no element"
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nf, nc))


class Level:
    """One level: its assembled operator, free mask, Chebyshev interval and the prolongation from the next level.

    ``base``: the smoother's base map v -> M v (default: D^-1 of the level); lam_max is then that of M A."""

    def __init__(self, A: sp.csr_matrix, free: np.ndarray, lam_max: float = 0.0, P: sp.csr_matrix | None = None,
                 base=None):
        self.free = free
        self.f = free.astype(float)
        self.A_full = A
        self.A = sp.diags(self.f) @ A @ sp.diags(self.f)  # masked operator
        self.dinv = np.where(free, 1.0 / A.diagonal(), 0.0)
        self.lam_max = lam_max
        self.P = P
        self.base = base


def vcycle(levels: list, r: np.ndarray, degree: int = 2, ratio: float = 10.0, coarse_rtol: float = 0.0,
           coarse_maxit: int = 20, coarse: str = "pcg", l: int = 0) -> np.ndarray:
    """z = V_l r, the V-cycle from level l (0 = finest) applied to a residual r.

    lam_hi = 1.1 lam_max of each level's D^-1 A. ``coarse='direct'`` solves the
    coarsest level exactly (sparse LU) in place of Jacobi-PCG.
    """
    lv = levels[l]
    r = r * lv.f
    if l == len(levels) - 1:
        if coarse == "direct":
            return direct_solve(lv.A_full, r, lv.free)
        x, _, _ = jacobi_pcg(lv.A_full, r, lv.free, tol=coarse_rtol, maxit=coarse_maxit)
        return x
    lam_hi = 1.1 * lv.lam_max
    lam_lo = lam_hi / ratio
    M = lv.dinv if lv.base is None else lv.base
    x = chebyshev_apply(lv.A, M, r, lam_lo, lam_hi, degree)  # pre-smoothing from 0
    t = (r - lv.A @ x) * lv.f
    rc = lv.P.T @ t
    ec = vcycle(levels, rc, degree, ratio, coarse_rtol, coarse_maxit, coarse, l + 1)
    x = x + (lv.P @ ec) * lv.f  # coarse correction
    t = (r - lv.A @ x) * lv.f
    return x + chebyshev_apply(lv.A, M, t, lam_lo, lam_hi, degree)  # post-smoothing


def flexible_pcg(A: sp.csr_matrix, b: np.ndarray, free: np.ndarray, precond, tol: float = 1e-8,
                 maxit: int = 1000):
    """CG with the Polak-Ribiere beta (flexible CG), for a preconditioner that is not exactly linear.

    Returns (x, iterations, relative true residual)."""
    f = free.astype(float)
    Am = sp.diags(f) @ A @ sp.diags(f)
    x = np.zeros_like(b)
    r = b * f
    bn = np.linalg.norm(r)
    if bn == 0.0:
        return x, 0, 0.0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * bn and it < maxit:
        w = Am @ p
        alpha = rz / (p @ w)
        x += alpha * p
        r_prev = r.copy()
        r = r - alpha * w
        z = precond(r)
        beta = ((r - r_prev) @ z) / rz
        rz = r @ z
        p = z + beta * p
        it += 1
    return x, it, np.linalg.norm((b - A @ x) * f) / bn
