"""Krylov solves and preconditioners on the assembled matrix, FP64 (oracle; test infrastructure only).

Benchmarks section: the bake-off problems are CG solves of (alpha A + beta B) u
= B f with homogeneous Dirichlet conditions u = 0 on the boundary; the
constrained nodes are removed, i.e. the system solved is the free-free block
A_II u_I = b_I. Miniapps section (Nekbone): CG with a diagonal (Jacobi)
preconditioner. The stopping rule used throughout is ||b - A x||_2 <= tol
||b||_2 over the free nodes, from x0 = 0.

The Chebyshev preconditioner is not in the paper: it is the textbook
Chebyshev acceleration of the Jacobi-preconditioned operator D^-1 A on an
interval [lam_lo, lam_hi], run for ``degree`` steps from z = 0, so that the
residual polynomial is the scaled Chebyshev polynomial
T_k(theta(lam)) / T_k(theta(0)), theta(lam) = (lam_hi + lam_lo - 2 lam)/(lam_hi - lam_lo).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def free_mask(boundary: np.ndarray, ncomp: int = 1) -> np.ndarray:
    m = boundary == 0
    return np.repeat(m, ncomp) if ncomp > 1 else m


def expand(A: sp.csr_matrix, ncomp: int) -> sp.csr_matrix:
    """Scalar matrix acting on each of ``ncomp`` interleaved components."""
    return A if ncomp == 1 else sp.kron(A, sp.identity(ncomp), format="csr")


def direct_solve(A: sp.csr_matrix, b: np.ndarray, free: np.ndarray) -> np.ndarray:
    """x with x_B = 0 and A_II x_I = b_I (sparse LU)."""
    x = np.zeros_like(b)
    Aii = A[free][:, free].tocsc()
    x[free] = spla.spsolve(Aii, b[free])
    return x


def jacobi_pcg(A: sp.csr_matrix, b: np.ndarray, free: np.ndarray, tol: float = 1e-8,
               maxit: int = 20000, x0=None):
    """Preconditioned CG (Hestenes-Stiefel form) with z = D^-1 r on the free nodes.

    Returns (x, iterations, relative true residual). Constrained entries of
    x, r, z, p stay zero.
    """
    f = free.astype(float)
    dinv = np.where(free, 1.0 / A.diagonal(), 0.0)
    x = np.zeros_like(b) if x0 is None else x0 * f
    r = (b - A @ x) * f
    bn = np.linalg.norm(b * f)
    if bn == 0.0:
        return x, 0, 0.0
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * bn and it < maxit:
        w = (A @ p) * f
        alpha = rz / (p @ w)
        x += alpha * p
        r -= alpha * w
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    true_res = np.linalg.norm((b - A @ x) * f) / bn
    return x, it, true_res


def chebyshev_apply(A: sp.csr_matrix, dinv: np.ndarray, r: np.ndarray, lam_lo: float,
                    lam_hi: float, degree: int = 4) -> np.ndarray:
    """z = s(D^-1 A) D^-1 r by the three-term Chebyshev recurrence, ``degree`` steps from z = 0.

    Uses degree-1 operator applies. ``dinv`` is zero on constrained nodes, so
    z stays zero there. ``dinv`` may instead be a map v -> M v (a base other
    than the diagonal, such as the learned element map): the same recurrence
    then gives z = s(M A) M r.
    """
    M = dinv if callable(dinv) else (lambda v: dinv * v)
    theta = 0.5 * (lam_hi + lam_lo)
    delta = 0.5 * (lam_hi - lam_lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = M(r) / theta
    z = d.copy()
    for _ in range(degree - 1):
        res = r - A @ z
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * M(res)
        z = z + d
        rho = rho_new
    return z


def chebyshev_pcg(A: sp.csr_matrix, b: np.ndarray, free: np.ndarray, lam_lo: float, lam_hi: float,
                  degree: int = 4, tol: float = 1e-8, maxit: int = 20000):
    """CG preconditioned by ``chebyshev_apply`` on the masked operator. Returns (x, iterations, rel. residual)."""
    f = free.astype(float)
    Am = sp.diags(f) @ A @ sp.diags(f)
    dinv = np.where(free, 1.0 / A.diagonal(), 0.0)
    x = np.zeros_like(b)
    r = b * f
    bn = np.linalg.norm(r)
    z = chebyshev_apply(Am, dinv, r, lam_lo, lam_hi, degree)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * bn and it < maxit:
        w = Am @ p
        alpha = rz / (p @ w)
        x += alpha * p
        r -= alpha * w
        z = chebyshev_apply(Am, dinv, r, lam_lo, lam_hi, degree)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, np.linalg.norm((b - A @ x) * f) / bn


def jacobi_lambda_max(A: sp.csr_matrix, free: np.ndarray) -> float:
    """Largest eigenvalue of D^-1 A_II (Lanczos on the symmetric form D^-1/2 A D^-1/2)."""
    Aii = A[free][:, free]
    s = 1.0 / np.sqrt(Aii.diagonal())
    S = sp.diags(s) @ Aii @ sp.diags(s)
    if S.shape[0] <= 64:
        return float(np.linalg.eigvalsh(S.toarray())[-1])
    return float(spla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0])
