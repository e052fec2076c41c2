"""Dense element matrices and the assembled global operator, FP64 (oracle; test infrastructure only).

Benchmarks section: isoparametric Q_p bricks, each mapped from the reference
cube [-1,1]^3 by x^e(r); stiffness A_ij = int grad phi_i . grad phi_j dV and
mass B_ij = int phi_i phi_j dV, integrated with the element's quadrature rule.
Here every brick is trilinear, so its map is the Q_1 interpolant of its eight
vertices; a Q_1 map is exactly representable in Q_p, so this is the same map
as the isoparametric one built on the Q_p nodes.

libCEED section (operator decomposition): the matrix-free action equals
P^T G^T B^T D B G P applied to a vector; its exact value is the assembled
sparse matrix built here from the element matrices (element restriction G =
the index array ``elem_nodes``, summed by the sparse-matrix constructor).
For m = 3 components the operator is the same scalar operator on each
component, with components interleaved in the L-vector (index 3*node + c).

Diffusion with a coefficient: A_ij = int kappa grad phi_i . grad phi_j dV;
kappa is the random-Fourier-feature field of the input recipe, evaluated at
the physical quadrature points.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .quadrature import gll_rule, lagrange_deriv_table, lagrange_table, rule_points

CORNERS = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=float)  # index a+2b+4c


def reference_tables(p: int, q: int, rule: str):
    """Nodes (GLL of degree p), 1D points and weights, phi[a,i], dphi[a,i]."""
    xn, _ = gll_rule(p)
    xq, wq = rule_points(p, q, rule)
    return xn, xq, wq, lagrange_table(xn, xq), lagrange_deriv_table(xn, xq)


def tensor_tables(phi: np.ndarray, dphi: np.ndarray, wq: np.ndarray):
    """3D tables: point index a + q(b + q c), node index i + P(j + P k).

    Phi[pt, node] = l_i(r1) l_j(r2) l_k(r3); dPhi[d] is its derivative along r_{d+1};
    w3[pt] = w_a w_b w_c.
    """
    q, P = phi.shape

    def outer(tz, ty, tx):
        return np.einsum("ck,bj,ai->cbakji", tz, ty, tx).reshape(q ** 3, P ** 3)

    Phi = outer(phi, phi, phi)
    dPhi = np.stack([outer(phi, phi, dphi), outer(phi, dphi, phi), outer(dphi, phi, phi)])
    w3 = np.einsum("c,b,a->cba", wq, wq, wq).ravel()
    return Phi, dPhi, w3


def reference_points3(xq: np.ndarray) -> np.ndarray:
    """(q^3, 3) reference coordinates (r1, r2, r3) in the point order of ``tensor_tables``."""
    c, b, a = np.meshgrid(xq, xq, xq, indexing="ij")
    return np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)


def trilinear_map(V8: np.ndarray, r: np.ndarray):
    """Physical points x(r) and Jacobians J[pt, a, d] = dx_a/dr_d of the trilinear brick.

    V8 (8, 3): vertex coordinates, corner index a + 2b + 4c at reference (2a-1, 2b-1, 2c-1).
    r (npt, 3): reference coordinates in [-1, 1]^3.
    """
    s = 2.0 * CORNERS - 1.0  # (8, 3) signs
    f = 0.5 * (1.0 + r[:, None, :] * s[None, :, :])  # (npt, 8, 3) 1D factors
    N = f[:, :, 0] * f[:, :, 1] * f[:, :, 2]  # (npt, 8)
    dN = np.empty(f.shape)
    dN[:, :, 0] = 0.5 * s[None, :, 0] * f[:, :, 1] * f[:, :, 2]
    dN[:, :, 1] = 0.5 * s[None, :, 1] * f[:, :, 0] * f[:, :, 2]
    dN[:, :, 2] = 0.5 * s[None, :, 2] * f[:, :, 0] * f[:, :, 1]
    x = N @ V8
    J = np.einsum("nca,ncd->nad", np.broadcast_to(V8, (r.shape[0], 8, 3)), dN)
    return x, J


def det_and_inverse(J: np.ndarray):
    """detJ and J^{-1} of (npt, 3, 3) matrices by the adjugate formula."""
    a = J
    cof = np.empty_like(a)
    cof[:, 0, 0] = a[:, 1, 1] * a[:, 2, 2] - a[:, 1, 2] * a[:, 2, 1]
    cof[:, 0, 1] = -(a[:, 1, 0] * a[:, 2, 2] - a[:, 1, 2] * a[:, 2, 0])
    cof[:, 0, 2] = a[:, 1, 0] * a[:, 2, 1] - a[:, 1, 1] * a[:, 2, 0]
    cof[:, 1, 0] = -(a[:, 0, 1] * a[:, 2, 2] - a[:, 0, 2] * a[:, 2, 1])
    cof[:, 1, 1] = a[:, 0, 0] * a[:, 2, 2] - a[:, 0, 2] * a[:, 2, 0]
    cof[:, 1, 2] = -(a[:, 0, 0] * a[:, 2, 1] - a[:, 0, 1] * a[:, 2, 0])
    cof[:, 2, 0] = a[:, 0, 1] * a[:, 1, 2] - a[:, 0, 2] * a[:, 1, 1]
    cof[:, 2, 1] = -(a[:, 0, 0] * a[:, 1, 2] - a[:, 0, 2] * a[:, 1, 0])
    cof[:, 2, 2] = a[:, 0, 0] * a[:, 1, 1] - a[:, 0, 1] * a[:, 1, 0]
    det = a[:, 0, 0] * cof[:, 0, 0] + a[:, 0, 1] * cof[:, 0, 1] + a[:, 0, 2] * cof[:, 0, 2]
    inv = np.transpose(cof, (0, 2, 1)) / det[:, None, None]
    return det, inv


def kappa_eval(params: dict | None, x: np.ndarray) -> np.ndarray:
    """kappa(x) = exp(s g(x) + t), g(x) = sqrt(2/M) sum_m cos(omega_m . x + b_m); 1 if params is None."""
    if params is None:
        return np.ones(x.shape[0])
    om, ph = params["omega"], params["phase"]
    M = om.shape[0]
    g = np.sqrt(2.0 / M) * np.cos(x @ om.T + ph).sum(axis=1)
    return np.exp(params["scale"] * g + params["shift"])


class ElementRule:
    """Reference tables of one (p, q, rule) triple, shared by all elements of a mesh."""

    def __init__(self, p: int, q: int, rule: str):
        self.p, self.q, self.rule = p, q, rule
        self.xn, self.xq, self.wq, self.phi, self.dphi = reference_tables(p, q, rule)
        self.Phi, self.dPhi, self.w3 = tensor_tables(self.phi, self.dphi, self.wq)
        self.r3 = reference_points3(self.xq)


def element_matrix(V8: np.ndarray, er: ElementRule, kind: str, kappa=None) -> np.ndarray:
    """Dense element matrix by direct quadrature over all q^3 points.

    diffusion: A_e[i, j] = sum_pt w kappa detJ (J^-T grad_r phi_i) . (J^-T grad_r phi_j)
    mass:      B_e[i, j] = sum_pt w detJ phi_i phi_j
    """
    x, J = trilinear_map(V8, er.r3)
    det, inv = det_and_inverse(J)
    if np.any(det <= 0):
        raise ValueError("non-positive Jacobian determinant")
    if kind == "mass":
        wd = er.w3 * det
        return er.Phi.T @ (wd[:, None] * er.Phi)
    if kind == "diffusion":
        wd = er.w3 * det * kappa_eval(kappa, x)
        # physical gradient: (grad_x phi)_a = sum_d Jinv[d, a] d_r_d phi
        gx = np.einsum("nda,dni->ani", inv, er.dPhi)  # (3, npt, P^3)
        G = gx.reshape(3 * x.shape[0], -1)
        W = np.tile(wd, 3)
        return G.T @ (W[:, None] * G)
    raise ValueError(kind)


def element_matrices(mesh: dict, p: int, q: int, rule: str, kind: str, kappa=None, elems=None):
    """Element matrices of the listed elements (all if ``elems`` is None), shape (ne, P^3, P^3)."""
    er = ElementRule(p, q, rule)
    ids = np.arange(mesh["nelem"]) if elems is None else np.asarray(elems)
    V = mesh["verts"][mesh["elem_verts"][ids]]
    return np.stack([element_matrix(V[t], er, kind, kappa) for t in range(len(ids))])


def assemble(mesh: dict, p: int, q: int, rule: str, kind: str, kappa=None) -> sp.csr_matrix:
    """Global scalar matrix: sum over elements of G_e^T A_e G_e (duplicates summed by the CSR constructor)."""
    er = ElementRule(p, q, rule)
    en = mesh["elem_nodes"].astype(np.int64)
    E, P3 = en.shape
    n = mesh["nnodes"]
    V = mesh["verts"][mesh["elem_verts"]]
    A = sp.csr_matrix((n, n))
    chunk = max(1, int(2e7 // (P3 * P3)))
    for s0 in range(0, E, chunk):
        ids = range(s0, min(E, s0 + chunk))
        data = np.concatenate([element_matrix(V[e], er, kind, kappa).ravel() for e in ids])
        rows = np.concatenate([np.repeat(en[e], P3) for e in ids])
        cols = np.concatenate([np.tile(en[e], P3) for e in ids])
        A = A + sp.csr_matrix((data, (rows, cols)), shape=(n, n))
    A.sum_duplicates()
    return A


def assemble_helmholtz(mesh: dict, p: int, q: int, rule: str, alpha: float, beta: float,
                       kappa=None) -> sp.csr_matrix:
    """alpha A + beta B, both assembled with the same rule (Benchmarks section: the bake-off systems
    are (alpha A + beta B) u = B f)."""
    A = assemble(mesh, p, q, rule, "diffusion", kappa)
    B = assemble(mesh, p, q, rule, "mass")
    return (alpha * A + beta * B).tocsr()


def apply(A: sp.csr_matrix, x: np.ndarray, ncomp: int = 1) -> np.ndarray:
    """y = A x on an L-vector; for ncomp = 3 the scalar A acts on each interleaved component."""
    if ncomp == 1:
        return A @ x
    X = x.reshape(-1, ncomp)
    return (A @ X).reshape(-1)


def diagonal(A: sp.csr_matrix, ncomp: int = 1) -> np.ndarray:
    d = A.diagonal()
    return np.repeat(d, ncomp) if ncomp > 1 else d


def lor_mesh(mesh: dict, p: int) -> dict:
    """The low-order refined mesh of a degree-p mesh (Preconditioning section: a low-order discretization
    on a refined mesh, spectrally equivalent by the FEM-SEM equivalence): every element is split into p^3
    trilinear sub-hexahedra whose corners are its GLL nodes, sub-hex (i, j, k) taking element-local nodes
    (i + a, j + b, k + c), a, b, c in {0, 1}, as its vertex a + 2b + 4c. The nodes (and their coordinates,
    the vertices here) are those of the degree-p mesh; assembling it with p = 1 and the 2-point Gauss rule
    gives the low-order refined matrix."""
    P = p + 1
    E = mesh["nelem"]
    en = mesh["elem_nodes"].reshape(E, P, P, P)  # [e][k][j][i]
    subs = []
    for k in range(p):
        for j in range(p):
            for i in range(p):
                subs.append(np.stack([en[:, k + c, j + b, i + a] for c in (0, 1) for b in (0, 1) for a in (0, 1)],
                                     axis=1))
    ev = np.stack(subs, axis=1).reshape(E * p ** 3, 8)  # sub-hexes of element e are rows e p^3 .. (e+1) p^3 - 1
    return dict(verts=node_coordinates(mesh, p), elem_verts=ev.astype(np.int64), elem_nodes=ev.astype(np.int32),
                nnodes=mesh["nnodes"], nelem=E * p ** 3, boundary=mesh["boundary"])


def assemble_lor(mesh: dict, p: int, kappa=None) -> sp.csr_matrix:
    """The low-order refined diffusion matrix: Q1 on ``lor_mesh``, integrated with the 2-point GLL (vertex)
    rule per direction, kappa at the vertices. The vertex rule makes each sub-hex matrix the tensor form
    1D stiffness x lumped 1D mass that the FEM-SEM equivalence is stated for (the paper cites it without
    fixing a rule; with the 2-point Gauss rule the equivalence constants grow with p)."""
    return assemble(lor_mesh(mesh, p), 1, 2, "gll", "diffusion", kappa)


def node_coordinates(mesh: dict, p: int) -> np.ndarray:
    """Physical coordinates of every L-node (the trilinear map at the element's GLL nodes)."""
    xn, _ = gll_rule(p)
    r = reference_points3(xn)
    X = np.zeros((mesh["nnodes"], 3))
    V = mesh["verts"][mesh["elem_verts"]]
    for e in range(mesh["nelem"]):
        x, _ = trilinear_map(V[e], r)
        X[mesh["elem_nodes"][e]] = x
    return X


def element_apply(mesh: dict, p: int, q: int, rule: str, kind: str, x: np.ndarray, elems,
                  ncomp: int = 1, kappa=None) -> np.ndarray:
    """E-vector action A_e x_e (no scatter) of the listed elements, shape (ne, ncomp, P^3)."""
    Ae = element_matrices(mesh, p, q, rule, kind, kappa, elems)
    en = mesh["elem_nodes"][np.asarray(elems)].astype(np.int64)
    out = np.empty((len(en), ncomp, en.shape[1]))
    for c in range(ncomp):
        xe = x[ncomp * en + c]
        out[:, c, :] = np.einsum("eij,ej->ei", Ae, xe)
    return out
