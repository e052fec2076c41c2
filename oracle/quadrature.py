"""1D quadrature rules and Lagrange tables, FP64 (oracle; test infrastructure only).

Benchmarks section: the bake-off discretizations use C0 Lagrange bases of
degree p on a tensor-product reference cube [-1,1]^3; BP1-BP4 integrate with
q = p+2 Gauss-Legendre points per direction, BP5-BP6 on the (p+1) Gauss-Lobatto-
Legendre nodes. The rules are the textbook ones (Gauss: roots of P_q,
weights 2/((1-x^2) P_q'(x)^2); GLL: +-1 and the roots of P_p', weights
2/(p(p+1) P_p(x)^2)). Legendre polynomials are evaluated by numpy's Legendre
series routines, roots are found from the Legendre companion matrix and
polished by Newton steps.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def _legendre_coeffs(n: int) -> np.ndarray:
    c = np.zeros(n + 1)
    c[n] = 1.0
    return c


def _polish(coef: np.ndarray, x: np.ndarray, steps: int = 4) -> np.ndarray:
    dcoef = L.legder(coef)
    for _ in range(steps):
        x = x - L.legval(x, coef) / L.legval(x, dcoef)
    return x


def gauss_rule(q: int):
    """Gauss-Legendre nodes and weights on [-1, 1] with q points (exact to degree 2q-1)."""
    if q < 1:
        raise ValueError("q >= 1")
    c = _legendre_coeffs(q)
    x = np.sort(np.real(L.legroots(c)))
    x = _polish(c, x)
    dP = L.legval(x, L.legder(c))
    w = 2.0 / ((1.0 - x * x) * dP * dP)
    return x, w


def gll_rule(p: int):
    """Gauss-Lobatto-Legendre nodes and weights, p+1 points (exact to degree 2p-1)."""
    if p < 1:
        raise ValueError("p >= 1")
    c = _legendre_coeffs(p)
    if p == 1:
        x = np.array([-1.0, 1.0])
    else:
        dc = L.legder(c)
        xi = np.sort(np.real(L.legroots(dc)))
        xi = _polish(dc, xi)
        x = np.concatenate([[-1.0], xi, [1.0]])
    Pp = L.legval(x, c)
    w = 2.0 / (p * (p + 1) * Pp * Pp)
    return x, w


def lagrange_table(nodes: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """phi[a, i] = l_i(pts[a]), the Lagrange polynomial through ``nodes`` (product formula)."""
    nodes = np.asarray(nodes, float)
    pts = np.asarray(pts, float)
    P = nodes.size
    out = np.ones((pts.size, P))
    for i in range(P):
        for m in range(P):
            if m != i:
                out[:, i] *= (pts - nodes[m]) / (nodes[i] - nodes[m])
    return out


def lagrange_deriv_table(nodes: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """dphi[a, i] = l_i'(pts[a]) by the product rule applied to the product formula."""
    nodes = np.asarray(nodes, float)
    pts = np.asarray(pts, float)
    P = nodes.size
    out = np.zeros((pts.size, P))
    for i in range(P):
        for l in range(P):
            if l == i:
                continue
            term = np.full(pts.size, 1.0 / (nodes[i] - nodes[l]))
            for m in range(P):
                if m != i and m != l:
                    term *= (pts - nodes[m]) / (nodes[i] - nodes[m])
            out[:, i] += term
    return out


def rule_points(p: int, q: int, rule: str):
    """Quadrature points/weights of an operator: rule 'gauss' (q points) or 'gll' (q points = GLL of degree q-1)."""
    if rule == "gauss":
        return gauss_rule(q)
    if rule == "gll":
        return gll_rule(q - 1)
    raise ValueError(rule)
