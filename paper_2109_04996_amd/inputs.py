"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module holds no arithmetic of the finite-element method: no quadrature,
no basis, no geometric factors. It only builds index arrays of a structured
brick lattice, moves lattice vertices by the warps that define the synthetic
meshes, and draws seeded random numbers. Both sides of every parity check take
their inputs from here and compute everything else on their own.

Mesh recipe (Benchmarks section: the bake-off problems use Q_p bricks mapped
from the reference cube; here the bricks tile the unit cube):

* ``N**3`` trilinear bricks on ``[0,1]^3``; vertex lattice ``(N+1)**3``.
* warp ``"A"``: every vertex coordinate ``x_j`` is moved to
  ``x_j + 0.05 sin(2 pi x_j)``, axis by axis. Elements stay axis-aligned boxes
  of unequal sizes; the boundary is fixed, so the volume stays 1.
* warp ``"B"``: ``x_i <- x_i + 0.05 sin(2 pi x_{i+1}) sin(pi x_i)`` (cyclic in
  i), applied to vertices. Elements become non-affine trilinear bricks; the
  boundary planes are fixed, so the volume stays 1.
* warp ``None``: the uniform lattice.
* Elements are listed in a seeded random order (``default_rng(seed)
  .permutation(E)``). L-node ids are lexicographic on the ``(N p + 1)**3``
  node lattice, x fastest, independent of the element order.
* Element-local node order is lexicographic, i (x) fastest, so local node
  ``(i, j, k)`` of element ``(ex, ey, ez)`` is lattice node
  ``(ex p + i, ey p + j, ez p + k)``. Local vertex ``a + 2 b + 4 c`` is the
  corner ``(a, b, c)`` of the brick.
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = [
    "lattice_mesh",
    "rotate_elements",
    "renumber_rows",
    "uniform_vector",
    "kappa_field_params",
    "lattice_node_ijk",
]


def _warp(v: np.ndarray, warp):
    x = v.copy()
    if warp is None:
        return x
    if warp == "A":
        return x + 0.05 * np.sin(2.0 * np.pi * x)
    if warp == "B":
        out = x.copy()
        for i in range(3):
            out[:, i] = x[:, i] + 0.05 * np.sin(2.0 * np.pi * x[:, (i + 1) % 3]) * np.sin(np.pi * x[:, i])
        return out
    raise ValueError(f"unknown warp {warp!r}")


def lattice_mesh(N: int, p: int, warp="A", shuffle_seed=0) -> dict:
    """Brick lattice of the unit cube with its Q_p node numbering.

    Returns a dict with
      ``verts``       (nv, 3) float64 vertex coordinates (after the warp),
      ``elem_verts``  (E, 8) int64 vertex ids per element (corner a+2b+4c),
      ``elem_nodes``  (E, (p+1)**3) int32 L-node ids (local i fastest),
      ``boundary``    (n,) uint8, 1 on nodes of the cube's boundary,
      ``elem_ijk``    (E, 3) int64 lattice position of each element,
      ``N``, ``p``, ``nnodes``, ``nelem``.
    """
    if N < 1 or p < 1:
        raise ValueError("N and p must be >= 1")
    P = p + 1
    nv1 = N + 1
    g = np.arange(nv1) / N
    vz, vy, vx = np.meshgrid(g, g, g, indexing="ij")
    verts = np.stack([vx.ravel(), vy.ravel(), vz.ravel()], axis=1)
    verts = _warp(verts, warp)

    ez, ey, ex = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    eijk = np.stack([ex.ravel(), ey.ravel(), ez.ravel()], axis=1).astype(np.int64)
    if shuffle_seed is not None:
        perm = np.random.default_rng(shuffle_seed).permutation(eijk.shape[0])
        eijk = eijk[perm]

    c = np.arange(8)
    ca, cb, cc = c & 1, (c >> 1) & 1, (c >> 2) & 1
    elem_verts = ((eijk[:, 0:1] + ca) + nv1 * ((eijk[:, 1:2] + cb) + nv1 * (eijk[:, 2:3] + cc))).astype(np.int64)

    M = N * p + 1
    loc = np.arange(P ** 3)
    li, lj, lk = loc % P, (loc // P) % P, loc // (P * P)
    gi = eijk[:, 0:1] * p + li
    gj = eijk[:, 1:2] * p + lj
    gk = eijk[:, 2:3] * p + lk
    elem_nodes = (gi + M * (gj + M * gk)).astype(np.int32)

    n = M ** 3
    nid = np.arange(n)
    ni, nj, nk = nid % M, (nid // M) % M, nid // (M * M)
    boundary = ((ni == 0) | (ni == M - 1) | (nj == 0) | (nj == M - 1) | (nk == 0) | (nk == M - 1)).astype(np.uint8)
    return dict(verts=verts, elem_verts=elem_verts, elem_nodes=elem_nodes, boundary=boundary,
                elem_ijk=eijk, N=N, p=p, nnodes=n, nelem=eijk.shape[0])


def _rotations():
    """The 24 proper rotations of the reference cube as (axis permutation, flips)."""
    out = []
    for perm in itertools.permutations(range(3)):
        inv = sum(1 for i in range(3) for j in range(i + 1, 3) if perm[i] > perm[j])
        for flips in itertools.product((0, 1), repeat=3):
            if (-1) ** inv * (-1) ** sum(flips) == 1:
                out.append((perm, flips))
    return out


def rotate_elements(mesh: dict, p: int, frac: float, seed: int) -> dict:
    """Renumber the local nodes and corners of a seeded random subset (fraction ``frac``) of the
    elements by a proper rotation of the reference cube: the same hexahedra and the same assembled
    operator, with other local orientations (so chains of face-adjacent elements break and no
    element-wise affine numbering exists)."""
    P = p + 1
    rng = np.random.default_rng(seed)
    E = mesh["nelem"]
    en = mesh["elem_nodes"].reshape(E, P, P, P).copy()  # [e][k][j][i]
    ev = mesh["elem_verts"].reshape(E, 2, 2, 2).copy()  # [e][c][b][a]
    rots = [r for r in _rotations() if r != ((0, 1, 2), (0, 0, 0))]
    for e in np.flatnonzero(rng.random(E) < frac):
        perm, flips = rots[rng.integers(len(rots))]
        for arr in (en, ev):
            a = np.transpose(arr[e].transpose(2, 1, 0), perm)  # axes (r1, r2, r3), permuted
            for d in range(3):
                if flips[d]:
                    a = np.flip(a, axis=d)
            arr[e] = a.transpose(2, 1, 0)
    out = dict(mesh)
    out["elem_nodes"] = np.ascontiguousarray(en.reshape(E, P ** 3))
    out["elem_verts"] = np.ascontiguousarray(ev.reshape(E, 8))
    return out


def renumber_rows(mesh: dict, seed: int) -> dict:
    """Relabel the L-nodes of a lattice mesh by a seeded permutation of whole x-rows of the node
    lattice: node ``i + M r`` (row ``r = j + M k``) becomes ``i + M perm[r]``. Every element's rows
    along its first local axis keep consecutive ids, but no element-wise affine numbering is left.
    ``boundary`` moves with the nodes; ``verts`` and ``elem_verts`` are unchanged."""
    M = mesh["N"] * mesh["p"] + 1
    perm = np.random.default_rng(seed).permutation(M * M)
    old = np.arange(M ** 3)
    new = perm[old // M] * M + old % M
    out = dict(mesh)
    out["elem_nodes"] = new[mesh["elem_nodes"]].astype(np.int32)
    bnd = np.empty_like(mesh["boundary"])
    bnd[new] = mesh["boundary"]
    out["boundary"] = bnd
    return out


def lattice_node_ijk(N: int, p: int) -> np.ndarray:
    """(n, 3) integer lattice position of every L-node (index arithmetic only)."""
    M = N * p + 1
    nid = np.arange(M ** 3)
    return np.stack([nid % M, (nid // M) % M, nid // (M * M)], axis=1)


def uniform_vector(n: int, seed: int, ncomp: int = 1) -> np.ndarray:
    """Seeded U[-1, 1] float64 vector of length n*ncomp (components interleaved)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n * ncomp)


def kappa_field_params(seed: int, M: int = 512, ell: float = 0.1, contrast: float = 100.0,
                       grid: int = 48) -> dict:
    """Random-Fourier-feature parameters of a smooth Gaussian random field.

    The coefficient is ``kappa(x) = exp(s * g(x) + t)`` with
    ``g(x) = sqrt(2/M) * sum_m cos(omega_m . x + b_m)``, ``omega_m ~ N(0, ell^-2 I)``,
    ``b_m ~ U[0, 2 pi)`` (a squared-exponential covariance of correlation length
    ``ell``). ``s`` and ``t`` map the range of ``g`` over a ``grid**3`` sample
    lattice of the unit cube onto ``[-ln sqrt(contrast), +ln sqrt(contrast)]``,
    so kappa spans about ``contrast`` (0.1 .. 10 for 1e2).
    """
    rng = np.random.default_rng(seed)
    omega = rng.normal(0.0, 1.0 / ell, size=(M, 3))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=M)
    g1 = (np.arange(grid) + 0.5) / grid
    Z, Y, X = np.meshgrid(g1, g1, g1, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    gmin, gmax = np.inf, -np.inf
    for s0 in range(0, pts.shape[0], 8192):
        arg = pts[s0:s0 + 8192] @ omega.T + phase
        gv = np.sqrt(2.0 / M) * np.cos(arg).sum(axis=1)
        gmin, gmax = min(gmin, gv.min()), max(gmax, gv.max())
    half = 0.5 * np.log(contrast)
    s = 2.0 * half / (gmax - gmin)
    t = -half - s * gmin
    return dict(omega=omega, phase=phase, scale=float(s), shift=float(t), M=M)
