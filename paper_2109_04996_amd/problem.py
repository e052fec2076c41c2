"""Build library handles for a synthetic lattice problem (mesh, basis, operator) on the current GPU.

Everything numeric happens in libhexpa: node coordinates (``hx_mesh_nodes_trilinear``),
coloring and restriction (``hx_mesh_create``), geometric factors (``hx_op_create``).
This module only moves the seeded inputs of ``inputs`` into those calls.
"""
from __future__ import annotations

import numpy as np

from . import hexpa as hx
from . import inputs

RULES = {"gauss": hx.HX_GAUSS, "gll": hx.HX_GLL}
KINDS = {"mass": hx.HX_MASS, "diffusion": hx.HX_DIFFUSION, "helmholtz": hx.HX_HELMHOLTZ, "lor": hx.HX_LOR}


class Problem:
    """One operator on a lattice mesh: ``Problem(N, p, q, rule, kind, ncomp, warp, shuffle_seed, kappa)``;
    kind ``"helmholtz"`` is ``alpha A + beta B`` (``helmholtz=(alpha, beta)``)."""

    def __init__(self, N: int, p: int, q: int, rule: str, kind: str, ncomp: int = 1, warp="A",
                 shuffle_seed=0, kappa: dict | None = None, dirichlet: bool = True, mesh: dict | None = None,
                 helmholtz=(1.0, 1.0)):
        import torch
        self.torch = torch
        self.N, self.p, self.q, self.rule, self.kind, self.ncomp = N, p, q, rule, kind, ncomp
        self.mesh = mesh if mesh is not None else inputs.lattice_mesh(N, p, warp=warp, shuffle_seed=shuffle_seed)
        m = self.mesh
        self.xyz = hx.hx_mesh_nodes_trilinear(p, m["elem_verts"], m["verts"], m["elem_nodes"], m["nnodes"])
        self.h_mesh = hx.hx_mesh_create(p, m["elem_nodes"], self.xyz, m["boundary"] if dirichlet else None)
        self.h_basis = hx.hx_basis_create(p, q, RULES[rule])
        if kind == "helmholtz":
            self.h_op = hx.hx_op_create_helmholtz(self.h_mesh, self.h_basis, ncomp, helmholtz[0], helmholtz[1], kappa)
        elif kind == "lor":
            # the low-order refined matrix of the mesh (q and rule are not used)
            self.h_op = hx.hx_op_create_lor(self.h_mesh, kappa)
        else:
            self.h_op = hx.hx_op_create(self.h_mesh, self.h_basis, KINDS[kind], ncomp, kappa)
        self.n = m["nnodes"] * ncomp
        self.stats = hx.hx_mesh_get_stats(self.h_mesh)

    # ---- device vectors
    def zeros(self, dtype=None):
        return self.torch.zeros(self.n, dtype=dtype or self.torch.float64, device="cuda")

    def to_dev(self, a: np.ndarray, dtype=None):
        return self.torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype or self.torch.float64)

    def apply(self, x, y=None):
        y = self.zeros(x.dtype) if y is None else y
        hx.hx_op_apply(self.h_op, x, y)
        return y

    def apply_f32(self, x, qdata_prec=hx.HX_FP64, y=None):
        y = self.zeros(self.torch.float32) if y is None else y
        hx.hx_op_apply_f32(self.h_op, qdata_prec, x, y)
        return y

    def apply_bf16(self, x, y=None, prec=hx.HX_BF16):
        y = self.zeros(self.torch.float32) if y is None else y
        hx.hx_op_apply_bf16(self.h_op, x, y, prec=prec)
        return y

    def apply_elem(self, x):
        P3 = (self.p + 1) ** 3
        ye = self.torch.empty(self.mesh["nelem"] * self.ncomp * P3, dtype=self.torch.float64, device="cuda")
        hx.hx_op_apply_elem(self.h_op, x, ye)
        return ye.view(self.mesh["nelem"], self.ncomp, P3)

    def diagonal(self):
        d = self.zeros()
        hx.hx_op_diagonal(self.h_op, d)
        return d

    def solve(self, b, x=None, raise_on_error=True, **opts):
        x = self.zeros() if x is None else x
        if "mlp" in opts and hasattr(opts["mlp"], "value"):
            opts["mlp"] = opts["mlp"].value  # a network handle
        o = hx.hx_solve_opts_default(**opts)
        info = hx.hx_pcg_solve(self.h_op, b, x, o, raise_on_error=raise_on_error)
        return x, info

    def close(self):
        if getattr(self, "h_op", None):
            hx.hx_op_destroy(self.h_op)
            self.h_op = None
        if getattr(self, "h_basis", None):
            hx.hx_basis_destroy(self.h_basis)
            self.h_basis = None
        if getattr(self, "h_mesh", None):
            hx.hx_mesh_destroy(self.h_mesh)
            self.h_mesh = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hierarchy:
    """p-multigrid over polynomial degrees on one lattice mesh.

    ``Hierarchy(N, degrees, rule, kind, warp, shuffle_seed, kappa, meshes, ncomp, helmholtz, lor, **pmg_opts)``:
    level l is a ``Problem`` of degree ``degrees[l]`` (strictly decreasing) with
    q = p + 1 GLL points or q = p + 2 Gauss points, on the same elements (same
    shuffle); ``meshes`` overrides the lattice meshes level by level. ``lor``: level 0
    is the low-order refined operator of degree ``degrees[0]`` (a preconditioner for
    the high-order operator of the same nodes), the others diffusion.
    """

    def __init__(self, N: int, degrees, rule: str = "gll", kind: str = "diffusion", warp="A", shuffle_seed=0,
                 kappa: dict | None = None, meshes=None, ncomp: int = 1, helmholtz=(1.0, 1.0), lor=False,
                 **pmg_opts):
        self.levels = []
        for l, p in enumerate(degrees):
            q = p + 1 if rule == "gll" else p + 2
            self.levels.append(Problem(N, p, q, rule, "lor" if (lor and l == 0) else kind, ncomp=ncomp, warp=warp,
                                       shuffle_seed=shuffle_seed,
                                       kappa=kappa, mesh=None if meshes is None else meshes[l], helmholtz=helmholtz))
        self.h = hx.hx_pmg_create([pr.h_op for pr in self.levels], hx.hx_pmg_opts_default(**pmg_opts))

    @property
    def fine(self) -> Problem:
        return self.levels[0]

    def lambda_max(self, level: int) -> float:
        return hx.hx_pmg_lambda_max(self.h, level)

    def vcycle(self, r, z=None):
        z = self.fine.zeros() if z is None else z
        hx.hx_pmg_vcycle(self.h, r, z)
        return z

    def prolong(self, level: int, x_coarse):
        y = self.levels[level].zeros()
        hx.hx_pmg_prolong(self.h, level, x_coarse, y)
        return y

    def restrict(self, level: int, r_fine):
        y = self.levels[level + 1].zeros()
        hx.hx_pmg_restrict(self.h, level, r_fine, y)
        return y

    def solve(self, b, x=None, raise_on_error=True, **opts):
        return self.fine.solve(b, x, raise_on_error=raise_on_error, precond=hx.HX_PC_PMG, pmg=self.h.value, **opts)

    def close(self):
        if getattr(self, "h", None):
            hx.hx_pmg_destroy(self.h)
            self.h = None
        for pr in getattr(self, "levels", []):
            pr.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
