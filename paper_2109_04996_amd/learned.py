"""Training data, training and evaluation of the learned element preconditioner.

The network learns an element-local approximate inverse. Its training pairs come from exact FP64
solves of element-patch problems on seeded variable-coefficient fields: for a group of elements
whose node sets are not coupled by A (no element touches two of them), the library's PCG solves
A e = r to 1e-12 with every node outside the group's elements held at zero. The system is then
block diagonal with one block A_ee (the rows and columns of the assembled A at element e's
nodes) per group element, so each element's error is exactly e_e = A_ee^-1 r_e. The residuals r
are Jacobi-PCG iterates r_k = b - A x_k of the field's own problem (k in ``snapshots``; each x_k
is the library's PCG run with maxit = k from zero) plus seeded uniform noise. Targets are e_e
(network-only form, mode 0) or e_e - D^-1 r_e (the part a Jacobi step misses, modes 1 and 2);
the library scales them into the network's Jacobi-scaled variables.

Residual/error pairs of the global problem (e = x* - x_k) are not used: their error is dominated
by smooth global modes that no element-local map can predict from r_e.

The library turns vectors into element rows (``hx_op_mlp_features`` / ``hx_op_mlp_targets``); the
network is trained on the GPU by ``hx_mlp_train`` (FP32, Adam).
"""
from __future__ import annotations

import numpy as np

from . import hexpa as hx
from .inputs import kappa_field_params
from .problem import Problem


def rhs_ones(pr: Problem, mass: Problem):
    """b = B 1 (the right-hand side f = 1), masked to the free nodes."""
    torch = pr.torch
    one = torch.ones(pr.n, dtype=torch.float64, device="cuda")
    b = mass.apply(one)
    b *= pr.to_dev((pr.mesh["boundary"] == 0).astype(np.float64))
    return b


def problem_with_kappa(N, p, q, rule, seed, warp="A", shuffle_seed=0, kappa_M=512):
    kp = kappa_field_params(seed, M=kappa_M)
    pr = Problem(N, p, q, rule, "diffusion", warp=warp, shuffle_seed=shuffle_seed, kappa=kp)
    mass = Problem(N, p, max(q, p + 2) if rule == "gauss" else p + 2, "gauss", "mass", mesh=pr.mesh)
    b = rhs_ones(pr, mass)
    mass.close()
    return pr, b


def patch_groups(mesh: dict) -> list[np.ndarray]:
    """Element groups (caller element ids) whose node sets are pairwise uncoupled by A.

    Two elements conflict when some element shares a node with each of them (their nodes are then
    coupled by that element's matrix). Greedy coloring of that distance-2 graph, elements taken
    in caller order; on a lattice this gives about 27 groups.
    """
    import scipy.sparse as sp
    EN = mesh["elem_nodes"]
    E, P3 = EN.shape
    inc = sp.csr_matrix((np.ones(E * P3, dtype=np.int8), EN.ravel(), np.arange(0, E * P3 + 1, P3)),
                        shape=(E, mesh["nnodes"]))
    adj = (inc @ inc.T).astype(bool).astype(np.int32)
    conf = (adj @ adj).tocsr()
    color = -np.ones(E, dtype=np.int64)
    for e in range(E):
        nb = color[conf.indices[conf.indptr[e]:conf.indptr[e + 1]]]
        used = set(nb[nb >= 0].tolist())
        c = 0
        while c in used:
            c += 1
        color[e] = c
    return [np.flatnonzero(color == c) for c in range(color.max() + 1)]


def training_set(p, q, rule, N, seeds, snapshots=(1, 3, 10, 30), noise=1, groups_per_field=6, kappa_M=512,
                 sample_seed=11, mode=1):
    """(X, T) device FP32 tensors of element inputs and targets (see the module docstring).

    Per coefficient seed: ``groups_per_field`` seeded element groups, each solved exactly for every
    residual (``len(snapshots)`` Jacobi-PCG iterates plus ``noise`` uniform random vectors). Every
    pair is returned twice, the second time with the residual part of the input and the target
    negated."""
    torch = __import__("torch")
    rng = np.random.default_rng(sample_seed)
    Xs, Ts = [], []
    P3 = (p + 1) ** 3
    for seed in seeds:
        pr, b = problem_with_kappa(N, p, q, rule, seed, kappa_M=kappa_M)
        with pr:
            mesh = pr.mesh
            E = mesh["nelem"]
            free = pr.to_dev((mesh["boundary"] == 0).astype(np.float64))
            dinv = free / pr.diagonal()
            res = []
            for k in snapshots:
                xk, _ = pr.solve(b, rtol=1e-30, maxit=k, check_every=k, raise_on_error=False)
                res.append((b - pr.apply(xk)) * free)
            for _ in range(noise):
                res.append(pr.to_dev(rng.uniform(-1.0, 1.0, pr.n)) * free)
            groups = patch_groups(mesh)
            pick = rng.choice(len(groups), size=min(groups_per_field, len(groups)), replace=False)
            X = torch.empty(E, 2 * P3, dtype=torch.float32, device="cuda")
            rn = torch.empty(E, dtype=torch.float32, device="cuda")
            T = torch.empty(E, P3, dtype=torch.float32, device="cuda")
            for g in pick:
                elems = groups[g]
                bnd = mesh["boundary"].copy()
                inside = np.zeros(mesh["nnodes"], dtype=bool)
                inside[mesh["elem_nodes"][elems].ravel()] = True
                bnd[~inside] = 1
                kp = kappa_field_params(seed, M=kappa_M)
                with Problem(N, p, q, rule, "diffusion", mesh=dict(mesh, boundary=bnd), kappa=kp) as patch:
                    sel = torch.from_numpy(elems).to("cuda")
                    for r in res:
                        e, info = patch.solve(r, rtol=1e-12, maxit=20000)
                        if mode != 0:
                            e = e - dinv * r
                        hx.hx_op_mlp_features(patch.h_op, r, X, rn)
                        hx.hx_op_mlp_targets(patch.h_op, e, rn, T)
                        keep = sel[rn[sel] > 0]
                        Xs.append(X[keep].clone())
                        Ts.append(T[keep].clone())
    X, T = torch.cat(Xs), torch.cat(Ts)
    # the target map is linear in r: each pair also holds with the residual's sign flipped
    Xn = X.clone()
    Xn[:, :P3] = -Xn[:, :P3]
    return torch.cat([X, Xn]), torch.cat([T, -T])


def train(X, T, n_hidden=128, seed=7, **opts):
    net = hx.hx_mlp_create(X.shape[1], n_hidden, T.shape[1], seed)
    o = hx.hx_train_opts_default(**opts)
    info = hx.hx_mlp_train(net, X, T, o)
    return net, info


FORMS = {
    "jacobi": dict(),
    "chebyshev4": dict(precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP64),
    "chebyshev4_fp32": dict(precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP32),
    "learned": dict(precond=hx.HX_PC_MLP, fallback=hx.HX_PC_JACOBI, mlp_mode=1),
    "learned_cheb4": dict(precond=hx.HX_PC_MLP, fallback=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP64, mlp_mode=2),
}


def compare_solves(pr: Problem, b, net, rtol=1e-8, maxit=20000, forms=None, learned_opts=None):
    """Iterations, operator applies and time to rtol for each form (default: all of FORMS). The
    learned forms run flexible CG with the network (``learned_opts`` added to their options) and
    fall back to Jacobi / Chebyshev PCG."""
    out = {}
    for name in forms or FORMS:
        o = dict(FORMS[name])
        if o.get("precond") == hx.HX_PC_MLP:
            o["mlp"] = net.value
            o.update(learned_opts or {})
        pr.torch.cuda.synchronize()
        x, info = pr.solve(b, rtol=rtol, maxit=maxit, check_every=10, raise_on_error=False, **o)
        out[name] = dict(status=info["status"], iterations=info["iterations"], applies=info["operator_applies"],
                         seconds=round(info["solve_seconds"], 4), setup_seconds=round(info["setup_seconds"], 4),
                         true_rel_residual=info["true_rel_residual"], fallback_used=info["fallback_used"],
                         fallback_iterations=info["fallback_iterations"], fallback_reason=info["fallback_reason"])
    return out
