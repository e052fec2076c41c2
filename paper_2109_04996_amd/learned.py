"""Training data, training and evaluation of the learned element preconditioner.

Residual/error pairs come from exact FP64 solves on seeded variable-coefficient problems: for
each training coefficient seed, the Jacobi-PCG iterates x_k (k in ``snapshots``, each obtained by
running the library's PCG with maxit = k from zero, which reproduces the iterate) give the
residual r_k = b - A x_k and the error e_k = x* - x_k against a tight solve x*. The library turns
them into element rows (``hx_op_mlp_features`` / ``hx_op_mlp_targets``); a seeded subset of the
elements of every snapshot forms the training set. The network is trained on the GPU by
``hx_mlp_train`` (FP32, Adam).
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


def training_set(p, q, rule, N, seeds, snapshots=(2, 5, 10, 20, 40, 80), rows_per_snapshot=400, sample_seed=11,
                 kappa_M=512, mode=0):
    """(X, T) device FP32 tensors: element inputs and targets from Jacobi-PCG iterates.

    mode 0: targets from the error e_k; mode 1: from e_k - D^-1 r_k, the part a Jacobi step misses
    (for the preconditioner form z = D^-1 r + correction)."""
    torch = __import__("torch")
    rng = np.random.default_rng(sample_seed)
    Xs, Ts = [], []
    P3 = (p + 1) ** 3
    for seed in seeds:
        pr, b = problem_with_kappa(N, p, q, rule, seed, kappa_M=kappa_M)
        with pr:
            E = pr.mesh["nelem"]
            xstar, _ = pr.solve(b, rtol=1e-12, maxit=100000)
            free = pr.to_dev((pr.mesh["boundary"] == 0).astype(np.float64))
            dinv = free / pr.diagonal() if mode == 1 else None
            X = torch.empty(E, 2 * P3, dtype=torch.float32, device="cuda")
            rn = torch.empty(E, dtype=torch.float32, device="cuda")
            T = torch.empty(E, P3, dtype=torch.float32, device="cuda")
            for k in snapshots:
                xk, info = pr.solve(b, rtol=1e-30, maxit=k, check_every=k, raise_on_error=False)
                r = (b - pr.apply(xk)) * free
                err = xstar - xk
                if mode == 1:
                    err = err - dinv * r
                hx.hx_op_mlp_features(pr.h_op, r, X, rn)
                hx.hx_op_mlp_targets(pr.h_op, err, rn, T)
                ok = torch.nonzero(rn > 0).flatten().cpu().numpy()
                pick = rng.choice(ok, size=min(rows_per_snapshot, ok.size), replace=False)
                idx = torch.from_numpy(pick).to("cuda")
                Xs.append(X[idx].clone())
                Ts.append(T[idx].clone())
    return torch.cat(Xs), torch.cat(Ts)


def train(X, T, n_hidden=128, seed=7, **opts):
    net = hx.hx_mlp_create(X.shape[1], n_hidden, T.shape[1], seed)
    o = hx.hx_train_opts_default(**opts)
    info = hx.hx_mlp_train(net, X, T, o)
    return net, info


def compare_solves(pr: Problem, b, net, rtol=1e-8, maxit=20000, cheb_prec=hx.HX_FP32, mode=0):
    """Time and iterations to rtol: Jacobi PCG, Chebyshev PCG, learned FCG (Jacobi fallback)."""
    torch = pr.torch
    out = {}
    forms = {
        "jacobi": dict(),
        "chebyshev4": dict(precond=hx.HX_PC_CHEBYSHEV, cheb_prec=cheb_prec),
        "learned": dict(precond=hx.HX_PC_MLP, mlp=net.value, fallback=hx.HX_PC_JACOBI, mlp_mode=mode),
    }
    for name, o in forms.items():
        torch.cuda.synchronize()
        x, info = pr.solve(b, rtol=rtol, maxit=maxit, check_every=10, raise_on_error=False, **o)
        out[name] = dict(status=info["status"], iterations=info["iterations"], applies=info["operator_applies"],
                         seconds=round(info["solve_seconds"], 4), setup_seconds=round(info["setup_seconds"], 4),
                         true_rel_residual=info["true_rel_residual"], fallback_used=info["fallback_used"],
                         fallback_iterations=info["fallback_iterations"])
    return out
