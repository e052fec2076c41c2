"""Throughput of the fused BP5 diffusion apply (p=7, q=8 GLL-collocated, FP64) on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--N 48] [--p 7] [--no-solves] [--no-cpu-baseline]
                [--no-extra-lines] [--no-suites]

A step is one operator apply y = A x over the whole L-vector (all element colors), inputs resident in
HBM. Prints one JSON line with the metric, the roofline object of the apply kernel (with the general
index path beside it), the BP6, Helmholtz and BP4 apply lines, time-to-1e-8 solves on the same mesh and
across the other workloads (3-component p = 5..8, the variable-coefficient p = 6 problem, the learned
preconditioner), and the oracle CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "GDOF/s diffusion apply p=7; time-to-1e-8 PCG solve, plain FP64 vs mixed/learned"
COUNTERS = os.path.join(ROOT, "profiles", "bp5_p7_n48_counters.json")
KERNEL_SOURCES = ["paper_2109_04996_amd/csrc/colloc_kernel.h", "paper_2109_04996_amd/csrc/strip_kernel.h",
                  "paper_2109_04996_amd/csrc/apply_launch.h", "paper_2109_04996_amd/csrc/mesh.cpp"]
KERNEL_NAME = "hx::k_colloc_strip<8, 1, double, double, 2>"  # strip scatter (degree 7, affine numbering)
KERNEL_NAME_ELEM = "hx::k_colloc<8, 1, double, double, false, true>"  # per-element scatter


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n: int, E: int, P: int, Q: int, ncq: int = 6, ncomp: int = 1) -> dict:
    """Bytes the method must move per apply: read x and write y once (8 B each per DOF), the stored
    pointwise data (ncq FP64 values per point), the element restriction (one int32 per element node)."""
    xy = 16 * n * ncomp
    qd = 8 * ncq * Q ** 3 * E
    ix = 4 * P ** 3 * E
    return dict(total=xy + qd + ix, xy=xy, qdata=qd, index=ix, per_element=(xy + qd + ix) / E)


def time_applies(pr, x, y, steps, warmup):
    import torch
    for _ in range(warmup):
        pr.apply(x, y)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per = []
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        pr.apply(x, y)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev0.elapsed_time(ev1)
    # per-apply distribution (events around each apply, separately)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * min(steps, 50))]
    for i in range(0, len(evs), 2):
        evs[i].record(stream)
        pr.apply(x, y)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(0, len(evs), 2))
    return total_ms, wall, per


def copy_probe(nbytes=4 << 30):
    """Device-to-device copy bandwidth (read + write) of a large buffer: the memcpy probe."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def read_heavy_probe(nbytes=4 << 30, parts=8):
    """Device bandwidth of a read-dominated stream: y = sum of ``parts`` slices of one buffer (``parts``
    reads per write, 8 of 9 bytes read for parts = 8, the mix of the diffusion apply)."""
    import torch
    m = nbytes // 8 // parts
    a = torch.empty(parts, m, dtype=torch.float64, device="cuda").uniform_()
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    for _ in range(3):
        torch.sum(a, dim=0, out=y)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    ev0.record()
    for _ in range(reps):
        torch.sum(a, dim=0, out=y)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, y
    torch.cuda.empty_cache()
    return (parts + 1) * m * 8 / (ms * 1e-3) / 1e9


def apply_line(pr, ab, dofs, steps=50, warmup=20, x=None):
    """Time ``steps`` applies of an operator (HIP events on the launch stream) and express the rate
    against the algorithmic bytes ``ab`` (bytes per apply). Each line follows seconds of host-side
    mesh setup with the GPU idle; the first tens of milliseconds of applies after that run 5-10%
    slower, hence 20 warm-up applies."""
    import torch

    from paper_2109_04996_amd.inputs import uniform_vector
    x = pr.to_dev(uniform_vector(pr.mesh["nnodes"], 1, pr.ncomp)) if x is None else x
    y = pr.zeros()
    total_ms, _, per = time_applies(pr, x, y, steps, warmup)
    ms = total_ms / steps
    del x, y
    return dict(ms_per_apply=round(ms, 4), median_ms=round(per[len(per) // 2], 4), gdofs=round(dofs / ms / 1e6, 3),
                algorithmic_bytes_per_dof=round(ab / dofs, 2),
                achieved_GBs=round(ab / (ms * 1e-3) / 1e9, 1), frac=round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                index_mode=pr.stats["index_mode"], strips=pr.stats["nstrips"],
                strip_groups=pr.stats["nstrip_groups"],
                launches_per_apply=pr.stats["nstrip_colors"] if pr.stats["nstrips"] > 0 else pr.stats["ncolors"])


def pmg_degrees(p):
    """Halving degree schedule of the p-multigrid hierarchy: p, p // 2, ..., 1."""
    d = [p]
    while d[-1] > 1:
        d.append(d[-1] // 2)
    return d


def pmg_hierarchy(pr, rule, warp="A", shuffle_seed=0, kappa=None, **opts):
    """p-multigrid over ``pr`` (level 0) and coarser operators on the same lattice elements; returns
    (handle, coarse problems, setup seconds)."""
    from paper_2109_04996_amd import hexpa as hx
    from paper_2109_04996_amd.problem import Problem
    t0 = time.perf_counter()
    coarse = [Problem(pr.N, pc, pc + 1 if rule == "gll" else pc + 2, rule, pr.kind, ncomp=pr.ncomp, warp=warp,
                      shuffle_seed=shuffle_seed, kappa=kappa) for pc in pmg_degrees(pr.p)[1:]]
    h = hx.hx_pmg_create([pr.h_op] + [c.h_op for c in coarse], hx.hx_pmg_opts_default(**opts))
    return h, coarse, time.perf_counter() - t0


def pmg_close(h, coarse):
    from paper_2109_04996_amd import hexpa as hx
    hx.hx_pmg_destroy(h)
    for c in coarse:
        c.close()


def solves(pr, mass_pr, maxit=20000):
    """Time-to-1e-8 for plain FP64 Jacobi-PCG and the mixed-precision forms, same RHS b = B f^."""
    import numpy as np
    import torch

    from paper_2109_04996_amd import hexpa as hx
    X = pr.xyz
    u_exact = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    f = 3 * np.pi ** 2 * u_exact
    b = mass_pr.apply(pr.to_dev(f))
    u_dev = pr.to_dev(u_exact)
    out = {}
    forms = {
        "fp64_jacobi": dict(),
        "fp64_cg_cheb4_fp32op": dict(precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP32),
        "ir_fp32_jacobi": dict(mode=hx.HX_SOLVE_IR, precond=hx.HX_PC_JACOBI, inner_qdata=hx.HX_FP32),
        "ir_fp32_cheb4": dict(mode=hx.HX_SOLVE_IR, precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP32,
                              inner_qdata=hx.HX_FP32),
        "mixed_fp32_jacobi": dict(mode=hx.HX_SOLVE_MIXED, inner_qdata=hx.HX_FP32),
        "mixed_fp32_cheb4": dict(mode=hx.HX_SOLVE_MIXED, precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP32,
                                 inner_qdata=hx.HX_FP32),
    }
    # p-multigrid V-cycle (degrees p, p/2, ..., 1) inside flexible CG
    mg, coarse, mg_setup = pmg_hierarchy(pr, "gll")
    forms["fp64_fcg_pmg"] = dict(precond=hx.HX_PC_PMG, pmg=mg.value)
    # the same V-cycle in FP32 (vectors, operators with FP32 geometric factors, smoothers) in the FP64 FCG
    mg32, coarse32, mg32_setup = pmg_hierarchy(pr, "gll", prec=hx.HX_FP32)
    forms["fp64_fcg_pmg_fp32"] = dict(precond=hx.HX_PC_PMG, pmg=mg32.value)
    # every form's difference is taken against an FP64 solve to 1e-12 (the p-multigrid FCG)
    ref = pr.solve(b, rtol=1e-12, maxit=2000, check_every=1, precond=hx.HX_PC_PMG, pmg=mg.value)[0].clone()
    for name, o in forms.items():
        print(f"[bench] solve {name}", file=sys.stderr, flush=True)
        x = pr.zeros()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # a V-cycle costs several applies: check every iteration
        x, info = pr.solve(b, x=x, rtol=1e-8, maxit=maxit, check_every=1 if "pmg" in o else 25,
                           raise_on_error=False, **o)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        xs = x.double()
        out[name] = dict(status=info["status"], iterations=info["iterations"],
                         outer=info["outer_iterations"], applies=info["operator_applies"],
                         seconds=round(info["solve_seconds"], 4), setup_seconds=round(info["setup_seconds"], 4),
                         wall_seconds=round(wall, 4), true_rel_residual=info["true_rel_residual"],
                         rel_error_vs_fp64_reference=float(torch.linalg.norm(xs - ref) / torch.linalg.norm(ref)),
                         # discretisation error: max-norm against u = sin sin sin at the nodes
                         err_vs_exact=float((xs - u_dev).abs().max() / u_dev.abs().max()),
                         gdofs_per_iteration=round(pr.n * info["iterations"] / max(info["solve_seconds"], 1e-9) / 1e9,
                                                   2))
    out["fp64_fcg_pmg"].update(degrees=pmg_degrees(pr.p), hierarchy_setup_seconds=round(mg_setup, 3),
                               opts={k: getattr(hx.hx_pmg_opts_default(), k) for k, _ in hx.hx_pmg_opts._fields_})
    out["fp64_fcg_pmg_fp32"].update(degrees=pmg_degrees(pr.p), hierarchy_setup_seconds=round(mg32_setup, 3))
    pmg_close(mg, coarse)
    pmg_close(mg32, coarse32)
    out["reference"] = "FP64 flexible CG with the FP64 p-multigrid V-cycle to 1e-12"
    return _speedups(out)


def _timed_solve(pr, b, ref=None, **o):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = pr.solve(b, rtol=o.pop("rtol", 1e-8), maxit=o.pop("maxit", 40000),
                       check_every=1 if "pmg" in o else 25, raise_on_error=False, **o)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rec = dict(status=info["status"], iterations=info["iterations"], outer=info["outer_iterations"],
               applies=info["operator_applies"], seconds=round(info["solve_seconds"], 4),
               setup_seconds=round(info["setup_seconds"], 4), wall_seconds=round(wall, 4),
               true_rel_residual=info["true_rel_residual"])
    if ref is not None:
        rec["rel_error_vs_fp64_reference"] = float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))
    if info.get("fallback_used"):
        rec["fallback_used"] = 1
        rec["fallback_iterations"] = info["fallback_iterations"]
    return x, rec


def reference_solution(pr, b, rule, kappa=None):
    """FP64 solution to a 1e-12 relative residual (flexible CG with the FP64 p-multigrid V-cycle), against
    which every form's error is reported."""
    mg, coarse, _ = pmg_hierarchy(pr, rule, kappa=kappa)
    ref, info = pr.solve(b, rtol=1e-12, maxit=2000, check_every=1, precond=pmg_precond(), pmg=mg.value)
    pmg_close(mg, coarse)
    if info["status"] != "HX_OK":
        raise RuntimeError(f"reference solve: {info}")
    return ref


def pmg_precond():
    from paper_2109_04996_amd import hexpa as hx
    return hx.HX_PC_PMG


def _speedups(out, base="fp64_jacobi"):
    """time of the plain FP64 Jacobi-PCG solve / time of each form (the solve, setup apart), and the same
    counting each form's own setup (Lanczos estimate, diagonal, p-multigrid hierarchy)."""
    t0 = out[base]["seconds"]
    for k, v in out.items():
        if isinstance(v, dict) and "seconds" in v and v.get("status") == "HX_OK":
            v["vs_fp64_jacobi"] = round(t0 / max(v["seconds"], 1e-9), 3)
            setup = v.get("hierarchy_setup_seconds", 0.0) + v.get("setup_seconds", 0.0)
            v["vs_fp64_jacobi_with_setup"] = round((t0 + out[base].get("setup_seconds", 0.0))
                                                   / max(v["seconds"] + setup, 1e-9), 3)
    return out


def _pmg_form(pr, b, ref, rule, out, name, kappa=None, **pmg_opts):
    from paper_2109_04996_amd import hexpa as hx
    mg, coarse, mg_setup = pmg_hierarchy(pr, rule, kappa=kappa, **pmg_opts)
    _, out[name] = _timed_solve(pr, b, ref, precond=hx.HX_PC_PMG, pmg=mg.value)
    out[name].update(degrees=pmg_degrees(pr.p), hierarchy_setup_seconds=round(mg_setup, 3))
    pmg_close(mg, coarse)


VECTOR_CASES = ((5, 30), (6, 30), (7, 26), (8, 22))  # (p, N): 3.4M to 6.1M nodes x 3 components


def suite_vector_ir(p=6, N=30):
    """Vector diffusion, 3 interleaved components, q = p+2 Gauss: plain FP64 PCG against the FP32-operator
    forms (refinement, one FP32 CG with FP64 residual replacement, FP32 Chebyshev in FP64 CG) and the
    p-multigrid V-cycle."""
    import numpy as np

    from paper_2109_04996_amd import hexpa as hx
    from paper_2109_04996_amd.inputs import lattice_mesh
    from paper_2109_04996_amd.problem import Problem
    print(f"[bench] vector suite p={p} N={N}", file=sys.stderr, flush=True)
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
    pr = Problem(N, p, p + 2, "gauss", "diffusion", ncomp=3, mesh=mesh)
    mass = Problem(N, p, p + 2, "gauss", "mass", ncomp=3, mesh=mesh)
    X = pr.xyz
    f = 3 * np.pi ** 2 * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    b = mass.apply(pr.to_dev((f[:, None] * np.array([1.0, -1.0, 0.5])[None, :]).ravel()))
    mass.close()
    ref = reference_solution(pr, b, "gauss")
    out = dict(workload=f"BP4-type vector diffusion, 3 components, p={p}, q={p + 2} Gauss, mesh A {N}^3, "
                        f"{mesh['nnodes']} nodes x 3, rtol 1e-8; reference: FP64 solve to 1e-12")
    _, out["fp64_jacobi"] = _timed_solve(pr, b, ref)
    _, out["ir_fp32op_fp32qdata"] = _timed_solve(pr, b, ref, mode=hx.HX_SOLVE_IR, inner_qdata=hx.HX_FP32)
    # one FP32 PCG with FP64 residual replacement (reliable updates): the Krylov space is kept
    _, out["mixed_fp32op_fp32qdata"] = _timed_solve(pr, b, ref, mode=hx.HX_SOLVE_MIXED, inner_qdata=hx.HX_FP32)
    _, out["fp64_cg_cheb4_fp32op"] = _timed_solve(pr, b, ref, precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP32)
    _, out["mixed_cheb4_fp32op"] = _timed_solve(pr, b, ref, mode=hx.HX_SOLVE_MIXED, precond=hx.HX_PC_CHEBYSHEV,
                                                cheb_prec=hx.HX_FP32, inner_qdata=hx.HX_FP32)
    _pmg_form(pr, b, ref, "gauss", out, "fp64_fcg_pmg_fp32", prec=hx.HX_FP32)
    pr.close()
    return _speedups(out)


def suite_kappa_cheb(p=6, N=61, kappa_seed=100):
    """Scalar variable-coefficient diffusion, p=6, q=8: FP64 PCG vs FP32/bf16-matrix-core Chebyshev forms and
    the p-multigrid V-cycle."""
    from paper_2109_04996_amd import hexpa as hx
    from paper_2109_04996_amd import learned
    from paper_2109_04996_amd.inputs import kappa_field_params
    print(f"[bench] kappa Chebyshev suite p={p} N={N}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    pr, b = learned.problem_with_kappa(N, p, p + 2, "gauss", kappa_seed)
    setup = time.perf_counter() - t0
    kp = kappa_field_params(kappa_seed, M=512)
    ref = reference_solution(pr, b, "gauss", kappa=kp)
    out = dict(workload=f"diffusion with kappa = exp(g), g a seeded random-Fourier-feature field (seed {kappa_seed}, "
                        f"contrast ~1e2), p={p}, q={p + 2} Gauss, mesh A {N}^3, {pr.mesh['nnodes']} DOFs, b = B 1, "
                        f"rtol 1e-8; reference: FP64 solve to 1e-12", problem_setup_seconds=round(setup, 2))
    _, out["fp64_jacobi"] = _timed_solve(pr, b, ref)
    _, out["fp64_cg_cheb4_fp32op"] = _timed_solve(pr, b, ref, precond=hx.HX_PC_CHEBYSHEV, cheb_prec=hx.HX_FP32)
    # the literal form: FP64 refinement, FP32 operator, Chebyshev(4) on the bf16 matrix cores
    _, out["ir_fp32op_cheb4_bf16mfma"] = _timed_solve(pr, b, ref, mode=hx.HX_SOLVE_IR, precond=hx.HX_PC_CHEBYSHEV,
                                                      cheb_prec=hx.HX_BF16, inner_qdata=hx.HX_FP32, flexible=1)
    # the same matrix cores with hi + lo bfloat16 operands
    _, out["fp64_cg_cheb4_bf16split"] = _timed_solve(pr, b, ref, precond=hx.HX_PC_CHEBYSHEV,
                                                     cheb_prec=hx.HX_BF16_SPLIT, flexible=0)
    _, out["ir_fp32op_cheb4_bf16split"] = _timed_solve(pr, b, ref, mode=hx.HX_SOLVE_IR, precond=hx.HX_PC_CHEBYSHEV,
                                                       cheb_prec=hx.HX_BF16_SPLIT, inner_qdata=hx.HX_FP32,
                                                       flexible=1)
    _, out["mixed_cheb4_bf16split"] = _timed_solve(pr, b, ref, mode=hx.HX_SOLVE_MIXED, precond=hx.HX_PC_CHEBYSHEV,
                                                   cheb_prec=hx.HX_BF16_SPLIT, inner_qdata=hx.HX_FP32, flexible=1)
    _pmg_form(pr, b, ref, "gauss", out, "fp64_fcg_pmg", kappa=kp)
    _pmg_form(pr, b, ref, "gauss", out, "fp64_fcg_pmg_fp32", kappa=kp, prec=hx.HX_FP32)
    # the FP32 hierarchy with the finest level's operator on the matrix cores (hi + lo bf16 operands)
    _pmg_form(pr, b, ref, "gauss", out, "fp64_fcg_pmg_bf16split", kappa=kp, prec=hx.HX_BF16_SPLIT)
    pr.close()
    return _speedups(out)


LOR_CASES = ((3, 57), (5, 35), (7, 25))  # (p, N): 5.1M to 5.5M DOFs


def suite_lor(p=5, N=35, kappa_seed=100):
    """Low-order refined preconditioning (Preconditioning section, FEM-SEM equivalence): the assembled LOR
    matrix (setup time, ELL SpMV rate against its bytes), and flexible CG on the high-order operator with
    the V-cycle of the hierarchy whose finest level is the LOR matrix, against Jacobi-PCG and the
    high-order p-multigrid V-cycle. Variable coefficient (seed 100), GLL-collocated q = p + 1, b = B 1."""
    import torch

    from paper_2109_04996_amd import hexpa as hx
    from paper_2109_04996_amd import learned
    from paper_2109_04996_amd.inputs import kappa_field_params, lattice_mesh
    from paper_2109_04996_amd.problem import Problem
    print(f"[bench] LOR suite p={p} N={N}", file=sys.stderr, flush=True)
    kp = kappa_field_params(kappa_seed, M=512)
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
    pr = Problem(N, p, p + 1, "gll", "diffusion", mesh=mesh, kappa=kp)
    mass = Problem(N, p, p + 2, "gauss", "mass", mesh=mesh)
    b = learned.rhs_ones(pr, mass)
    mass.close()
    n = mesh["nnodes"]
    ref = reference_solution(pr, b, "gll", kappa=kp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lor = Problem(N, p, p + 1, "gll", "lor", mesh=mesh, kappa=kp)
    torch.cuda.synchronize()
    t_lor = time.perf_counter() - t0
    w = lor_width(lor)
    spmv_bytes = (12 * w + 16) * n  # ELL column and value per entry, x read once, y written once
    out = dict(workload=f"diffusion with kappa (seed {kappa_seed}), p={p}, q={p + 1} GLL-collocated, mesh A {N}^3, "
                        f"{n} DOFs, b = B 1, rtol 1e-8; reference: FP64 solve to 1e-12",
               lor_assembly_seconds=round(t_lor, 3), lor_width=w,
               lor_spmv=dict(bound="hbm", peak=HBM_PEAK_GBS, **apply_line(lor, spmv_bytes, n)))
    _, out["fp64_jacobi"] = _timed_solve(pr, b, ref)
    t0 = time.perf_counter()
    coarse = [Problem(N, pc, pc + 1, "gll", "diffusion", mesh=lattice_mesh(N, pc, warp="A", shuffle_seed=0), kappa=kp)
              for pc in pmg_degrees(p)[1:]]
    mg = hx.hx_pmg_create([lor.h_op] + [c.h_op for c in coarse], hx.hx_pmg_opts_default())
    mg_setup = time.perf_counter() - t0
    _, out["fp64_fcg_lor_vcycle"] = _timed_solve(pr, b, ref, precond=hx.HX_PC_PMG, pmg=mg.value)
    out["fp64_fcg_lor_vcycle"].update(degrees=pmg_degrees(p), hierarchy_setup_seconds=round(mg_setup + t_lor, 3))
    hx.hx_pmg_destroy(mg)
    for c in coarse:
        c.close()
    lor.close()
    _pmg_form(pr, b, ref, "gll", out, "fp64_fcg_pmg", kappa=kp)
    pr.close()
    return _speedups(out)


def lor_width(pr):
    """ELL width of a low-order refined operator."""
    import ctypes

    from paper_2109_04996_amd import hexpa as hx
    w = ctypes.c_int()
    hx._check(hx.load().hx_op_lor_matrix(pr.h_op, ctypes.byref(w), None, None), "hx_op_lor_matrix")
    return w.value


LEARNED_CASES = ((4, 43), (5, 35), (6, 29), (7, 25))  # (p, N_eval): 5.2M to 5.5M DOFs


def suite_learned(p=5, N_eval=35, N_train=12, train_seeds=(1000, 1001, 1002, 1003), eval_seed=100):
    """Learned element preconditioner at one degree: training cost, then FCG with the network (alone and as
    the base of a Chebyshev polynomial) against Jacobi and Chebyshev PCG, and the p-multigrid V-cycle with
    the network as its finest smoother's base against the same V-cycle with Jacobi-Chebyshev smoothing, on
    a held-out coefficient field."""
    from paper_2109_04996_amd import hexpa as hx
    from paper_2109_04996_amd import learned
    from paper_2109_04996_amd.inputs import kappa_field_params
    print(f"[bench] learned suite p={p}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    X, T = learned.training_set(p, p + 2, "gauss", N_train, train_seeds, groups_per_field=6, mode=1)
    t_data = time.perf_counter() - t0
    net, info = learned.train(X, T, epochs=100, batch=256, lr=1e-3)
    print(f"[bench] learned: {X.shape[0]} rows, data {t_data:.1f} s, training {info['seconds']:.1f} s",
          file=sys.stderr, flush=True)
    pr, b = learned.problem_with_kappa(N_eval, p, p + 2, "gauss", eval_seed)
    res = learned.compare_solves(pr, b, net)
    # the stronger non-learned baseline: p-multigrid (degrees p, p/2, ..., 1) in flexible CG, and the same
    # V-cycle with the learned map as the base of its finest smoother
    kp = kappa_field_params(eval_seed, M=512)
    for name, extra in (("pmg", {}), ("pmg_learned_smoother", dict(smoother_mlp=net.value))):
        mg, coarse, mg_setup = pmg_hierarchy(pr, "gauss", kappa=kp, **extra)
        _, res[name] = _timed_solve(pr, b, None, precond=hx.HX_PC_PMG, pmg=mg.value)
        res[name].update(degrees=pmg_degrees(p), hierarchy_setup_seconds=round(mg_setup, 3))
        pmg_close(mg, coarse)
    out = dict(workload=f"diffusion with kappa (held-out seed {eval_seed}), p={p}, q={p + 2} Gauss, mesh A "
                        f"{N_eval}^3, {pr.mesh['nnodes']} DOFs, b = B 1, rtol 1e-8",
               training=dict(rows=int(X.shape[0]), data_seconds=round(t_data, 2),
                             train_seconds=round(info["seconds"], 2), steps=info["steps"],
                             first_loss=info["first_loss"], final_loss=info["final_loss"],
                             train_problems=f"{len(train_seeds)} coefficient seeds {train_seeds}, mesh {N_train}^3, "
                                            "exact element-patch solves of Jacobi-PCG residuals"),
               **res)
    t = {k: v["seconds"] for k, v in res.items()}
    # each learned form against its own fallback, against plain FP64 Jacobi PCG and against p-multigrid
    out["gain"] = dict(learned_vs_jacobi=round(t["jacobi"] / max(t["learned"], 1e-9), 3),
                       learned_cheb4_vs_chebyshev4=round(t["chebyshev4"] / max(t["learned_cheb4"], 1e-9), 3),
                       learned_cheb4_vs_jacobi=round(t["jacobi"] / max(t["learned_cheb4"], 1e-9), 3),
                       learned_smoother_vs_pmg=round(t["pmg"] / max(t["pmg_learned_smoother"], 1e-9), 3),
                       learned_smoother_iterations_vs_pmg=(res["pmg_learned_smoother"]["iterations"],
                                                           res["pmg"]["iterations"]),
                       best_learned_vs_pmg=round(t["pmg"] / max(min(t["learned"], t["learned_cheb4"],
                                                                    t["pmg_learned_smoother"]), 1e-9), 3))
    best_learned = min(t["learned"], t["learned_cheb4"], t["pmg_learned_smoother"])
    best_plain = min(t["jacobi"], t["chebyshev4"], t["chebyshev4_fp32"], t["pmg"])
    saved = best_plain - best_learned
    cost = t_data + info["seconds"]  # training data and training, paid once per operator family
    out["break_even_solves"] = (round(cost / saved, 1) if saved > 0 else None)
    saved_j = t["jacobi"] - best_learned
    out["break_even_solves_vs_jacobi"] = (round(cost / saved_j, 1) if saved_j > 0 else None)
    out["break_even_note"] = ("solves after which the training cost is repaid by the time the fastest learned form "
                              "saves per solve: over the fastest form without the network (break_even_solves), "
                              "and over plain FP64 Jacobi-PCG (break_even_solves_vs_jacobi); null where the learned "
                              "form saves nothing")
    pr.close()
    hx.hx_mlp_destroy(net)
    return out


SWEEP = [  # (label, kind, rule, p, q, ncomp, N list)
    ("BP5", "diffusion", "gll", 7, 8, 1, (15, 20, 28, 36, 44, 48)),
    ("BP5", "diffusion", "gll", 4, 5, 1, (25, 45, 65, 85)),
    ("BP5", "diffusion", "gll", 2, 3, 1, (50, 110, 170)),
    ("BP1", "mass", "gauss", 7, 9, 1, (15, 20, 28, 36, 44, 48)),
    ("BP1", "mass", "gauss", 4, 6, 1, (25, 45, 65, 85)),
    ("BP1", "mass", "gauss", 2, 4, 1, (50, 110, 170)),
    ("BP3", "diffusion", "gauss", 6, 8, 1, (48,)),
    ("BP3", "diffusion", "gauss", 7, 9, 1, (15, 28, 36, 48)),
    ("BP2", "mass", "gauss", 7, 9, 3, (32,)),
    ("BP4", "diffusion", "gauss", 7, 9, 3, (32,)),
    ("BP6", "diffusion", "gll", 7, 8, 3, (32,)),
]


CG_SWEEP_N = (2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48)


def cg_sweep(label="BP5", p=7, q=8, rule="gll", Ns=CG_SWEEP_N, short=20, long=60):
    """Throughput per CG iteration against problem size (the strong-scale limit on one GPU):
    FP64 Jacobi-PCG on BP5 (q = p+1 GLL) or BP3 (q = p+2 Gauss), mesh A, Dirichlet, b a seeded
    random vector on the free nodes, with the CG operator in both forms: the colored scatter (one
    launch per color) and the E-vector apply plus a node gather with p'Ap fused (two launches).
    Each is timed as the difference of a long and a short run, so the setup, the first residual and
    the final checks cancel. One JSON line per size, then r_max, n_0.8 and t_0.8 (the largest
    throughput, the smallest n reaching 80% of it, and its time per iteration) for each form and for
    the faster of the two at each size."""
    import numpy as np
    import torch

    from paper_2109_04996_amd import hexpa as hx
    from paper_2109_04996_amd.inputs import lattice_mesh, uniform_vector
    from paper_2109_04996_amd.problem import Problem
    forms = {"colors": hx.HX_SCATTER_COLORS, "gather": hx.HX_SCATTER_GATHER}
    rows = []
    for N in Ns:
        mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
        with Problem(N, p, q, rule, "diffusion", mesh=mesh) as pr:
            free = pr.to_dev((mesh["boundary"] == 0).astype(np.float64))
            b = pr.to_dev(uniform_vector(mesh["nnodes"], 2)) * free
            n = mesh["nnodes"]
            rec = dict(cg_sweep=label, p=p, q=q, N=N, dofs=n, dofs_paper=mesh["nelem"] * p ** 3)
            for fname, sc in forms.items():
                t = {}
                for k in (short, long):
                    best = None
                    for _ in range(3):
                        torch.cuda.synchronize()
                        x, info = pr.solve(b, rtol=1e-30, maxit=k, check_every=k, raise_on_error=False, scatter=sc)
                        if info["iterations"] != k:
                            raise RuntimeError(f"CG stopped after {info['iterations']} of {k} iterations at N={N}")
                        best = info["solve_seconds"] if best is None else min(best, info["solve_seconds"])
                    t[k] = best
                per_it = (t[long] - t[short]) / (long - short)
                rec[f"us_per_iteration_{fname}"] = round(per_it * 1e6, 2)
                rec[f"gdofs_per_iteration_{fname}"] = round(n / per_it / 1e9, 3)
            best = min(forms, key=lambda f: rec[f"us_per_iteration_{f}"])
            rec["us_per_iteration"] = rec[f"us_per_iteration_{best}"]
            rec["gdofs_per_iteration"] = rec[f"gdofs_per_iteration_{best}"]
            rec["faster"] = best
            rows.append(rec)
            print(json.dumps(rec), flush=True)
    summary = dict(cg_sweep_summary=label, p=p, q=q)
    for suffix in ("_colors", "_gather", ""):
        rmax = max(r["gdofs_per_iteration" + suffix] for r in rows)
        n08 = min((r for r in rows if r["gdofs_per_iteration" + suffix] >= 0.8 * rmax), key=lambda r: r["dofs"])
        summary.update({f"r_max_gdofs{suffix}": rmax, f"n_0_8{suffix}": n08["dofs"],
                        f"t_0_8_us{suffix}": n08["us_per_iteration" + suffix],
                        f"min_us_per_iteration{suffix}": min(r["us_per_iteration" + suffix] for r in rows)})
    print(json.dumps(summary), flush=True)


def sweep(steps=20, warmup=3):
    """Apply throughput over mesh sizes (p = 7, 4, 2) and the other operator kinds: one JSON line per
    case (FP64 operator; FP32-operator figures beside it)."""
    import torch

    from paper_2109_04996_amd import hexpa as hx
    from paper_2109_04996_amd.inputs import lattice_mesh, uniform_vector
    from paper_2109_04996_amd.problem import Problem

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    for label, kind, rule, p, q, nc, Ns in SWEEP:
        for N in Ns:
            print(f"[bench] sweep {label} p={p} q={q} ncomp={nc} N={N}", file=sys.stderr, flush=True)
            mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
            pr = Problem(N, p, q, rule, kind, ncomp=nc, mesh=mesh)
            n = mesh["nnodes"]
            x = pr.to_dev(uniform_vector(n, 1, nc))
            y = pr.zeros()
            x32, y32 = x.float(), torch.zeros(pr.n, dtype=torch.float32, device="cuda")
            ms = timed(lambda: pr.apply(x, y))
            ms32 = timed(lambda: hx.hx_op_apply_f32(pr.h_op, hx.HX_FP32, x32, y32))
            ab = algorithmic_bytes(n, mesh["nelem"], p + 1, q, 1 if kind == "mass" else 6, nc)
            dofs = n * nc
            print(json.dumps(dict(sweep=label, kind=kind, rule=rule, p=p, q=q, ncomp=nc, N=N, dofs=dofs,
                                  fp64_ms=round(ms, 4), fp64_gdofs=round(dofs / ms / 1e6, 2),
                                  algorithmic_bytes_per_dof=round(ab["total"] / dofs, 1),
                                  roofline_frac=round(ab["total"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
                                  fp32_q32_ms=round(ms32, 4), fp32_q32_gdofs=round(dofs / ms32 / 1e6, 2),
                                  cache_assisted=bool(ab["total"] < 1.5e9), strips=pr.stats["nstrips"])),
                  flush=True)
            pr.close()
            del x, y, x32, y32
            torch.cuda.empty_cache()


def _oracle_threads() -> int:
    """Host threads the oracle's SpMV uses: the cores this process may run on, at most 16 (the host
    share of one GPU on the measurement boxes)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(p: int, budget_s: float = 6.0):
    """The oracle on bounded samples of the same workload, on the host cores: the assembled-matrix SpMV
    (scipy CSR, one thread and all threads over row blocks), and the oracle's Jacobi-PCG to 1e-8 beside
    the GPU's on the same small problems (the CPU-scale configuration, N=4 p=3 q=5 Gauss, and BP5 p=7 on
    6^3 elements)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    from oracle import fem, solvers
    from paper_2109_04996_amd.inputs import lattice_mesh, uniform_vector
    from paper_2109_04996_amd.problem import Problem
    N = 6
    t0 = time.perf_counter()
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
    A = fem.assemble(mesh, p, p + 1, "gll", "diffusion").tocsr()
    t_asm = time.perf_counter() - t0
    n = mesh["nnodes"]
    x = uniform_vector(n, 1)

    def rate(fn):
        fn()
        reps, t = 0, 0.0
        while t < budget_s and reps < 400:
            t1 = time.perf_counter()
            fn()
            t += time.perf_counter() - t1
            reps += 1
        return n * reps / t / 1e9, reps, t

    r1, reps1, t1 = rate(lambda: A @ x)
    nt = _oracle_threads()
    cuts = np.linspace(0, n, nt + 1).astype(np.int64)
    blocks = [A[cuts[i]:cuts[i + 1]] for i in range(nt)]
    y = np.empty(n)

    def part(i):
        y[cuts[i]:cuts[i + 1]] = blocks[i] @ x

    with ThreadPoolExecutor(nt) as ex:
        rn, repsn, tn = rate(lambda: list(ex.map(part, range(nt))))
    assert np.allclose(y, A @ x, rtol=1e-13, atol=1e-13 * np.abs(y).max())
    out = dict(value=round(rn, 5), unit="GDOF/s", cores=nt, kind="oracle",
               sample=f"oracle scipy CSR SpMV of the assembled BP5 p={p} q={p + 1} GLL matrix, mesh A {N}^3 "
                      f"elements, {n} DOFs, nnz {A.nnz}: {nt} threads over row blocks, {repsn} applies in "
                      f"{tn:.2f} s; assembly {t_asm:.1f} s excluded",
               one_core_value=round(r1, 5), one_core_sample=f"the same SpMV on one thread, {reps1} applies in {t1:.2f} s")

    # the oracle's Jacobi-PCG (one thread) and the GPU's on the same problems, b = B f^, rtol 1e-8
    pcg = []
    for (Np, pp, q, rule) in ((4, 3, 5, "gauss"), (N, p, p + 1, "gll")):
        m = mesh if (Np, pp) == (N, p) else lattice_mesh(Np, pp, warp="A", shuffle_seed=0)
        X = fem.node_coordinates(m, pp)
        f = 3 * np.pi ** 2 * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
        Ao = A if (Np, pp) == (N, p) else fem.assemble(m, pp, q, rule, "diffusion").tocsr()
        bo = fem.assemble(m, pp, pp + 2, "gauss", "mass") @ f
        free = solvers.free_mask(m["boundary"])
        t2 = time.perf_counter()
        xo, ito, reso = solvers.jacobi_pcg(Ao, bo, free, tol=1e-8)
        t_or = time.perf_counter() - t2
        with Problem(Np, pp, q, rule, "diffusion", mesh=m) as pr, \
                Problem(Np, pp, pp + 2, "gauss", "mass", mesh=m) as pm:
            Xg = pr.xyz
            b = pm.apply(pr.to_dev(3 * np.pi ** 2 * np.sin(np.pi * Xg[:, 0]) * np.sin(np.pi * Xg[:, 1])
                                   * np.sin(np.pi * Xg[:, 2])))
            pr.solve(b, rtol=1e-8)  # warm-up (diagonal, buffers)
            torch.cuda.synchronize()
            xg, info = pr.solve(b, rtol=1e-8, check_every=10)
            xg = xg.cpu().numpy()
        pcg.append(dict(problem=f"diffusion p={pp} q={q} {rule}, mesh A {Np}^3, {m['nnodes']} DOFs, b = B f^, "
                                f"rtol 1e-8", oracle_seconds=round(t_or, 4), oracle_iterations=int(ito),
                        oracle_threads=1, gpu_seconds=round(info["solve_seconds"], 5),
                        gpu_iterations=info["iterations"],
                        gpu_vs_oracle_rel_diff=float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))))
    out["pcg"] = pcg
    return out


def extra_lines(out, mesh, N, p, roof):
    """Apply lines beside the headline on the same 48^3 lattice: the general index path (20% of the
    elements rotated, so the kernels read the full element restriction), BP6 (3-component collocated
    diffusion) and the fused Helmholtz operator alpha A + beta B (collocated mass as a diagonal term);
    and BP4 (3-component Gauss diffusion, q = p + 2) on a 40^3 lattice."""
    import torch

    from paper_2109_04996_amd.inputs import lattice_mesh, rotate_elements
    from paper_2109_04996_amd.problem import Problem
    Q = p + 1
    E, n = mesh["nelem"], mesh["nnodes"]
    print("[bench] general index path (20% of elements rotated)", file=sys.stderr, flush=True)
    rot = rotate_elements(mesh, p, 0.2, seed=5)
    with Problem(N, p, Q, "gll", "diffusion", mesh=rot) as pg:
        ab = algorithmic_bytes(n, E, p + 1, Q)
        roof["general_path"] = dict(workload=f"BP5 p={p} N={N} with 20% of the elements rotated (seed 5): full "
                                             "element restriction", **apply_line(pg, ab["total"], n))
    del rot
    torch.cuda.empty_cache()
    print("[bench] BP6 vector apply", file=sys.stderr, flush=True)
    with Problem(N, p, Q, "gll", "diffusion", ncomp=3, mesh=mesh) as p6:
        ab = algorithmic_bytes(n, E, p + 1, Q, 6, 3)
        out["bp6"] = dict(workload=f"BP6 3-component diffusion apply, p={p}, q={Q} GLL-collocated, FP64, mesh A "
                                   f"{N}^3, {n} nodes x 3 interleaved", bound="hbm", peak=HBM_PEAK_GBS,
                          **apply_line(p6, ab["total"], 3 * n))
    torch.cuda.empty_cache()
    print("[bench] Helmholtz apply", file=sys.stderr, flush=True)
    with Problem(N, p, Q, "gll", "helmholtz", mesh=mesh, helmholtz=(1.0, 1.0)) as ph:
        ab = algorithmic_bytes(n, E, p + 1, Q, 7, 1)
        out["helmholtz"] = dict(workload=f"fused alpha A + beta B (alpha = beta = 1), p={p}, q={Q} GLL-collocated "
                                         f"(mass diagonal), FP64, mesh A {N}^3, {n} DOFs", bound="hbm",
                                peak=HBM_PEAK_GBS, **apply_line(ph, ab["total"], n))
    torch.cuda.empty_cache()
    # BP4 on its own 40^3 lattice (q = p + 2 Gauss points, 3 components: the joint-component kernel)
    N4 = 40
    print(f"[bench] BP4 vector apply ({N4}^3)", file=sys.stderr, flush=True)
    mesh4 = lattice_mesh(N4, p, warp="A", shuffle_seed=0)
    n4 = mesh4["nnodes"]
    with Problem(N4, p, p + 2, "gauss", "diffusion", ncomp=3, mesh=mesh4) as p4:
        ab = algorithmic_bytes(n4, mesh4["nelem"], p + 1, p + 2, 6, 3)
        out["bp4"] = dict(workload=f"BP4 3-component diffusion apply, p={p}, q={p + 2} Gauss, FP64, mesh A {N4}^3, "
                                   f"{n4} nodes x 3 interleaved", bound="hbm", peak=HBM_PEAK_GBS,
                          **apply_line(p4, ab["total"], 3 * n4))
    del mesh4
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--N", type=int, default=48)
    ap.add_argument("--p", type=int, default=7)
    ap.add_argument("--no-solves", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-lines", action="store_true",
                    help="skip the general-index-path, BP6 vector and Helmholtz apply lines")
    ap.add_argument("--copy-probe", action="store_true", help="(the copy probe always runs; kept for old commands)")
    ap.add_argument("--no-suites", action="store_true",
                    help="skip the time-to-solution suites (vector p = 5..8, variable coefficient, learned)")
    ap.add_argument("--all", action="store_true", help="(the suites always run unless --no-suites; kept for old "
                                                       "commands)")
    ap.add_argument("--sweep", action="store_true",
                    help="apply throughput over the size sweep and the other operator kinds (one JSON line each)")
    ap.add_argument("--pmc-workload", default="bp5", choices=["bp5", "general", "bp4"],
                    help="workload of --pmc-run: BP5 p=7 48^3 (default), the same with 20%% of the elements rotated, "
                         "or BP4 3-component p=7 q=9 40^3")
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for rocprofv3 counter passes: a 1 GiB reference copy, then 6 applies")
    ap.add_argument("--cg-sweep", action="store_true",
                    help="throughput per Jacobi-PCG iteration against problem size (BP5 and BP3 at p=7, 3e3 to 38M DOFs)")
    ap.add_argument("--pmc-kernels", action="store_true",
                    help="short run for the FLOP-rate counter pass: 4 applies of each hot kernel (BP5 p=7 FP64 and "
                         "FP32; p=6 q=8 Gauss FP64, FP32 and both bf16 matrix-core forms; BP4 p=7 q=9 FP64 and FP32)")
    ap.add_argument("--pmg-sweep", action="store_true",
                    help="p-multigrid FCG (FP64 and FP32 V-cycles) against Jacobi-PCG on BP5 p=7 over mesh sizes")
    ap.add_argument("--pmg-vcycles", type=int, default=0,
                    help="time this many p-multigrid V-cycles (degrees p, p/2, ..., 1) on the BP5 problem and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): the library implements the single-GPU "
              "path; multi-GPU sharding is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2109_04996_amd import hexpa as hx
    from paper_2109_04996_amd.inputs import lattice_mesh, uniform_vector
    from paper_2109_04996_amd.problem import Problem

    hx.load()
    torch.cuda.set_device(0)
    if a.sweep:
        sweep()
        return
    if a.pmg_sweep:
        import numpy as np
        for Ns in (12, 24, 36, 48):
            print(f"[bench] pmg sweep N={Ns}", file=sys.stderr, flush=True)
            mesh_s = lattice_mesh(Ns, 7, warp="A", shuffle_seed=0)
            pr_s = Problem(Ns, 7, 8, "gll", "diffusion", mesh=mesh_s)
            mass_s = Problem(Ns, 7, 9, "gauss", "mass", mesh=mesh_s)
            X = pr_s.xyz
            f = 3 * np.pi ** 2 * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
            b_s = mass_s.apply(pr_s.to_dev(f))
            mass_s.close()
            rec = dict(pmg_sweep="BP5", p=7, N=Ns, dofs=pr_s.n)
            _, rec["fp64_jacobi"] = _timed_solve(pr_s, b_s)
            for name, prec in (("fp64_fcg_pmg", hx.HX_FP64), ("fp64_fcg_pmg_fp32", hx.HX_FP32)):
                mg, coarse, mg_setup = pmg_hierarchy(pr_s, "gll", prec=prec)
                _, rec[name] = _timed_solve(pr_s, b_s, precond=hx.HX_PC_PMG, pmg=mg.value)
                rec[name]["hierarchy_setup_seconds"] = round(mg_setup, 3)
                pmg_close(mg, coarse)
            print(json.dumps(rec), flush=True)
            pr_s.close()
        return
    if a.cg_sweep:
        cg_sweep("BP5", 7, 8, "gll")
        cg_sweep("BP3", 7, 9, "gauss")
        return
    if a.pmc_run and a.pmc_workload != "bp5":
        # reference copy of known size (1 GiB read + 1 GiB written), then 6 applies of the named workload
        from paper_2109_04996_amd.inputs import rotate_elements
        if a.pmc_workload == "general":
            mesh_w = rotate_elements(lattice_mesh(48, 7, warp="A", shuffle_seed=0), 7, 0.2, seed=5)
            pw = Problem(48, 7, 8, "gll", "diffusion", mesh=mesh_w)
        else:
            # the BP4 line's size (40^3 elements, 3 x 22.2M DOFs)
            mesh_w = lattice_mesh(40, 7, warp="A", shuffle_seed=0)
            pw = Problem(40, 7, 9, "gauss", "diffusion", ncomp=3, mesh=mesh_w)
        xw = pw.to_dev(uniform_vector(mesh_w["nnodes"], 1, pw.ncomp))
        yw = pw.zeros()
        ref_a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").uniform_()
        ref_b = torch.empty_like(ref_a)
        ref_b.copy_(ref_a)
        for _ in range(6):
            pw.apply(xw, yw)
        torch.cuda.synchronize()
        ab = algorithmic_bytes(mesh_w["nnodes"], mesh_w["nelem"], 8, pw.q, 6, pw.ncomp)
        st = pw.stats
        launches = st["nstrip_colors"] if st["nstrips"] > 0 and pw.q == 8 else st["ncolors"]
        print(json.dumps(dict(pmc_run=True, workload=a.pmc_workload, copy_bytes=2 << 30,
                              algorithmic_bytes_per_apply=ab["total"], launches_per_apply=launches,
                              index_mode=st["index_mode"])), flush=True)
        pw.close()
        return
    N, p = a.N, a.p
    P = Q = p + 1
    print(f"[bench] building BP5 mesh N={N} p={p}", file=sys.stderr, flush=True)
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
    pr = Problem(N, p, Q, "gll", "diffusion", mesh=mesh)
    n, E = mesh["nnodes"], mesh["nelem"]
    x = pr.to_dev(uniform_vector(n, 1))
    y = pr.zeros()
    if a.pmc_kernels:
        from paper_2109_04996_amd import hexpa as hxm
        for _ in range(4):
            pr.apply(x, y)
        x32, y32 = x.float(), pr.zeros(torch.float32)
        for _ in range(4):
            pr.apply_f32(x32, hxm.HX_FP32, y32)
        pr.close()
        mesh6 = lattice_mesh(48, 6, warp="A", shuffle_seed=0)
        with Problem(48, 6, 8, "gauss", "diffusion", mesh=mesh6) as p6:
            x6 = p6.to_dev(uniform_vector(mesh6["nnodes"], 1))
            y6 = p6.zeros()
            x6f, y6f = x6.float(), p6.zeros(torch.float32)
            for _ in range(4):
                p6.apply(x6, y6)
            for _ in range(4):
                p6.apply_f32(x6f, hxm.HX_FP32, y6f)
            for prec in (hxm.HX_BF16, hxm.HX_BF16_SPLIT):
                for _ in range(4):
                    p6.apply_bf16(x6f, y6f, prec=prec)
            torch.cuda.synchronize()
        del mesh6
        mesh4 = lattice_mesh(32, 7, warp="A", shuffle_seed=0)
        with Problem(32, 7, 9, "gauss", "diffusion", ncomp=3, mesh=mesh4) as p4:
            x4 = p4.to_dev(uniform_vector(mesh4["nnodes"], 1, 3))
            y4 = p4.zeros()
            x4f, y4f = x4.float(), p4.zeros(torch.float32)
            for _ in range(4):
                p4.apply(x4, y4)
            for _ in range(4):
                p4.apply_f32(x4f, hxm.HX_FP32, y4f)
            torch.cuda.synchronize()
        print(json.dumps(dict(pmc_kernels=True, workloads=["bp5_p7_n48 FP64 and FP32",
                                                           "p6_q8_gauss_n48 FP64, FP32, bf16, bf16 split",
                                                           "bp4_p7_q9_n32 FP64 and FP32"])),
              flush=True)
        return
    if a.pmg_vcycles:
        mg, coarse, mg_setup = pmg_hierarchy(pr, "gll")
        r = pr.to_dev(uniform_vector(n, 2) * (mesh["boundary"] == 0))
        z = pr.zeros()
        for _ in range(2):
            hx.hx_pmg_vcycle(mg, r, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.pmg_vcycles):
            hx.hx_pmg_vcycle(mg, r, z)
        torch.cuda.synchronize()
        ms_vc = 1e3 * (time.perf_counter() - t0) / a.pmg_vcycles
        print(json.dumps(dict(pmg_vcycles=a.pmg_vcycles, ms_per_vcycle=round(ms_vc, 3), degrees=pmg_degrees(p),
                              setup_seconds=round(mg_setup, 3), workload=f"bp5_p{p}_n{N}",
                              opts={k: getattr(hx.hx_pmg_opts_default(), k) for k, _ in hx.hx_pmg_opts._fields_})),
              flush=True)
        pmg_close(mg, coarse)
        pr.close()
        return
    if a.pmc_run:
        # reference copy of known size (1 GiB read + 1 GiB written) for scaling the counters
        ref_a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").uniform_()
        ref_b = torch.empty_like(ref_a)
        ref_b.copy_(ref_a)
        for _ in range(6):
            pr.apply(x, y)
        torch.cuda.synchronize()
        strips = pr.stats["nstrips"] > 0
        print(json.dumps(dict(pmc_run=True, kernel=KERNEL_NAME if strips else KERNEL_NAME_ELEM,
                              kernel_hash=kernel_hash(), workload=f"bp5_p{p}_n{N}", copy_bytes=2 << 30,
                              launches_per_apply=pr.stats["nstrip_colors"] if strips else pr.stats["ncolors"])),
              flush=True)
        return
    print(f"[bench] n={n} E={E} colors={pr.stats['ncolors']}; timing {a.steps} applies", file=sys.stderr, flush=True)
    total_ms, wall, per = time_applies(pr, x, y, a.steps, a.warmup)
    ms = total_ms / a.steps
    gdofs = n / (ms * 1e-3) / 1e9
    ab = algorithmic_bytes(n, E, P, Q)
    strips = pr.stats["nstrips"] > 0
    ncol = pr.stats["nstrip_colors"] if strips else pr.stats["ncolors"]  # launches per apply
    achieved = ab["total"] / (ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(COUNTERS):
        c = json.load(open(COUNTERS))
        if c.get("kernel_hash") == kernel_hash() and c.get("workload") == f"bp5_p{p}_n{N}":
            traffic = c.get("hbm_bytes_per_launch")
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=KERNEL_NAME if strips else KERNEL_NAME_ELEM,
                launches_per_apply=ncol, algorithmic_bytes_per_launch=round(ab["total"] / ncol),
                avg_launch_us=round(1e3 * ms / ncol, 2), algorithmic_bytes_per_dof=round(ab["total"] / n, 2),
                kernel_hash=kernel_hash())
    out = dict(metric=METRIC, value=round(gdofs, 3), unit="GDOF/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
               ms_per_step=round(ms, 4), higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload=f"BP5 scalar diffusion apply, p={p}, q={Q} GLL-collocated, FP64, "
                                    f"warped unit-cube mesh A {N}^3 elements shuffled (seed 0), {n} DOFs, "
                                    f"x ~ U[-1,1] (seed 1)",
                           N=N, p=p, q=Q, dofs=n, elements=E, element_colors=pr.stats["ncolors"],
                           strips=pr.stats["nstrips"], launches_per_apply=ncol),
               median_ms=round(per[len(per) // 2], 4), p10_ms=round(per[len(per) // 10], 4),
               p90_ms=round(per[(9 * len(per)) // 10], 4), roofline=roof)
    # the same algorithmic rate against a measured device-to-device copy of 4 GiB (read + write), and
    # against a read-heavy stream of 8 reads per write (the apply's mix: 89% of its bytes are reads)
    cp = copy_probe()
    roof["copy_probe_GBs"] = round(cp, 1)
    roof["frac_vs_copy"] = round(achieved / cp, 4)
    rh = read_heavy_probe()
    roof["read_heavy_probe_GBs"] = round(rh, 1)
    roof["frac_vs_read_heavy_probe"] = round(achieved / rh, 4)
    # the affine node numbering moves 16 bytes of index per element instead of 4 (p+1)^3
    if pr.stats["index_mode"] == 2:
        moved = ab["total"] - ab["index"] + 16 * E
        roof["frac_bytes_moved"] = round(moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        roof["bytes_moved_per_dof"] = round(moved / n, 2)
    roof["target_frac"] = 0.60
    if not a.no_solves:
        mass_pr = Problem(N, p, p + 2, "gauss", "mass", mesh=mesh)
        out["solves"] = dict(workload=f"BP5 p={p} N={N} Dirichlet, b = B f^, f = 3 pi^2 sin sin sin, rtol 1e-8",
                             **solves(pr, mass_pr))
        mass_pr.close()
    pr.close()
    del x, y
    if not a.no_extra_lines:
        extra_lines(out, mesh, N, p, roof)
    if not a.no_suites:
        # time-to-1e-8 across the workloads: vector problems p = 5..8, the variable-coefficient problem, the
        # learned preconditioner; a suite that fails records its error instead of ending the run
        def run(name, fn, *args):
            torch.cuda.empty_cache()
            t0 = time.perf_counter()
            try:
                res = fn(*args)
            except Exception as e:  # noqa: BLE001 - reported in the line
                res = dict(error=f"{type(e).__name__}: {e}")
            res["suite_wall_seconds"] = round(time.perf_counter() - t0, 1)
            return res
        out["vector"] = {f"p{pv}": run("vector", suite_vector_ir, pv, Nv) for pv, Nv in VECTOR_CASES}
        out["kappa_chebyshev"] = run("kappa", suite_kappa_cheb)
        out["lor"] = {f"p{pl}": run("lor", suite_lor, pl, Nl) for pl, Nl in LOR_CASES}
        out["learned"] = {f"p{pl}": run("learned", suite_learned, pl, Nl) for pl, Nl in LEARNED_CASES}
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
