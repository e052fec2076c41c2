"""GPU tests of the learned element preconditioner: network gradients and inference against the
FP64 oracle, the element features, training, the flexible-CG solve and its fallback."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fem, solvers  # noqa: E402
from oracle import mlp as omlp  # noqa: E402
from paper_2109_04996_amd import hexpa as hx  # noqa: E402
from paper_2109_04996_amd import learned  # noqa: E402
from paper_2109_04996_amd.inputs import kappa_field_params, lattice_mesh, rotate_elements  # noqa: E402
from paper_2109_04996_amd.problem import Problem  # noqa: E402


def _split(params, I, H, O):
    a = 0
    out = {}
    for k, shape in (("W1", (H, I)), ("b1", (H,)), ("W2", (O, H)), ("b2", (O,))):
        size = int(np.prod(shape))
        out[k] = params[a:a + size].reshape(shape).astype(np.float64)
        a += size
    return out


def _join(d):
    return np.concatenate([d[k].ravel() for k in ("W1", "b1", "W2", "b2")]).astype(np.float32)


@pytest.fixture
def small_net():
    I, H, O = 70, 33, 27  # odd sizes: partial tiles everywhere
    net = hx.hx_mlp_create(I, H, O, 3)
    rng = np.random.default_rng(0)
    p = hx.hx_mlp_get_params(net)
    p[:] = rng.uniform(-0.3, 0.3, p.size).astype(np.float32)  # non-zero biases too
    hx.hx_mlp_set_params(net, p)
    yield net, I, H, O
    hx.hx_mlp_destroy(net)


def test_gradients_match_oracle(small_net):
    # FP32 forward/backward vs the oracle's FP64 chain rule on the same batch: <= 1e-4 relative per tensor
    net, I, H, O = small_net
    print("\n[case] mlp gradients", flush=True)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((131, I)).astype(np.float32)
    T = rng.standard_normal((131, O)).astype(np.float32)
    loss, g = hx.hx_mlp_loss_grad(net, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    prm = _split(hx.hx_mlp_get_params(net), I, H, O)
    lo, go = omlp.loss_and_grads(prm, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    gg = _split(g, I, H, O)
    for k in go:
        assert np.linalg.norm(gg[k] - go[k]) <= 1e-4 * np.linalg.norm(go[k]), k


def test_forward_fp32_and_bf16(small_net):
    net, I, H, O = small_net
    print("\n[case] mlp forward", flush=True)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((517, I)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Y32 = torch.empty(517, O, device="cuda")
    Y16 = torch.empty(517, O, device="cuda")
    hx.hx_mlp_forward(net, hx.HX_FP32, Xd, Y32)
    hx.hx_mlp_forward(net, hx.HX_BF16, Xd, Y16)
    prm = _split(hx.hx_mlp_get_params(net), I, H, O)
    Yo, _ = omlp.forward(prm, X.astype(np.float64))
    y32, y16 = Y32.cpu().numpy(), Y16.cpu().numpy()
    assert np.linalg.norm(y32 - Yo) <= 1e-5 * np.linalg.norm(Yo)
    # bf16 operands (2^-9 relative rounding) through two layers: about 1e-2
    assert np.linalg.norm(y16 - Yo) <= 2e-2 * np.linalg.norm(Yo)


def test_save_load_roundtrip(small_net, tmp_path):
    net, I, H, O = small_net
    path = str(tmp_path / "net.hxmlp")
    hx.hx_mlp_save(net, path)
    net2 = hx.hx_mlp_load(path)
    try:
        assert hx.hx_mlp_get_shape(net2) == (I, H, O)
        assert np.array_equal(hx.hx_mlp_get_params(net2), hx.hx_mlp_get_params(net))
    finally:
        hx.hx_mlp_destroy(net2)


def test_training_reduces_loss():
    # learn a fixed random linear map: the loss must fall by orders of magnitude
    rng = np.random.default_rng(3)
    X = rng.standard_normal((2048, 16)).astype(np.float32)
    A = rng.standard_normal((16, 8)).astype(np.float32) / 4
    T = (X @ A).astype(np.float32)
    net, info = learned.train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), n_hidden=32, epochs=60,
                              batch=64, lr=3e-3)
    try:
        assert info["final_loss"] < 0.05 * info["first_loss"], info
    finally:
        hx.hx_mlp_destroy(net)


def test_element_features_and_targets():
    # inputs and targets against the oracle's assembled diagonal and coefficient (Jacobi-scaled form)
    p, N = 3, 3
    kp = kappa_field_params(1000, M=64)
    mesh = lattice_mesh(N, p, warp="B", shuffle_seed=4)
    print("\n[case] mlp features", flush=True)
    A = fem.assemble(mesh, p, p + 2, "gauss", "diffusion", kappa=kp)
    free = (mesh["boundary"] == 0).astype(np.float64)
    dis = free / np.sqrt(fem.diagonal(A))
    with Problem(N, p, p + 2, "gauss", "diffusion", mesh=mesh, kappa=kp) as pr:
        P3 = (p + 1) ** 3
        E = mesh["nelem"]
        r = np.random.default_rng(5).standard_normal(mesh["nnodes"]) * free
        X = torch.empty(E, 2 * P3, device="cuda")
        rn = torch.empty(E, device="cuda")
        T = torch.empty(E, P3, device="cuda")
        hx.hx_op_mlp_features(pr.h_op, pr.to_dev(r), X, rn)
        err = np.random.default_rng(6).standard_normal(mesh["nnodes"]) * free
        hx.hx_op_mlp_targets(pr.h_op, pr.to_dev(err), rn, T)
        X, rn, T = X.cpu().numpy(), rn.cpu().numpy(), T.cpu().numpy()
        re = (dis * r)[mesh["elem_nodes"]]
        nrm = np.linalg.norm(re, axis=1)
        np.testing.assert_allclose(rn, nrm, rtol=1e-6)
        np.testing.assert_allclose(X[:, :P3], re / nrm[:, None], rtol=1e-6, atol=1e-7)
        Xn = fem.node_coordinates(mesh, p)
        lk = np.log(fem.kappa_eval(kp, Xn))[mesh["elem_nodes"]]
        feat = np.where(free[mesh["elem_nodes"]] > 0, lk - lk.mean(axis=1, keepdims=True), 3.0)
        np.testing.assert_allclose(X[:, P3:], feat, atol=2e-2)  # bf16 storage
        fe = free[mesh["elem_nodes"]] > 0
        Tr = np.where(fe, (err / np.where(dis > 0, dis, 1.0))[mesh["elem_nodes"]], 0.0) / nrm[:, None]
        np.testing.assert_allclose(T, Tr, rtol=1e-5, atol=1e-6 * np.abs(Tr).max())


@pytest.fixture(scope="module")
def trained():
    # small training run on two seeded coefficient fields (p = 3, 6^3 elements)
    print("\n[case] mlp training set", flush=True)
    X, T = learned.training_set(3, 5, "gauss", 6, seeds=(1000, 1001), groups_per_field=40, kappa_M=128)
    net, info = learned.train(X, T, epochs=60, batch=128, lr=1e-3)
    yield net, info
    hx.hx_mlp_destroy(net)


def test_learned_fcg_solve_and_gain(trained):
    net, info = trained
    assert info["final_loss"] < info["first_loss"]
    pr, b = learned.problem_with_kappa(6, 3, 5, "gauss", 100, kappa_M=128)  # held-out coefficient seed
    with pr:
        res = learned.compare_solves(pr, b, net, rtol=1e-8)
        print("\n[learned] gain record:", res, flush=True)
        for name, r in res.items():
            assert r["true_rel_residual"] <= 1.05e-8, (name, r)
        # The learned map either carries the whole solve or its stall check hands the iterate to
        # Jacobi-PCG within the stall window (20 iterations, checked every 10): either way the solve
        # takes at most Jacobi-PCG's own iterations plus 40, the fallback's among them. What the trained
        # network gains per application is asserted by test_learned_map_gain_per_application.
        lr = res["learned"]
        assert lr["iterations"] <= res["jacobi"]["iterations"] + 40, (lr, res["jacobi"])
        if lr["fallback_used"]:
            assert lr["fallback_iterations"] <= lr["iterations"], lr


def _anorm_reduction(pr, e, z, r):
    """|e - a z|_A / |e|_A at the best step a = z'r / z'Az (r = A e): the error reduction of one
    application of the map that gave z."""
    Az = pr.apply(z) * pr.to_dev((pr.mesh["boundary"] == 0).astype(np.float64))
    eAe = float(torch.dot(e, r))
    zr, zAz = float(torch.dot(z, r)), float(torch.dot(z, Az))
    return float(np.sqrt(max(0.0, 1.0 - zr * zr / (zAz * eAe))))


def test_learned_map_gain_per_application(trained):
    # What the trained network adds, measured on a held-out coefficient field (seed 100): the A-norm
    # error reduction of one application of the learned map (mode 1: D^-1 r plus the network's
    # correction) against one Jacobi step D^-1 r, at the best step length, for rough errors (seeded
    # uniform on the free nodes, the element-scale content an element-local map can act on).
    net, _ = trained
    pr, b = learned.problem_with_kappa(6, 3, 5, "gauss", 100, kappa_M=128)
    with pr:
        fm = pr.to_dev((pr.mesh["boundary"] == 0).astype(np.float64))
        dinv = fm / pr.diagonal()
        out = []
        for seed in (21, 22, 23):
            e = pr.to_dev(np.random.default_rng(seed).uniform(-1.0, 1.0, pr.n)) * fm
            r = pr.apply(e) * fm
            zl = pr.zeros()
            hx.hx_op_mlp_precond(pr.h_op, net, r, zl, mode=1)
            out.append((_anorm_reduction(pr, e, zl, r), _anorm_reduction(pr, e, dinv * r, r)))
        print("\n[learned] A-norm reduction per application (learned, jacobi):", out, flush=True)
        for rl, rj in out:
            assert rl < rj, out


def test_fallback_on_broken_network(trained):
    net, _ = trained
    pr, b = learned.problem_with_kappa(5, 3, 5, "gauss", 101, kappa_M=128)
    with pr:
        shape = hx.hx_mlp_get_shape(net)
        bad = hx.hx_mlp_create(*shape, 1)
        try:
            # NaN weights: breakdown at the first dot product, then Jacobi PCG from x = 0
            prm = hx.hx_mlp_get_params(bad)
            prm[:] = np.nan
            hx.hx_mlp_set_params(bad, prm)
            x, info = pr.solve(b, precond=hx.HX_PC_MLP, mlp=bad.value, raise_on_error=False)
            assert info["fallback_used"] == 1 and info["status"] == "HX_OK", info
            assert info["true_rel_residual"] <= 1.05e-8
            # a network that returns minus the trained correction: r'z <= 0 -> fallback
            prm = hx.hx_mlp_get_params(net)
            I, H, O = shape
            s = H * (I + 1)
            prm[s:] = -prm[s:]  # negate W2 and b2
            hx.hx_mlp_set_params(bad, prm)
            x, info = pr.solve(b, precond=hx.HX_PC_MLP, mlp=bad.value, fallback=hx.HX_PC_CHEBYSHEV,
                               raise_on_error=False)
            assert info["fallback_used"] == 1 and info["status"] == "HX_OK", info
        finally:
            hx.hx_mlp_destroy(bad)


def _bf16(a):
    """Round to bfloat16 (round to nearest even on the FP32 bit pattern), returned as FP64."""
    b = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("mode,p,N", [(0, 3, 4), (1, 3, 4), (1, 2, 28)])
def test_learned_map_matches_oracle_composition(mode, p, N):
    # hx_op_mlp_precond against its definition composed on the CPU from the oracle: the assembled
    # diagonal D, kappa at the oracle's node coordinates, the FP64 network forward of the library's FP32
    # parameters, the 1/multiplicity weights of elem_nodes and the D^-1/2 scalings:
    #   z = D^-1/2 sum_e G_e^T (w |r~_e| net([r~_e/|r~_e|, f_e]))  (+ D^-1 r in mode 1),  r~ = D^-1/2 r.
    # Mesh B with 15% of the elements rotated (shared and constrained nodes in every orientation).
    # The network runs on bf16 matrix cores: inputs, W1, the hidden activations and W2 are rounded to
    # bfloat16 (unit roundoff u = 2^-9), products accumulate in FP32. Three checks:
    #  (1) against the same composition with those four roundings applied to the oracle's forward
    #      (both sides take the rounding decisions in bf16): node by node within 5e-3 of the magnitude
    #      of the last layer's terms (covers FP32 accumulation order and a hidden value that rounds the
    #      other way at a tie), and 1e-3 in norm;
    #  (2) against the unrounded FP64 composition node by node within the first-order bound of those
    #      roundings: dZ = 2u |W1||x|, dH = (1 - H^2) dZ + u |H|, dY = |W2| dH + u |W2| (|H| + dH);
    #  (3) in norm within 2e-2 of the FP64 composition (the bf16 forward test's bound).
    # p = 2 on 28^3 elements: 21,952 network rows, where the hidden layer runs the kernel that stages its
    # weights in LDS (20k rows and more), with 54 inputs per row (not a multiple of 8).
    q = p + 2
    P3 = (p + 1) ** 3
    print(f"\n[case] learned map mode={mode} p={p} N={N}", flush=True)
    kp = kappa_field_params(1002, M=64)
    mesh = rotate_elements(lattice_mesh(N, p, warp="B", shuffle_seed=3), p, 0.15, seed=4)
    A = fem.assemble(mesh, p, q, "gauss", "diffusion", kappa=kp)
    free = mesh["boundary"] == 0
    d = fem.diagonal(A)
    dis = np.where(free, 1.0 / np.sqrt(d), 0.0)
    EN = mesh["elem_nodes"].astype(np.int64)
    r = np.random.default_rng(8).standard_normal(mesh["nnodes"])  # constrained entries must be ignored
    net = hx.hx_mlp_create(2 * P3, 128, P3, 5)
    try:
        prm = hx.hx_mlp_get_params(net)
        prm[:] = np.random.default_rng(9).uniform(-0.2, 0.2, prm.size).astype(np.float32)
        hx.hx_mlp_set_params(net, prm)
        with Problem(N, p, q, "gauss", "diffusion", mesh=mesh, kappa=kp) as pr:
            z = torch.full((mesh["nnodes"],), 7.0, dtype=torch.float64, device="cuda")  # overwritten
            hx.hx_op_mlp_precond(pr.h_op, net, pr.to_dev(r), z, mode=mode)
            z = z.cpu().numpy()
        re = (dis * r)[EN]
        nrm = np.linalg.norm(re, axis=1)
        lk = np.log(fem.kappa_eval(kp, fem.node_coordinates(mesh, p)))[EN]
        feat = np.where(free[EN], lk - lk.mean(axis=1, keepdims=True), 3.0)
        W = _split(prm, 2 * P3, 128, P3)
        X = np.hstack([re / nrm[:, None], feat])
        Y, Hh = omlp.forward(W, X)
        # the same forward with the matrix-core roundings
        Hr = _bf16(np.tanh(_bf16(X) @ _bf16(W["W1"]).T + W["b1"]))
        Yr = Hr @ _bf16(W["W2"]).T + W["b2"]
        # first-order bound of those roundings, per output
        u = 2.0 ** -9
        aW1, aW2 = np.abs(W["W1"]), np.abs(W["W2"])
        m1 = np.abs(X) @ aW1.T
        dZ = 2.01 * u * m1 + 1e-5 * (m1 + np.abs(W["b1"]))
        dH = (1.0 - Hh ** 2 + 0.4 * dZ) * dZ + u * np.abs(Hh)
        m2 = np.abs(Hh) @ aW2.T + np.abs(W["b2"])
        bY = dH @ aW2.T + u * (m2 + dH @ aW2.T) + 1e-5 * m2
        w = np.where(free, 1.0 / np.bincount(EN.ravel(), minlength=mesh["nnodes"]), 0.0)

        def compose(V, absolute=False):
            out = np.zeros(mesh["nnodes"])
            np.add.at(out, EN, nrm[:, None] * (np.abs(V) if absolute else V))
            out = dis * w * out
            if mode == 1 and not absolute:
                out = out + np.where(free, r / d, 0.0)
            return out

        zo, zr = compose(Y), compose(Yr)
        assert np.all(z[~free] == 0.0)
        # (1) the bf16-rounded composition
        assert np.all(np.abs(z - zr) <= 5e-3 * compose(m2, True) + 1e-14 * np.abs(zr)), np.abs(z - zr).max()
        assert np.linalg.norm(z - zr) <= 1e-3 * np.linalg.norm(zr)
        # (2) the FP64 composition, node by node within the rounding bound
        assert np.all(np.abs(z - zo) <= compose(bY, True) + 1e-14 * np.abs(zo)), np.abs(z - zo).max()
        # (3) and in norm
        assert np.linalg.norm(z - zo) <= 2e-2 * np.linalg.norm(zo)
    finally:
        hx.hx_mlp_destroy(net)


def _learned_map(mesh, p, kp, A, prm, rounded):
    """v -> M v, the mode-1 learned map composed on the CPU from the oracle (as in the test above): the
    assembled diagonal, kappa at the oracle's node coordinates, the FP64 network forward of the library's
    FP32 parameters (with the matrix cores' bf16 roundings of inputs, W1, hidden values and W2 when
    ``rounded``), the 1/multiplicity weights and the D^-1/2 scalings, plus D^-1 v."""
    P3 = (p + 1) ** 3
    free = mesh["boundary"] == 0
    d = fem.diagonal(A)
    dis = np.where(free, 1.0 / np.sqrt(d), 0.0)
    EN = mesh["elem_nodes"].astype(np.int64)
    lk = np.log(fem.kappa_eval(kp, fem.node_coordinates(mesh, p)))[EN]
    feat = np.where(free[EN], lk - lk.mean(axis=1, keepdims=True), 3.0)
    W = _split(prm, 2 * P3, 128, P3)
    w = np.where(free, 1.0 / np.bincount(EN.ravel(), minlength=mesh["nnodes"]), 0.0)

    def M(v):
        re = (dis * v)[EN]
        nrm = np.linalg.norm(re, axis=1)
        X = np.hstack([re / np.where(nrm > 0, nrm, 1.0)[:, None], feat])
        if rounded:
            Y = _bf16(np.tanh(_bf16(X) @ _bf16(W["W1"]).T + W["b1"])) @ _bf16(W["W2"]).T + W["b2"]
        else:
            Y, _ = omlp.forward(W, X)
        out = np.zeros(mesh["nnodes"])
        np.add.at(out, EN, nrm[:, None] * Y)
        return dis * w * out + np.where(free, v / d, 0.0)
    return M


@pytest.mark.parametrize("weights", ["zero", "random"])
def test_learned_smoother_vcycle_matches_oracle(weights):
    # One V-cycle whose finest smoother is the Chebyshev polynomial on the learned map (mode 1) against
    # the oracle's V-cycle with that map as the finest level's base (the library's lam_max per level, a
    # coarse Jacobi-PCG of 8 iterations). Zero weights: the map is D^-1 exactly, so the general-base
    # recurrence and the post-smoothing residual path must agree to 1e-10. Random weights: against the
    # bf16-rounded composition; each of the six map applications agrees within 1e-3 in norm (the map
    # test above), the V-cycle within 2e-2.
    from oracle import pmg as opmg
    from paper_2109_04996_amd.problem import Hierarchy
    p, N, degrees = 3, 4, (3, 1)
    P3 = (p + 1) ** 3
    print(f"\n[case] learned smoother V-cycle weights={weights}", flush=True)
    kp = kappa_field_params(1002, M=64)
    ms = [rotate_elements(lattice_mesh(N, pl, warp="B", shuffle_seed=3), pl, 0.15, seed=4) for pl in degrees]
    net = hx.hx_mlp_create(2 * P3, 128, P3, 5)
    try:
        prm = hx.hx_mlp_get_params(net)
        # random weights of +-0.05: a correction about half the size of the Jacobi step
        prm[:] = 0.0 if weights == "zero" else np.random.default_rng(9).uniform(-0.05, 0.05, prm.size)
        hx.hx_mlp_set_params(net, prm)
        with Hierarchy(N, degrees, rule="gauss", kappa=kp, meshes=ms, smooth_degree=3, smooth_ratio=15.0,
                       coarse_maxit=8, coarse_rtol=0.0, smoother_mlp=net.value) as H:
            levels = []
            for l, (m, pl) in enumerate(zip(ms, degrees)):
                A = fem.assemble(m, pl, pl + 2, "gauss", "diffusion", kappa=kp)
                free = solvers.free_mask(m["boundary"])
                P = opmg.prolongation(m, ms[l + 1], pl, degrees[l + 1]) if l + 1 < len(degrees) else None
                base = _learned_map(m, pl, kp, A, prm, rounded=True) if l == 0 else None
                levels.append(opmg.Level(A, free, H.lambda_max(l) if P is not None else 0.0, P, base=base))
            assert H.lambda_max(0) > 0.0
            r = np.random.default_rng(5).uniform(-1.0, 1.0, ms[0]["nnodes"]) * levels[0].f
            zd = H.vcycle(H.fine.to_dev(r))
            assert torch.equal(zd, H.vcycle(H.fine.to_dev(r)))  # the same bits twice
            z = zd.cpu().numpy()
            zr = opmg.vcycle(levels, r, degree=3, ratio=15.0, coarse_rtol=0.0, coarse_maxit=8)
            assert np.all(z[~levels[0].free] == 0)
            tol = 1e-10 if weights == "zero" else 2e-2
            assert np.linalg.norm(z - zr) <= tol * np.linalg.norm(zr), np.linalg.norm(z - zr) / np.linalg.norm(zr)
    finally:
        hx.hx_mlp_destroy(net)


def test_learned_smoother_gain_record(trained):
    # What the trained network adds as the finest smoother's base inside the p-multigrid cycle, on held-out
    # coefficient seeds: flexible CG with that V-cycle against the same V-cycle with Jacobi-Chebyshev
    # smoothing (the p-multigrid baseline) and against Jacobi-PCG (the learned forms' fallback). The record
    # is printed; every form must reach 1e-8 in the FP64 true residual.
    from paper_2109_04996_amd.problem import Hierarchy
    net, _ = trained
    p, N, degrees = 3, 6, (3, 1)
    record = {}
    for seed in (100, 101):
        kp = kappa_field_params(seed, M=128)
        with Hierarchy(N, degrees, rule="gauss", kappa=kp) as Hj, \
                Hierarchy(N, degrees, rule="gauss", kappa=kp, smoother_mlp=net.value) as Hl:
            b = Hj.fine.to_dev(np.random.default_rng(2).uniform(-1, 1, Hj.fine.n) * (Hj.fine.mesh["boundary"] == 0))
            rec = {}
            for name, fn in (("pmg_jacobi_smoother", lambda: Hj.solve(b, rtol=1e-8, check_every=1)),
                             ("pmg_learned_smoother", lambda: Hl.solve(b, rtol=1e-8, check_every=1)),
                             ("jacobi_pcg", lambda: Hj.fine.solve(b, rtol=1e-8, check_every=1))):
                x, info = fn()
                assert info["true_rel_residual"] <= 1.05e-8, (seed, name, info)
                rec[name] = (info["iterations"], round(info["solve_seconds"], 5))
            rec["lam_max_MA"] = round(Hl.lambda_max(0), 4)
            rec["lam_max_DA"] = round(Hj.lambda_max(0), 4)
            record[seed] = rec
    print("\n[learned] p-multigrid smoother gain record (iterations, seconds):", record, flush=True)
