"""GPU tests of the strip scatter (collocated diffusion at every degree p >= 2, scalar Gauss-point mass at
p = 7, scalar Gauss diffusion with q = 8 at p = 6, 7).

The strip kernels scatter chains of face-adjacent elements together. Their results are checked
against the FP64 oracle on meshes whose elements have random proper rotations (so chains break
and strips of every length from 1 to 8 occur), and at the full benchmark size against the
E-vector path (element kernel, no scatter) summed node by node. The 3-component Gauss cases of the
same meshes run the joint-component kernel instead (element colors) and are checked the same way,
on the oracle's meshes and at the 3-component benchmark size.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fem  # noqa: E402
from paper_2109_04996_amd.inputs import lattice_mesh, rotate_elements, uniform_vector  # noqa: E402
from paper_2109_04996_amd.problem import Problem  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("p,N,nstrips", [(7, 4, 16), (4, 4, 16), (2, 4, 16), (3, 4, 16), (6, 4, 16), (4, 9, 162),
                                         (2, 9, 162), (1, 4, 0), (5, 4, 0), (8, 4, 0)])
def test_strip_counts(p, N, nstrips):
    # chains of N elements along r1, cut into strips of 8 (7 at p = 2); strips at p = 2, 3, 4, 6 and 7 only
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=3)
    with Problem(N, p, p + 1, "gll", "diffusion", mesh=mesh) as pr:
        assert pr.stats["nstrips"] == nstrips
        if nstrips:
            assert pr.stats["nstrip_colors"] >= 2
            # whole strips packed into groups of at most 8 (7 at p = 2) elements
            sl = 7 if p == 2 else 8
            assert -(-mesh["nelem"] // sl) <= pr.stats["nstrip_groups"] <= nstrips


@pytest.mark.parametrize("kind,rule,p,q", [("diffusion", "gll", 7, 8), ("mass", "gauss", 7, 9),
                                           ("diffusion", "gll", 4, 5), ("diffusion", "gll", 2, 3),
                                           ("diffusion", "gauss", 6, 8), ("diffusion", "gauss", 7, 8),
                                           ("diffusion", "gauss", 7, 9), ("diffusion", "gauss", 4, 6),
                                           ("mass", "gauss", 6, 8)])
@pytest.mark.parametrize("ncomp", [1, 3])
def test_strip_apply_rotated_elements_matches_oracle(ncomp, kind, rule, p, q):
    N = 4 if p > 2 else 6
    print(f"\n[case] strips rotated N={N} p={p} q={q} {kind} ncomp={ncomp}", flush=True)
    mesh = rotate_elements(lattice_mesh(N, p, warp="B", shuffle_seed=5), p, 0.15, seed=ncomp)
    A = fem.assemble(mesh, p, q, rule, kind)
    with Problem(N, p, q, rule, kind, ncomp=ncomp, mesh=mesh) as pr:
        assert 0 < pr.stats["nstrips"] < mesh["nelem"]
        # short chains: workgroups hold several whole strips
        assert 0 < pr.stats["nstrip_groups"] < pr.stats["nstrips"]
        x = uniform_vector(mesh["nnodes"], 7, ncomp)
        y = pr.apply(pr.to_dev(x)).cpu().numpy()
        yr = fem.apply(A, x, ncomp)
        assert rel(y, yr) <= 1e-12, rel(y, yr)
        absax = fem.apply(abs(A), np.abs(x), ncomp)
        assert np.max(np.abs(y - yr)) <= 1e-12 * absax.max()
        if ncomp == 1:
            # FP32 operator with FP64 and with FP32 geometric factors through the same strips
            from paper_2109_04996_amd import hexpa as hx
            yr32 = fem.apply(A, x.astype(np.float32).astype(np.float64), ncomp)
            for qp in (hx.HX_FP64, hx.HX_FP32):
                y32 = pr.apply_f32(pr.to_dev(x, torch.float32), qp).double().cpu().numpy()
                assert rel(y32, yr32) <= 6e-6


def _scatter_evector(pr, ye):
    """sum_e G_e^T y_e on the device (torch index_add_ over the caller's element nodes)."""
    idx = torch.from_numpy(pr.mesh["elem_nodes"].astype(np.int64)).cuda().view(-1)
    y = torch.zeros(pr.n, dtype=torch.float64, device="cuda")
    y.index_add_(0, idx, ye.reshape(-1))
    return y


@pytest.mark.parametrize("kind,rule,p,q", [("diffusion", "gll", 7, 8), ("mass", "gauss", 7, 9),
                                           ("diffusion", "gll", 4, 5), ("diffusion", "gll", 2, 3),
                                           ("diffusion", "gauss", 6, 8)])
@pytest.mark.parametrize("N,frac", [(9, 0.0), (9, 0.2), (48, 0.0), (48, 0.2)])
def test_strip_apply_matches_evector_sum(N, frac, kind, rule, p, q):
    # N = 9: chains of 9 cut into 8 + 1 (7 + 2 at p = 2); N = 48: the benchmark mesh. Below p = 7
    # the strip kernel runs only when a color has 512 strips on average (else the element kernel):
    # at N = 48, with and without rotated elements
    print(f"\n[case] strips vs E-vector N={N} frac={frac} {kind} q={q}", flush=True)
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
    if frac > 0:
        mesh = rotate_elements(mesh, p, frac, seed=11)
    with Problem(N, p, q, rule, kind, mesh=mesh) as pr:
        assert pr.stats["nstrips"] > 0
        x = pr.to_dev(uniform_vector(mesh["nnodes"], 1))
        y = pr.apply(x)
        ye = pr.apply_elem(x)
        yref = _scatter_evector(pr, ye)
        err = float(torch.linalg.norm(y - yref) / torch.linalg.norm(yref))
        assert err <= 1e-13, err
        # the strip path is deterministic
        assert torch.equal(y, pr.apply(x))


def _scatter_evector_nc(pr, ye, nc):
    """sum_e G_e^T y_e for nc interleaved components (y_e of shape (E, nc, nodes per element))."""
    en = torch.from_numpy(pr.mesh["elem_nodes"].astype(np.int64)).cuda()
    y = torch.zeros(pr.mesh["nnodes"] * nc, dtype=torch.float64, device="cuda")
    for c in range(nc):
        y.index_add_(0, (en * nc + c).view(-1), ye[:, c, :].contiguous().view(-1))
    return y


@pytest.mark.parametrize("kind,p,q,N,frac", [("diffusion", 7, 9, 9, 0.0), ("diffusion", 7, 9, 40, 0.0),
                                             ("diffusion", 7, 9, 40, 0.2), ("mass", 7, 9, 9, 0.2),
                                             ("diffusion", 6, 8, 9, 0.0), ("diffusion", 4, 6, 9, 0.2),
                                             ("diffusion", 7, 8, 9, 0.0), ("mass", 6, 8, 9, 0.0)])
def test_joint_kernel_matches_evector_sum(kind, p, q, N, frac):
    # 3 components through the joint-component kernel on meshes with strips (which it does not use:
    # element colors); N = 40 is the 3-component benchmark mesh, with and without rotated elements
    print(f"\n[case] joint kernel vs E-vector N={N} frac={frac} {kind} p={p} q={q}", flush=True)
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
    if frac > 0:
        mesh = rotate_elements(mesh, p, frac, seed=11)
    with Problem(N, p, q, "gauss", kind, ncomp=3, mesh=mesh) as pr:
        assert pr.stats["nstrips"] > 0
        x = pr.to_dev(uniform_vector(mesh["nnodes"], 1, 3))
        y = pr.apply(x)
        ye = pr.apply_elem(x)
        assert ye.shape == (mesh["nelem"], 3, (p + 1) ** 3)
        yref = _scatter_evector_nc(pr, ye, 3)
        err = float(torch.linalg.norm(y - yref) / torch.linalg.norm(yref))
        assert err <= 1e-13, err
        assert torch.equal(y, pr.apply(x))
        # FP32 through the same strips
        x32 = x.float()
        y32 = pr.apply_f32(x32).double()
        yref32 = _scatter_evector_nc(pr, pr.apply_elem(x32.double()), 3)
        assert float(torch.linalg.norm(y32 - yref32) / torch.linalg.norm(yref32)) <= 6e-6


@pytest.mark.parametrize("kind,rule,q,N,ncomp,rot", [("diffusion", "gll", 8, 48, 1, 0.0), ("mass", "gauss", 9, 48, 1, 0.0),
                                                      ("diffusion", "gauss", 9, 40, 3, 0.0),
                                                      ("diffusion", "gll", 8, 48, 3, 0.0),
                                                      ("diffusion", "gll", 8, 48, 1, 0.2)])
def test_full_size_sampled_nodes_match_oracle(kind, rule, q, N, ncomp, rot):
    """The benchmark workloads (mesh A, N^3 elements shuffled with seed 0, x ~ U[-1,1] from seed 1:
    BP5 at 48^3, 38.3M DOFs; the 3-component BP4 line at 40^3, 3 x 22.2M DOFs; BP6 at 48^3; BP5 on
    the same mesh with 20% of its elements rotated, seed 5, the full-index path) through the launches
    the benchmark times, checked against the oracle at every node of 16 seeded elements: interior,
    face, edge and corner nodes, strip ends among them. Each reference value sums the oracle's dense
    element matrices of all elements holding the node (per component: the vector operators act on
    each component alone)."""
    p = 7
    print(f"\n[case] full size N={N} p={p} q={q} {kind} ncomp={ncomp} rotated {rot} sampled nodes", flush=True)
    mesh = lattice_mesh(N, p, warp="A", shuffle_seed=0)
    if rot > 0:
        mesh = rotate_elements(mesh, p, rot, seed=5)
    en = mesh["elem_nodes"]
    x = uniform_vector(mesh["nnodes"], 1, ncomp)
    with Problem(N, p, q, rule, kind, ncomp=ncomp, mesh=mesh) as pr:
        if rot > 0:
            assert pr.stats["index_mode"] == 0 and pr.stats["nstrips"] > 0
        else:
            assert pr.stats["nstrips"] == N * N * (-(-N // 8)) and pr.stats["nstrip_colors"] == 8
        y = pr.apply(pr.to_dev(x)).cpu().numpy()
    rng = np.random.default_rng(5)
    sel = rng.choice(mesh["nelem"], 16, replace=False)
    targets = np.unique(en[sel].ravel())
    touch = np.flatnonzero(np.isin(en, targets).any(axis=1))
    Ae = fem.element_matrices(mesh, p, q, rule, kind, None, touch)
    xv = x.reshape(mesh["nnodes"], ncomp)
    yv = y.reshape(mesh["nnodes"], ncomp)
    for c in range(ncomp):
        xe = xv[en[touch].astype(np.int64), c]
        yref = np.zeros(mesh["nnodes"])
        babs = np.zeros(mesh["nnodes"])
        np.add.at(yref, en[touch].ravel(), np.einsum("eij,ej->ei", Ae, xe).ravel())
        np.add.at(babs, en[touch].ravel(), np.einsum("eij,ej->ei", np.abs(Ae), np.abs(xe)).ravel())
        err = rel(yv[targets, c], yref[targets])
        assert err <= 1e-12, (c, err)
        assert np.max(np.abs(yv[targets, c] - yref[targets])) <= 1e-12 * babs[targets].max()
