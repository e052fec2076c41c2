"""GPU tests of the row-compressed element restriction (one id per r1-row of each element).

A lattice mesh whose L-nodes are relabelled by a seeded permutation of whole x-rows keeps every
element's r1-rows as runs of consecutive ids but has no element-wise affine numbering, so the
fused kernels read one base id per row (index mode 1). Each kernel family that has this path (the
collocated strip kernel, the Gauss-point strip kernel, the one-element collocated kernel with its
E-vector output) is compared with the FP64 oracle's assembled operator on such a mesh.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fem, solvers  # noqa: E402
from paper_2109_04996_amd.inputs import lattice_mesh, renumber_rows, uniform_vector  # noqa: E402
from paper_2109_04996_amd.problem import Problem  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("kind,rule,p,q,strips", [("diffusion", "gll", 7, 8, True), ("mass", "gauss", 7, 9, True),
                                                  ("diffusion", "gauss", 6, 8, True),
                                                  ("diffusion", "gauss", 7, 8, True),
                                                  ("diffusion", "gll", 4, 5, False),
                                                  ("diffusion", "gll", 5, 6, False),
                                                  ("diffusion", "gauss", 4, 6, False)])
@pytest.mark.parametrize("ncomp", [1, 3])
def test_row_compressed_apply_matches_oracle(ncomp, kind, rule, p, q, strips):
    N = 4
    print(f"\n[case] rows N={N} p={p} q={q} {rule} {kind} ncomp={ncomp}", flush=True)
    mesh = renumber_rows(lattice_mesh(N, p, warp="B", shuffle_seed=6), seed=17)
    A = fem.assemble(mesh, p, q, rule, kind)
    with Problem(N, p, q, rule, kind, ncomp=ncomp, mesh=mesh) as pr:
        assert pr.stats["index_mode"] == 1
        if strips:  # the strip kernels run (degree 7 builds strips on any lattice)
            assert pr.stats["nstrips"] > 0
        x = uniform_vector(mesh["nnodes"], 1, ncomp)
        yr = fem.apply(A, x, ncomp)
        y = pr.apply(pr.to_dev(x)).cpu().numpy()
        assert rel(y, yr) <= 1e-12
        assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()
        # a second call gives the same bits
        assert np.array_equal(pr.apply(pr.to_dev(x)).cpu().numpy(), y)
        # FP32 vectors with FP32 geometric factors through the same index path (the FP32 bound of
        # the lattice-numbered parity tests: ~100 roundings of 2^-24)
        y32 = pr.apply_f32(pr.to_dev(x, torch.float32), qdata_prec=1).double().cpu().numpy()
        assert rel(y32, fem.apply(A, x.astype(np.float32).astype(np.float64), ncomp)) <= 6e-6


@pytest.mark.parametrize("p,q", [(7, 8), (4, 5)])
def test_row_compressed_element_vectors(p, q):
    # the E-vector output (no scatter) reads the rows too: element by element against A_e x_e
    N = 3
    mesh = renumber_rows(lattice_mesh(N, p, warp="B", shuffle_seed=1), seed=3)
    x = uniform_vector(mesh["nnodes"], 4)
    ref = fem.element_apply(mesh, p, q, "gll", "diffusion", x, np.arange(mesh["nelem"]))
    with Problem(N, p, q, "gll", "diffusion", mesh=mesh) as pr:
        assert pr.stats["index_mode"] == 1
        ye = pr.apply_elem(pr.to_dev(x)).cpu().numpy()
        assert rel(ye, ref) <= 1e-12
        assert np.abs(ye - ref).max() <= 1e-12 * np.abs(ref).max()


def test_row_compressed_strips_at_degree_4_large_mesh():
    # collocated strips below degree 7 run only when a color averages >= 512 strips (N = 32 at p = 4):
    # too large for the assembled oracle, so the strip scatter is checked against the E-vector path
    # (one-element kernel, no scatter; itself pinned above) summed node by node
    N, p = 32, 4
    mesh = renumber_rows(lattice_mesh(N, p, warp="A", shuffle_seed=0), seed=5)
    with Problem(N, p, p + 1, "gll", "diffusion", mesh=mesh) as pr:
        assert pr.stats["index_mode"] == 1 and pr.stats["nstrips"] >= 512 * pr.stats["nstrip_colors"]
        x = pr.to_dev(uniform_vector(mesh["nnodes"], 1))
        y = pr.apply(x).cpu().numpy()
        ye = pr.apply_elem(x).cpu().numpy()
    ys = np.zeros(mesh["nnodes"])
    np.add.at(ys, mesh["elem_nodes"], ye[:, 0, :])
    assert rel(y, ys) <= 1e-13


def test_row_compressed_solve():
    # Jacobi-PCG on the renumbered mesh reaches the oracle's direct solution
    N, p, q = 3, 7, 8
    mesh = renumber_rows(lattice_mesh(N, p, warp="A", shuffle_seed=2), seed=9)
    A = fem.assemble(mesh, p, q, "gll", "diffusion")
    free = solvers.free_mask(mesh["boundary"])
    b = uniform_vector(mesh["nnodes"], 2) * free
    xd = solvers.direct_solve(A, b, free)
    with Problem(N, p, q, "gll", "diffusion", mesh=mesh) as pr:
        x, info = pr.solve(pr.to_dev(b), rtol=1e-12)
        assert rel(x.cpu().numpy(), xd) <= 1e-9, info
