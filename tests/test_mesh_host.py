"""Host logic of the mesh builder, on the CPU.

hx_mesh_plan runs the element coloring, internal order, ownership masks, index-mode detection and
strip construction of hx_mesh_create without a device. These tests recompute, with numpy, every
invariant the atomic-free scatter relies on (libCEED section: G^T adds each element's contribution
into the L-vector): no node twice in one launch, exactly one first writer per node in launch order,
strips whose members share only their r1 faces with their neighbours in the strip, and the index
modes the fused kernels read."""
import ctypes as C

import numpy as np
import pytest

from paper_2109_04996_amd import hexpa as hx
from paper_2109_04996_amd.inputs import lattice_mesh, renumber_rows, rotate_elements


def _plan(mesh, p):
    xyz = hx.hx_mesh_nodes_trilinear(p, mesh["elem_verts"], mesh["verts"], mesh["elem_nodes"], mesh["nnodes"])
    h = hx.hx_mesh_plan(p, mesh["elem_nodes"], xyz, mesh["boundary"])
    try:
        st = hx.hx_mesh_get_stats(h)
        order, cs = hx.hx_mesh_get_order(h, st["nelem"], st["ncolors"])
        arr = hx.hx_mesh_plan_arrays(h, p)
    finally:
        hx.hx_mesh_destroy(h)
    return st, order, cs, arr


def _launches_disjoint(idx, starts):
    """No node appears twice within one launch range [starts[c], starts[c+1]) of rows of idx."""
    for c in range(len(starts) - 1):
        nodes = idx[starts[c]:starts[c + 1]].ravel()
        if np.unique(nodes).size != nodes.size:
            return False
    return True


def _first_writers(nodes_in_order, positions):
    """Positions of the first occurrence of each node in a launch-ordered stream of (node, position)."""
    _, first = np.unique(nodes_in_order, return_index=True)
    return set(map(tuple, positions[first]))


def _own_positions(own, P):
    """(element, local node) pairs whose ownership bit is set: bit k of own[t][j*P+i] is node i+P(j+Pk)."""
    t, ij = np.nonzero(own)
    out = set()
    for a, b in zip(t, ij):
        bits = int(own[a, b])
        for k in range(P):
            if bits >> k & 1:
                out.add((int(a), int(b) + P * P * k))
    return out


def _strips(arr, st):
    """Strips as lists of internal element positions, in launch order, with their color."""
    out = []
    scs = arr["strip_color_start"]
    for c in range(st["nstrip_colors"]):
        for g in range(scs[c], scs[c + 1]):
            cur = []
            for w in range(8):
                e = int(arr["strip_elems"][g, w])
                if e < 0:
                    break
                cur.append(e)
                if not (int(arr["strip_link"][g]) >> w & 1):
                    out.append((c, cur))
                    cur = []
            assert not cur, "a strip group's link bits run past its last element"
    return out


CASES = [
    ("lattice N=6 p=7", lambda: lattice_mesh(6, 7, warp="A", shuffle_seed=0), 7, 2),
    ("lattice N=10 p=7 (strips of 8 and 2)", lambda: lattice_mesh(10, 7, warp="A", shuffle_seed=3), 7, 2),
    ("lattice N=9 p=2 (strips of 7)", lambda: lattice_mesh(9, 2, warp="A", shuffle_seed=1), 2, 2),
    ("lattice N=5 p=4 warp B", lambda: lattice_mesh(5, 4, warp="B", shuffle_seed=2), 4, 2),
    ("rows renumbered N=6 p=7", lambda: renumber_rows(lattice_mesh(6, 7, warp="A", shuffle_seed=0), 4), 7, 1),
    ("20% rotated N=8 p=7", lambda: rotate_elements(lattice_mesh(8, 7, warp="A", shuffle_seed=0), 7, 0.2, 5), 7, 0),
    ("15% rotated N=6 p=3 warp B", lambda: rotate_elements(lattice_mesh(6, 3, warp="B", shuffle_seed=0), 3, 0.15, 7), 3, 0),
    ("one element p=5", lambda: lattice_mesh(1, 5, warp="A", shuffle_seed=0), 5, 2),
] + [
    (f"lattice N=4 p={q}", (lambda q=q: lattice_mesh(4, q, warp="A", shuffle_seed=q)), q, 2) for q in (1, 3, 5, 6, 8)
] + [
    (f"25% rotated N=4 p={q} warp B", (lambda q=q: rotate_elements(lattice_mesh(4, q, warp="B", shuffle_seed=q), q,
                                                                    0.25, q)), q, 0) for q in (1, 2, 4, 7, 8)
]


@pytest.mark.parametrize("name,make,p,index_mode", CASES, ids=[c[0] for c in CASES])
def test_plan_invariants(name, make, p, index_mode):
    mesh = make()
    P = p + 1
    P3 = P ** 3
    E, n = mesh["nelem"], mesh["nnodes"]
    st, order, cs, arr = _plan(mesh, p)
    idx = arr["idx"]

    # internal order: a permutation, and idx is the caller's restriction in that order
    assert np.array_equal(np.sort(order), np.arange(E))
    assert np.array_equal(idx, mesh["elem_nodes"][order])
    assert st["nelem"] == E and st["nnodes"] == n
    assert st["nfree"] == int((mesh["boundary"] == 0).sum())
    assert st["nuntouched"] == n - np.unique(idx).size
    assert st["index_mode"] == index_mode

    # element colors: no node twice in one color's launch
    assert cs[0] == 0 and cs[-1] == E and np.all(np.diff(cs) > 0)
    assert _launches_disjoint(idx, cs)
    assert st["max_color"] == int(np.diff(cs).max())
    if E >= 8 and index_mode > 0 and "warp B" not in name:
        assert st["ncolors"] == 8  # a lattice of mesh A needs and gets 8 colors

    # ownership: exactly one owner per node, the first element (internal order, local order) listing it
    pos = np.stack(np.meshgrid(np.arange(E), np.arange(P3), indexing="ij"), axis=-1).reshape(-1, 2)
    assert _own_positions(arr["own"], P) == _first_writers(idx.ravel(), pos)

    if st["nstrips"] == 0:
        return
    strips = _strips(arr, st)
    assert len(strips) == st["nstrips"]
    assert arr["strip_link"].size == st["nstrip_groups"]
    members = np.concatenate([np.array(s) for _, s in strips])
    assert np.array_equal(np.sort(members), np.arange(E))  # every element in exactly one strip
    slen = 7 if P == 3 else 8
    sub = idx.reshape(E, P, P, P)  # [t][k][j][i]
    writers_nodes, writers_pos = [], []
    for c, s in strips:
        assert 1 <= len(s) <= slen
        for a, b in zip(s[:-1], s[1:]):
            # b follows a along r1: b's i = 0 face is a's i = p face, node by node
            assert np.array_equal(sub[b, :, :, 0], sub[a, :, :, p])
        for w, e in enumerate(s):
            loc = np.arange(P3) if w == 0 else np.flatnonzero(np.arange(P3) % P != 0)
            writers_nodes.append(idx[e, loc])
            writers_pos.append(np.stack([np.full(loc.size, e), loc], axis=1))
    # strip colors: distinct strips of one color share no node
    for c in range(st["nstrip_colors"]):
        nodes = [np.unique(idx[s].ravel()) for cc, s in strips if cc == c]
        allnodes = np.concatenate(nodes)
        assert np.unique(allnodes).size == allnodes.size, f"strips of color {c} share a node"
    # strip ownership: one owner per node, the first writer in launch order; a member w > 0 never
    # owns its i = 0 face (its predecessor writes the shared face)
    wn, wp = np.concatenate(writers_nodes), np.concatenate(writers_pos)
    assert _own_positions(arr["strip_own"], P) == _first_writers(wn, wp)
    assert np.unique(wn).size == n - st["nuntouched"]


def test_lattice_strip_counts():
    # 16^3 elements at p = 7: every r1 chain of 16 elements gives two strips of 8, in 8 colors of 64
    st, _, _, arr = _plan(lattice_mesh(16, 7, warp="A", shuffle_seed=0), 7)
    assert st["nstrips"] == 16 * 16 * 2 and st["nstrip_colors"] == 8 and st["nstrip_groups"] == st["nstrips"]
    assert np.array_equal(np.diff(arr["strip_color_start"]), np.full(8, 64))


def test_checks_catch_a_wrong_coloring():
    # the disjointness and ownership checks above fail on a plan with a planted mistake
    mesh = lattice_mesh(4, 3, warp="A", shuffle_seed=0)
    st, order, cs, arr = _plan(mesh, 3)
    merged = np.array([cs[0], cs[2]] + list(cs[3:]))  # two colors launched together
    assert _launches_disjoint(arr["idx"], cs) and not _launches_disjoint(arr["idx"], merged)
    strips = _strips(arr, st) if st["nstrips"] else []
    assert strips, "the 4^3 lattice at p = 3 has strips"
    c0 = [sorted(set(arr["idx"][s].ravel())) for c, s in strips if c == 0]
    c1 = [sorted(set(arr["idx"][s].ravel())) for c, s in strips if c == 1]
    joined = np.concatenate(c0 + c1)  # two strip colors launched together share nodes
    assert np.unique(joined).size < joined.size
    own = arr["own"].copy()
    own[0, 0] ^= 1  # drop (or add) one owner bit
    pos = np.stack(np.meshgrid(np.arange(st["nelem"]), np.arange(64), indexing="ij"), axis=-1).reshape(-1, 2)
    assert _own_positions(own, 4) != _first_writers(arr["idx"].ravel(), pos)


def test_plan_rejected_by_operator_creation():
    mesh = lattice_mesh(2, 2, warp="A", shuffle_seed=0)
    xyz = hx.hx_mesh_nodes_trilinear(2, mesh["elem_verts"], mesh["verts"], mesh["elem_nodes"], mesh["nnodes"])
    h = hx.hx_mesh_plan(2, mesh["elem_nodes"], xyz, None)
    b = hx.hx_basis_create(2, 3, hx.HX_GLL)
    try:
        out = C.c_void_p()
        code = hx.load().hx_op_create(h, b, hx.HX_DIFFUSION, 1, None, None, C.byref(out))
        assert code == hx.HX_EINVAL and not out.value
        assert "host-only plan" in hx.load().hx_last_error().decode()
        code = hx.load().hx_op_create_lor(h, None, None, C.byref(out))
        assert code == hx.HX_EINVAL and not out.value
    finally:
        hx.hx_basis_destroy(b)
        hx.hx_mesh_destroy(h)


def test_plan_rejects_bad_input():
    mesh = lattice_mesh(2, 2, warp="A", shuffle_seed=0)
    xyz = np.zeros((mesh["nnodes"], 3))
    bad = mesh["elem_nodes"].copy()
    bad[1, 3] = mesh["nnodes"]
    with pytest.raises(hx.HexpaError):
        hx.hx_mesh_plan(2, bad, xyz, None)
    twice = mesh["elem_nodes"].copy()
    twice[0, 1] = twice[0, 0]  # an element listing one node twice
    with pytest.raises(hx.HexpaError):
        hx.hx_mesh_plan(2, twice, xyz, None)


def test_benchmark_mesh_plan():
    # the BP5 p = 7 benchmark mesh (mesh A, 48^3 elements shuffled with seed 0, 38,272,753 nodes): 8
    # launches of 1,728 strips of 8 elements, the affine numbering, 8 element colors of 13,824, and
    # one owner per node under both orders (bit counts; the positions are checked on the small meshes)
    st, _, cs, arr = _plan(lattice_mesh(48, 7, warp="A", shuffle_seed=0), 7)
    assert (st["nstrips"], st["nstrip_colors"], st["nstrip_groups"], st["index_mode"]) == (13824, 8, 13824, 2)
    assert np.array_equal(np.diff(arr["strip_color_start"]), np.full(8, 1728))
    assert np.all(arr["strip_link"] == 0x7f) and np.all(arr["strip_elems"] >= 0)
    assert st["ncolors"] == 8 and np.array_equal(np.diff(cs), np.full(8, 13824))
    assert _launches_disjoint(arr["idx"], cs)
    for own in (arr["own"], arr["strip_own"]):
        assert int(np.unpackbits(own.view(np.uint8)).sum()) == st["nnodes"] == 38272753
