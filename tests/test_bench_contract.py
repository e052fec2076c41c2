"""CPU tests of bench.py's contract: one GPU only, and the algorithmic byte count behind roofline.frac."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_bp5_bytes_per_dof():
    # BP5, p = 7, 48^3 elements: 337^3 nodes; per node x read and y written (16 B); per element 8^3
    # points of 6 FP64 factors and 8^3 int32 node ids
    p, N = 7, 48
    n, E = (p * N + 1) ** 3, N ** 3
    ab = bench.algorithmic_bytes(n, E, p + 1, p + 1)
    assert n == 38_272_753 and E == 110_592
    assert ab["xy"] == 16 * 38_272_753
    assert ab["qdata"] == 110_592 * 512 * 48
    assert ab["index"] == 110_592 * 512 * 4
    assert round(ab["total"] / n, 2) == 92.93
    # three interleaved components: vectors triple, the factors and ids do not
    ab3 = bench.algorithmic_bytes(n, E, p + 1, p + 1, ncomp=3)
    assert ab3["total"] - ab["total"] == 2 * ab["xy"]


def test_secondary_line_bytes_per_dof():
    # the bench line's other apply records, from the element and node counts alone
    # BP4: p = 7, q = 9 Gauss, 40^3 elements, 3 components; 9^3 points of 6 factors per element
    n4, E4 = (7 * 40 + 1) ** 3, 40 ** 3
    ab = bench.algorithmic_bytes(n4, E4, 8, 9, 6, 3)
    assert ab["total"] == 48 * n4 + 8 * 6 * 729 * E4 + 4 * 512 * E4 == 3_435_585_968
    assert round(ab["total"] / (3 * n4), 2) == 51.61
    # BP6: p = 7 collocated, 48^3 elements, 3 components
    n6, E6 = (7 * 48 + 1) ** 3, 48 ** 3
    assert round(bench.algorithmic_bytes(n6, E6, 8, 8, 6, 3)["total"] / (3 * n6), 2) == 41.64
    # fused Helmholtz alpha A + beta B: a seventh stored value per point (beta w detJ)
    assert round(bench.algorithmic_bytes(n6, E6, 8, 8, 7, 1)["total"] / n6, 2) == 104.77
