"""Host-side arithmetic of the benchmark: the kernel-window cell count it reports for the bubble
half (eq. (18)-(19): the cells whose extent overlaps the support [x - n, x + n], n = 1.5 d,
clipped to the lattice), checked against a brute-force count over every cell."""
import numpy as np

import bench
import workloads as W


def _brute(pos, d, shape, factor):
    total = 0
    for b in range(len(d)):
        n = factor * d[b]
        cells = 1
        for a, ext in enumerate(shape):
            c = np.arange(ext)
            cells *= int(np.count_nonzero((c + 0.5 > pos[a, b] - n) & (c - 0.5 < pos[a, b] + n)))
        total += cells
    return total


def test_window_cells_match_a_brute_force_count():
    rng = np.random.default_rng(3)
    shape = (20, 14, 30)
    pos = np.stack([rng.uniform(-1.0, s, 40) for s in shape])  # some windows cross the faces
    d = rng.uniform(0.5, 5.0, 40)
    assert bench.window_cells(pos, d, shape, 1.5) == _brute(pos, d, shape, 1.5)
    # a window that ends on a cell face does not take the cell beyond it
    assert bench.window_cells(np.array([[10.0], [7.0], [15.0]]), np.array([1.0]), shape, 1.5) == 27


def test_dense_column_windows_average_about_1273_cells():
    w = W.dense()
    per = bench.window_cells(w.pos, w.d, w.shape, 1.5) / w.nb
    assert 1250 < per < 1300
