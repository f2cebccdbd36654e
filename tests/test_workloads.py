"""Seeded synthetic inputs: determinism, shapes and ranges of the workload generators (CPU only)."""
import numpy as np

from paper_2212_09807_amd import workloads as W


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a.columns(), b.columns()))


def test_cfg1_shape_and_determinism():
    a, b = W.make_workload(1).events[0], W.make_workload(1).events[0]
    assert a.n == 200 and _same(a, b)
    p0 = np.c_[a.x0, a.y0, a.z0].astype(float)
    p1 = np.c_[a.x1, a.y1, a.z1].astype(float)
    assert np.linalg.norm(p1[-1] - p0[0]) >= 30.0 - 1e-4
    hi = np.array([70 * W.PITCH_CM, 70 * W.PITCH_CM, 30.0]) + 1e-4
    assert np.all(p0 >= -1e-4) and np.all(p0 <= hi) and np.all(p1 <= hi)
    assert np.all(a.energy > 0)


def test_cfg2_shape():
    e = W.make_workload(2).events[0]
    assert e.n == 20000
    for c in (e.x0, e.x1, e.y0, e.y1):
        assert c.min() >= -1e-4 and c.max() <= 140 * W.PITCH_CM + 1e-4
    assert e.z0.min() >= -1e-4 and e.z0.max() <= 50.0 + 1e-4


def test_spill_sizes():
    s = W.spill_sizes(np.random.default_rng(0), 64)
    assert s.shape == (64,) and s.min() >= 500 and s.max() <= 200000


def test_table_shapes():
    for k, shape in ((1, (200, 10, 10)), (2, (1950, 45, 45))):
        w = W.config(k)
        t = W.response_table(w.table, w.readout, w.physics.v_drift)
        assert t.shape == shape and t.dtype == np.float32 and t.flags.c_contiguous


def test_large_spill_tiles_and_halo():
    rng = np.random.default_rng(5)
    tiles, ids = W.large_spill(rng, n_segments=20000)
    assert len(tiles) == W.TILES_X * W.TILES_Y == len(ids)
    total = sum(t.n for t in tiles)
    assert total >= 20000                      # halo segments are replicated to neighbouring tiles
    for t in tiles:
        if t.n:
            mx = 0.5 * (t.x0.astype(float) + t.x1)
            assert mx.min() >= -2.4 - 1e-3 and mx.max() <= W.MODULE_W + 2.4 + 1e-3


def test_bench_refuses_more_than_one_gpu():
    import subprocess, sys, os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
