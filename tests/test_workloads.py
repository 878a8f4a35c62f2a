"""Seeded input generators: shapes, determinism and motif-set sizes."""
import numpy as np

from paper_2507_14813_amd import workloads as W


def test_motif_set_sizes():
    assert len(W.enumerate_motifs(3, 3)) == 36
    assert len(W.enumerate_motifs(3, 4)) == 60
    assert len(W.enumerate_motifs(4, 4)) == 696
    assert len(W.enumerate_motifs(3, 4, connected=False)) == 74
    assert len(W.enumerate_motifs(4, 4, connected=False)) == 868
    for m in W.enumerate_motifs(4, 4):
        assert m[0] == (0, 1) and all(u != v for u, v in m)


def test_random_motifs_distinct_and_bounded():
    ms = W.random_extension_motifs(16, (5,), 5, 53)
    assert len(ms) == len(set(ms)) == 16
    for m in ms:
        assert len(m) == 5 and max(max(e) for e in m) < 5


def test_generators_deterministic_and_valid():
    a = W.powerlaw_graph(2000, 30000, 2.1, 10 ** 6, seed=9)
    b = W.powerlaw_graph(2000, 30000, 2.1, 10 ** 6, seed=9)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    s, d, t = a
    assert (s != d).all() and (np.diff(t) >= 0).all()
    assert t.min() >= 0 and t.max() < 10 ** 6
    deg = np.bincount(s, minlength=2000)
    assert deg.max() > 20 * deg.mean()            # heavy tail
    s, d, t = W.uniform_graph(50, 1000, 100, seed=1)
    assert (s != d).all() and (np.diff(t) >= 0).all() and s.max() < 50


def test_config_shapes_small():
    for k in (1, 2, 4, 5):
        wl = W.make_config(k, scale=0.0005 if k > 1 else 1.0)
        assert len(wl.graphs) == 1
        s, d, t, n = wl.graphs[0]
        assert len(s) == len(d) == len(t) and s.max() < n
    wl = W.make_config(1)
    assert len(wl.graphs[0][0]) == 20000 and wl.deltas == [10000]
    wl = W.make_config(5, scale=0.0001)
    assert wl.deltas == [900, 3600, 21600] and len(wl.motif_sets[0]) == 48
