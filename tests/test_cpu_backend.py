"""The CPU backend (generated nested loops per trie level, or the interpreted
trie) against the oracle on host-only graphs, and the paper's co-mining
heuristic.  Runs without a GPU."""
import numpy as np
import pytest

from paper_2507_14813_amd import api, workloads as W
from oracle import OracleGraph
from conftest import tiny_graph

BIG = 10 ** 12


def oracle_counts(og, motifs, delta, roots=None):
    return np.array([og.count(m, delta, roots=roots) for m in motifs], dtype=np.uint64)


def _motifs(seed):
    ms = []
    for k in (1, 2, 3):
        ms += W.enumerate_motifs(k, 2 * k, connected=False)
    rng = np.random.default_rng(seed)
    four = W.enumerate_motifs(4, 5, connected=False)
    five = W.enumerate_motifs(5, 6, connected=False)
    return ms + [four[i] for i in rng.choice(len(four), 20, replace=False)] + \
        [five[i] for i in rng.choice(len(five), 20, replace=False)]


@pytest.mark.parametrize("codegen", [True, False])
def test_cpu_backend_tiny_graphs(codegen):
    rng = np.random.default_rng(31)
    for rep in range(3):
        n = int(rng.integers(3, 8))
        s, d, t = tiny_graph(rng, n, int(rng.integers(8, 16)), 10, self_loops=rep == 1)
        perm = rng.permutation(len(s))
        s, d, t = s[perm], d[perm], t[perm]
        og = OracleGraph(s, d, t, n)
        g = api.Graph(s, d, t, n, host_only=True)
        ms = _motifs(rep)
        for delta in (0, 3, BIG):
            want = oracle_counts(og, ms, delta)
            assert np.array_equal(api.count_cpu(g, api.Tree(ms, delta), codegen=codegen), want)


def test_cpu_backend_medium_modes_windows_roots():
    rng = np.random.default_rng(5)
    s, d, t = tiny_graph(rng, 40, 5000, 800, self_loops=True)
    ms = W.random_extension_motifs(25, (2, 3, 4, 5), 6, 3) + [[(0, 1), (2, 3), (1, 2)]]
    og = OracleGraph(s, d, t, 40)
    g = api.Graph(s, d, t, 40, host_only=True)
    windows = [9, 30, 0]
    want = np.stack([oracle_counts(og, ms, w) for w in windows])
    tr = api.Tree(ms, windows)
    for codegen in (True, False):
        for mode in ("comine", "per_motif"):
            got, ms_ = api.count_cpu(g, tr, mode=mode, codegen=codegen, timed=True)
            assert np.array_equal(got, want), (codegen, mode)
            assert ms_ >= 0
    roots = np.arange(2, len(s), 9)
    want_r = oracle_counts(og, ms, 30, roots)
    assert np.array_equal(api.count_cpu(g, api.Tree(ms, 30), roots=roots, threads=3), want_r)


def test_host_only_graph_refused_by_gpu_entry_points():
    s = np.array([0, 1, 2], np.int32)
    g = api.Graph(s, (s + 1) % 3, np.array([1, 2, 3]), 3, host_only=True)
    tr = api.Tree([[(0, 1), (1, 2)]], 5)
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        api.count(g, tr)
    assert api.count_cpu(g, tr).tolist() == [2]


def test_comining_heuristic():
    """Bipartite graphs always co-mine; on the GPU a group below SM 0.44
    does not; the CPU co-mines otherwise."""
    rng = np.random.default_rng(2)
    left = rng.integers(0, 50, 2000)
    right = rng.integers(50, 100, 2000)
    flip = rng.random(2000) < 0.5
    s = np.where(flip, left, right).astype(np.int32)
    d = np.where(flip, right, left).astype(np.int32)
    t = np.sort(rng.integers(0, 10000, 2000))
    bip = api.Graph(s, d, t, 100, host_only=True)
    low = api.Tree([[(0, 1), (1, 2), (2, 3)], [(0, 1), (2, 1), (3, 0)], [(0, 1), (0, 2)]], 50)
    assert low.info()["similarity"] < 0.44
    a = api.comine_advice(bip, low, "gpu")
    assert a["bipartite"] == 1 and a["co_mine"] == 1
    s2, d2, t2 = tiny_graph(rng, 30, 2000, 10000, self_loops=False)
    gen = api.Graph(s2, d2, t2, 30, host_only=True)
    a = api.comine_advice(gen, low, "gpu")
    assert a["bipartite"] == 0 and a["co_mine"] == 0 and a["threshold"] == pytest.approx(0.44)
    assert api.comine_advice(gen, low, "cpu")["co_mine"] == 1
    high = api.Tree(W.enumerate_motifs(3, 3), 50)
    assert api.comine_advice(gen, high, "gpu")["co_mine"] == 1
