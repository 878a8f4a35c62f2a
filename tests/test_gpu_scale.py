"""Parity at configuration scale: the benchmark graph's whole count vector
against the oracle, the large configurations on uniformly drawn roots and on
the heaviest roots of their cost logs, the 64-graph batch (plain and learned)
on every graph, windows long enough to reach the chunk limit of the search,
and a process that exits with live handles."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2507_14813_amd import api, workloads as W
from oracle import OracleGraph

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    api.lib()
    return torch


def oracle_counts(og, motifs, delta, roots=None):
    return np.array([og.count(m, delta, roots=roots) for m in motifs], dtype=np.uint64)


def sample_roots(rng, cost, n_uniform, n_heavy):
    """Roots drawn uniformly, plus roots drawn from the heaviest 1 % of the
    per-root cost log (where root splits and window hints act)."""
    E = len(cost)
    uni = rng.choice(E, min(E, n_uniform), replace=False)
    top = np.argsort(cost)[-max(1, E // 100):]
    heavy = rng.choice(top, min(len(top), n_heavy), replace=False)
    return np.unique(np.concatenate([uni, heavy]))


def test_config2_whole_count_vector():
    """The benchmark's graph (20M edges, 36 motifs), launched exactly as the
    benchmark launches it, against the oracle over every root edge."""
    wl = W.make_config(2)
    s, d, t, n = wl.graphs[0]
    ms, delta = wl.motif_sets[0], wl.deltas[0]
    say("config 2: GPU")
    g = api.Graph(s, d, t, n, sorted_by_t=True)
    tr = api.Tree(ms, delta)
    got = api.count(g, tr)
    say("config 2: oracle over every root")
    og = OracleGraph(s, d, t, n)
    want = oracle_counts(og, ms, delta)
    og.close()
    assert want.sum() > 10 ** 8
    assert np.array_equal(got, want)
    assert np.array_equal(api.count(g, tr, mode="per_motif"), want)


@pytest.mark.parametrize("k,scale", [(4, 1.0), (5, 0.25)])
def test_large_config_uniform_and_heavy_roots(k, scale):
    """Config 4 at full size (50M edges, 756 motifs) and config 5 at a quarter
    (50M edges, 48 motifs of 3-5 edges, its three windows in one search):
    uniformly drawn roots and roots from the heaviest 1 % against the oracle,
    the plain schedule and the learned one (the model's split of heavy roots
    included), co-mined and per motif."""
    wl = W.make_config(k, scale=scale)
    s, d, t, n = wl.graphs[0]
    ms = wl.motif_sets[0]
    windows = list(wl.deltas)
    E = len(s)
    say("config", k, "scale", scale, "E", E)
    g = api.Graph(s, d, t, n, sorted_by_t=True)
    tr = api.Tree(ms, windows if len(windows) > 1 else windows[0])
    _, cost = api.count(g, tr, root_cost=True)
    rng = np.random.default_rng(k)
    roots = sample_roots(rng, cost, 2048, 128)
    say("config", k, "oracle on", len(roots), "roots")
    og = OracleGraph(s, d, t, n)
    want = np.stack([oracle_counts(og, ms, w, roots) for w in windows])
    og.close()
    want = want if len(windows) > 1 else want[0]
    assert want.sum() > 0
    got = api.count(g, tr, roots=roots)
    assert np.array_equal(got, want)
    assert np.array_equal(api.count(g, tr, roots=roots, mode="per_motif"), want)
    # the learned schedule searches every root: its full counts equal the plain ones
    full = api.count(g, tr)
    model = api.Model(seed=7)
    live = np.flatnonzero(cost > 0)
    pick = rng.choice(live, min(len(live), 20000), replace=False)
    model.train(api.root_features(g, tr, roots=pick), np.log1p(cost[pick]).astype(np.float32),
                epochs=2, lr=2e-3, seed=1)
    say("config", k, "learned schedule")
    assert np.array_equal(api.count(g, tr, model=model), full)


def test_config3_batch_every_graph():
    """The 64-graph batch, plain (autotuned, captured) and learned: equal to
    each graph's own count, and each graph's count equal to the oracle on
    roots drawn from that graph."""
    wl = W.make_config(3)
    graphs = [api.Graph(s, d, t, n, sorted_by_t=True) for (s, d, t, n) in wl.graphs]
    trees = [api.Tree(ms, dl) for ms, dl in zip(wl.motif_sets, wl.deltas)]
    single = [api.count(g, tr) for g, tr in zip(graphs, trees)]
    rng = np.random.default_rng(3)
    for j, ((s, d, t, n), ms, dl) in enumerate(zip(wl.graphs, wl.motif_sets, wl.deltas)):
        roots = np.sort(rng.choice(len(s), min(len(s), 384), replace=False))
        og = OracleGraph(s, d, t, n)
        want = oracle_counts(og, ms, dl, roots)
        og.close()
        assert np.array_equal(api.count(graphs[j], trees[j], roots=roots), want), j
    say("config 3 batch plain")
    b = api.Batch(graphs, trees)
    for _ in range(2):
        for j, (a, w) in enumerate(zip(b.count(), single)):
            assert np.array_equal(a, w), j
    feats, labels = [], []
    for j in range(0, 64, 8):
        _, cost = api.count(graphs[j], trees[j], root_cost=True)
        live = np.flatnonzero(cost > 0)
        pick = rng.choice(live, min(len(live), 4000), replace=False)
        feats.append(api.root_features(graphs[j], trees[j], roots=pick))
        labels.append(np.log1p(cost[pick]).astype(np.float32))
    model = api.Model(seed=3)
    model.train(np.concatenate(feats), np.concatenate(labels), epochs=2, lr=2e-3, seed=2)
    say("config 3 batch learned")
    bl = api.Batch(graphs, trees, model=model)
    assert bl.info()["learned"] == 1 and bl.info()["predict_ms"] > 0
    for j, (a, w) in enumerate(zip(bl.count(), single)):
        assert np.array_equal(a, w), j


def test_windows_past_the_chunk_limit():
    """Whole-list windows of 68M entries (at least 2^26, so the search sums
    window lengths in 64 bits) from 34 roots in one 64-root batch (2.3e9
    candidates, more than one pass of at most 2^31 - 1 can hold)."""
    n_late, n_roots = 68_000_000, 34
    rng = np.random.default_rng(21)
    V = 1000
    E = n_roots + n_late
    s = rng.integers(0, V, E).astype(np.int32)
    d = ((s + 1 + rng.integers(0, V - 1, E)) % V).astype(np.int32)
    t = np.ones(E, np.int64)
    t[:n_roots] = 0
    ms = [[(0, 1), (2, 3)], [(0, 1)]]
    roots = np.arange(n_roots)
    say("chunk limit: GPU")
    g = api.Graph(s, d, t, V, sorted_by_t=True)
    tr = api.Tree(ms, 1)
    got = api.count(g, tr, roots=roots)
    say("chunk limit: oracle")
    og = OracleGraph(s, d, t, V)
    want = oracle_counts(og, ms, 1, roots)
    og.close()
    assert want[0] > 2 ** 31 and want[1] == n_roots
    assert np.array_equal(got, want)


def test_hub_root_windows_longer_than_16_bits():
    """A hub with 70,000 out-edges in one window: the root windows of its
    early edges in out(hub) have more than 65,533 entries, so deeper windows
    on that list keep only the root window's end (and search their start from
    the list's start).  Two- and three-edge motifs that reach out(hub) again
    below the root, in co-mining, per-motif and leaf-parent paths, one and
    two windows, against the oracle on the hub's first roots."""
    rng = np.random.default_rng(31)
    V, n_hub, n_rest = 1001, 70_000, 3_000
    hs = np.zeros(n_hub, np.int32)
    hd = rng.integers(1, V, n_hub).astype(np.int32)
    ht = np.arange(1, n_hub + 1, dtype=np.int64)
    rs = rng.integers(1, V, n_rest).astype(np.int32)
    rd = ((rs + rng.integers(1, V - 1, n_rest)) % (V - 1) + 1).astype(np.int32)
    rt = rng.integers(0, n_hub + 1, n_rest).astype(np.int64)
    s, d, t = np.concatenate([hs, rs]), np.concatenate([hd, rd]), np.concatenate([ht, rt])
    o = np.argsort(t, kind="stable")
    s, d, t = s[o], d[o], t[o]
    roots = np.flatnonzero(s == 0)[:6]
    roots = np.concatenate([roots, rng.choice(len(s), 6, replace=False)])
    ms = [[(0, 1), (0, 2), (2, 3)],      # sets the root's out(a) window (> 65,533 entries)
          [(0, 1), (1, 2), (0, 3)],      # reads out(a) again below the root
          [(0, 1), (1, 2), (0, 2)],
          [(0, 1), (2, 1), (0, 3)],
          [(0, 1), (1, 2)]]
    delta = 100_000
    g = api.Graph(s, d, t, V, sorted_by_t=True)
    og = OracleGraph(s, d, t, V)
    say("long hints: oracle")
    want = oracle_counts(og, ms, delta, roots)
    want2 = np.stack([oracle_counts(og, ms, 30_000, roots), want])
    og.close()
    assert want[1] > 0
    for mode in ("comine", "per_motif"):
        for ls in (0, 1):
            say("long hints:", mode, ls)
            got = api.count(g, api.Tree(ms, delta), roots=roots, mode=mode, leaf_scan=ls)
            assert np.array_equal(got, want), (mode, ls)
    assert np.array_equal(api.count(g, api.Tree(ms, [30_000, delta]), roots=roots), want2)


def test_exit_with_live_handles():
    """A process that leaves graphs, trees, a batch and a model open and exits
    ends cleanly (handles still alive at exit are left to the process end)."""
    code = (
        "import numpy as np, torch\n"
        "from paper_2507_14813_amd import api\n"
        "rng = np.random.default_rng(0)\n"
        "s = rng.integers(0, 50, 5000).astype(np.int32)\n"
        "d = ((s + 1 + rng.integers(0, 49, 5000)) % 50).astype(np.int32)\n"
        "t = np.sort(rng.integers(0, 10000, 5000))\n"
        "g = api.Graph(s, d, t, 50, sorted_by_t=True)\n"
        "tr = api.Tree([[(0, 1), (1, 2)], [(0, 1), (1, 0)]], 100)\n"
        "b = api.Batch([g, g], [tr, tr])\n"
        "m = api.Model(seed=1)\n"
        "c = api.count(g, tr)\n"
        "assert all(np.array_equal(x, c) for x in b.count())\n"
        "print('done', int(c.sum()), flush=True)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    assert r.stdout.startswith("done")
