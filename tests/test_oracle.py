"""Pins of the CPU oracle to things other than itself: hand-worked examples,
brute force over the definition, closed forms, an independent triple
enumerator, invariants and metamorphic relations.  CPU only."""
import itertools

import numpy as np
import pytest

from oracle import brute
from paper_2507_14813_amd import workloads as W
from conftest import edges_of, tiny_graph

BIG = 10 ** 12


def test_golden_examples(oracle_mod, golden_examples):
    for ex in golden_examples:
        s, d, t, n = edges_of(ex)
        for c in ex["cases"]:
            m = [tuple(e) for e in c["motif"]]
            assert oracle_mod.count(s, d, t, n, m, c["delta"]) == c["count"], (ex["name"], c)
            assert brute.count(s, d, t, m, c["delta"]) == c["count"], (ex["name"], c)


def test_enumeration_oracle_pins(oracle_mod, golden_examples):
    """The brute-force enumeration lists exactly the hand-listed tuples of
    Example A, and on random tiny graphs (unsorted input, ties, self-loops)
    as many tuples as the C oracle counts, each one a match of the motif."""
    A = golden_examples[0]
    s, d, t, n = edges_of(A)
    for c in A["cases"]:
        if "matches" in c:
            m = [tuple(e) for e in c["motif"]]
            assert brute.matches(s, d, t, m, c["delta"]) == [tuple(x) for x in c["matches"]]
    rng = np.random.default_rng(77)
    for _ in range(4):
        nv = int(rng.integers(3, 6))
        s, d, t = tiny_graph(rng, nv, int(rng.integers(8, 13)), 9, self_loops=True)
        perm = rng.permutation(len(s))
        s, d, t = s[perm], d[perm], t[perm]
        for m in _tiny_motifs()[::7]:
            for delta in (0, 3, BIG):
                got = brute.matches(s, d, t, m, delta)
                assert len(got) == oracle_mod.count(s, d, t, nv, m, delta)
                for tup in got:
                    assert brute.is_match([(int(s[i]), int(d[i]), int(t[i])) for i in tup], m, delta)
                    assert all(t[a] < t[b] for a, b in zip(tup, tup[1:]))


def _tiny_motifs():
    ms = []
    for k in (1, 2, 3):
        ms += W.enumerate_motifs(k, 2 * k, connected=False)
    rng = np.random.default_rng(7)
    four = W.enumerate_motifs(4, 5, connected=False)
    ms += [four[i] for i in rng.choice(len(four), 25, replace=False)]
    return ms


@pytest.mark.parametrize("seed", range(6))
def test_oracle_equals_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    n_nodes = int(rng.integers(2, 7))
    s, d, t = tiny_graph(rng, n_nodes, int(rng.integers(6, 11)), 10,
                         self_loops=bool(seed % 2))
    for m in _tiny_motifs():
        for delta in (0, 1, 3, 5, BIG):
            want = brute.count(s, d, t, m, delta)
            got = oracle_mod.count(s, d, t, n_nodes, m, delta)
            assert got == want, (m, delta)


def test_single_edge_and_zero_window(oracle_mod):
    rng = np.random.default_rng(3)
    s, d, t = tiny_graph(rng, 30, 500, 200, self_loops=True)
    assert oracle_mod.count(s, d, t, 30, [(0, 1)], 5) == int((s != d).sum())
    for m in W.CONFIG1_MOTIFS + [((0, 1), (0, 1)), ((0, 1), (1, 0))]:
        assert oracle_mod.count(s, d, t, 30, m, 0) == 0


def _within(times_sorted, lo, hi):
    """number of times in (lo, hi] per query"""
    return (np.searchsorted(times_sorted, hi, side="right")
            - np.searchsorted(times_sorted, lo, side="right"))


@pytest.mark.parametrize("delta", [0, 3, 17, 1000])
def test_closed_forms_two_edges(oracle_mod, delta):
    rng = np.random.default_rng(11)
    s, d, t = tiny_graph(rng, 12, 800, 400)
    # repeated edge [(0,1),(0,1)]: per ordered pair, later times within delta
    want_rep = 0
    want_rec = 0
    by_pair = {}
    for a, b, x in zip(s.tolist(), d.tolist(), t.tolist()):
        by_pair.setdefault((a, b), []).append(x)
    by_pair = {k: np.sort(np.array(v)) for k, v in by_pair.items()}
    for (a, b), ts in by_pair.items():
        want_rep += int(_within(ts, ts, ts + delta).sum())
        back = by_pair.get((b, a))
        if back is not None:
            want_rec += int(_within(back, ts, ts + delta).sum())
    assert oracle_mod.count(s, d, t, 12, [(0, 1), (0, 1)], delta) == want_rep
    assert oracle_mod.count(s, d, t, 12, [(0, 1), (1, 0)], delta) == want_rec


@pytest.mark.parametrize("delta", [4, 25])
def test_partition_identity_three_edges(oracle_mod, delta):
    """The 36 three-edge motifs on <= 3 vertices partition all window triples
    on <= 3 vertices (each triple has exactly one first-appearance form)."""
    rng = np.random.default_rng(5)
    s, d, t = tiny_graph(rng, 7, 70, 60)
    o = np.lexsort((np.arange(len(t)), t))
    s, d, t = s[o], d[o], t[o]
    triples = 0
    for i, j, k in itertools.combinations(range(len(t)), 3):
        if not (t[i] < t[j] < t[k]) or t[k] - t[i] > delta:
            continue
        if len({s[i], d[i], s[j], d[j], s[k], d[k]}) <= 3:
            triples += 1
    got = sum(oracle_mod.count(s, d, t, 7, m, delta) for m in W.enumerate_motifs(3, 3))
    assert got == triples and triples > 0


def _medium():
    rng = np.random.default_rng(21)
    s, d, t = tiny_graph(rng, 15, 400, 300)
    motifs = list(W.CONFIG1_MOTIFS) + W.random_extension_motifs(12, (2, 3, 4), 5, 9)
    return s, d, t, 15, motifs, 20


def test_metamorphic_relations(oracle_mod):
    s, d, t, n, motifs, delta = _medium()
    base = [oracle_mod.count(s, d, t, n, m, delta) for m in motifs]
    assert sum(base) > 0
    perm = np.random.default_rng(1).permutation(n).astype(np.int32)
    rev = lambda m: [(v, u) for u, v in m]
    for i, m in enumerate(motifs):
        # relabel graph vertices
        assert oracle_mod.count(perm[s], perm[d], t, n, m, delta) == base[i]
        # shift time
        assert oracle_mod.count(s, d, t + 12345, n, m, delta) == base[i]
        # scale time and window together
        assert oracle_mod.count(s, d, 7 * t, n, m, 7 * delta) == base[i]
        # reverse time together with the motif's edge order
        assert oracle_mod.count(s, d, 1000 - t, n, list(m)[::-1], delta) == base[i]
        # reverse every edge of graph and motif
        assert oracle_mod.count(d, s, t, n, rev(m), delta) == base[i]
        # arbitrary motif labels
        lab = {x: 10 * x + 3 for e in m for x in e}
        assert oracle_mod.count(s, d, t, n, [(lab[u], lab[v]) for u, v in m],
                                delta) == base[i]


def test_window_monotone(oracle_mod):
    s, d, t, n, motifs, _ = _medium()
    for m in motifs:
        c = [oracle_mod.count(s, d, t, n, m, dl) for dl in (0, 5, 20, 80, BIG)]
        assert all(a <= b for a, b in zip(c, c[1:])), (m, c)


def test_per_root_and_level_logs(oracle_mod):
    s, d, t, n, motifs, delta = _medium()
    s = s.copy()
    s[::17] = d[::17]            # plant self-loops
    o = np.lexsort((np.arange(len(t)), t))
    for m in motifs:
        tot, pr, lv = oracle_mod.count(s, d, t, n, m, delta, per_root=True, level=True)
        assert int(pr.sum()) == tot
        assert np.array_equal(lv[:, -1], pr)
        assert np.array_equal(lv[:, 0], (s[o] != d[o]).astype(np.uint64))
        roots = np.arange(3, len(t), 5)
        assert oracle_mod.count(s, d, t, n, m, delta, roots=roots) == int(pr[roots].sum())
        assert brute.count(s[:40], d[:40], t[:40], m, delta, roots=[0, 5, 9]) == \
            oracle_mod.count(s[:40], d[:40], t[:40], n, m, delta, roots=[0, 5, 9])


@pytest.mark.parametrize("mutant", [1, 2, 3, 4])
def test_pins_catch_planted_mistakes(oracle_mod, golden_examples, mutant):
    """Each planted mistake (non-strict order, no injectivity for new
    vertices, exclusive window, window from the previous edge) is caught by
    the golden examples or by brute force."""
    caught = False
    for ex in golden_examples:
        s, d, t, n = edges_of(ex)
        for c in ex["cases"]:
            m = [tuple(e) for e in c["motif"]]
            caught |= oracle_mod.count(s, d, t, n, m, c["delta"], mutant=mutant) != c["count"]
    assert caught
    rng = np.random.default_rng(100)
    s, d, t = tiny_graph(rng, 5, 10, 10)
    diff = 0
    for m in _tiny_motifs()[:40]:
        diff += oracle_mod.count(s, d, t, 5, m, 3, mutant=mutant) != brute.count(s, d, t, m, 3)
    assert diff > 0


def _union_connected(pairs):
    """Whether the undirected union of the edges is one connected piece."""
    parent = {}

    def find(x):
        while parent.setdefault(x, x) != x:
            x = parent[x]
        return x
    for a, b in pairs:
        parent[find(a)] = find(b)
    return len({find(x) for e in pairs for x in e}) == 1


def _window_motifs():
    ms = []
    for k in (1, 2, 3):
        ms += W.enumerate_motifs(k, 2 * k, connected=False)
    rng = np.random.default_rng(17)
    four = W.enumerate_motifs(4, 5, connected=False)
    return ms + [four[i] for i in rng.choice(len(four), 12, replace=False)]


@pytest.mark.parametrize("seed", range(3))
def test_window_and_level_logs_match_brute_force(oracle_mod, seed):
    """The per-root logs the GPU statistics and the scheduler's cost label are
    judged by: window entries per motif edge (the list chosen by the oracle's
    candidate rule, entries with t_prev < t <= t_first + delta, summed over the
    partial matches of the preceding edges) and partial matches per level,
    both recomputed by enumerating edge subsets against the definition."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(3, 7))
    s, d, t = tiny_graph(rng, n, int(rng.integers(8, 12)), 8, self_loops=seed == 1)
    og = oracle_mod.OracleGraph(s, d, t, n)
    for m in _window_motifs():
        for delta in (0, 3, BIG):
            tot, lv, wn, wr = og.count(list(m), delta, level=True, windows=True,
                                       windows_per_root=True)
            want_w = np.array(brute.window_entries(s, d, t, m, delta), dtype=np.uint64)
            assert np.array_equal(wr, want_w), (m, delta)
            assert np.array_equal(wn, want_w.sum(0)), (m, delta)
            for j in range(len(m)):
                col = [brute.count(s, d, t, m[:j + 1], delta, roots=[r]) for r in range(len(s))]
                assert lv[:, j].tolist() == col, (m, delta, j)
            assert int(lv[:, -1].sum()) == tot


def test_search_node_identity(oracle_mod):
    """Per-motif search nodes minus co-mined search nodes equals the sum over
    shared prefixes p of (multiplicity(p) - 1) * count(p).  Per-motif nodes come
    from the oracle's level logs; prefix counts and multiplicities from brute
    force and the motif set."""
    rng = np.random.default_rng(41)
    s, d, t = tiny_graph(rng, 6, 22, 14, self_loops=True)
    motifs = list(W.CONFIG1_MOTIFS) + W.random_extension_motifs(10, (2, 3, 4), 5, 44)
    delta = 6
    og = oracle_mod.OracleGraph(s, d, t, 6)
    mult = {}
    for m in motifs:
        for j in range(1, len(m) + 1):
            mult[tuple(m[:j])] = mult.get(tuple(m[:j]), 0) + 1
    cnt = {p: brute.count(s, d, t, list(p), delta) for p in mult}
    per_motif = 0
    for m in motifs:
        _, lv = og.count(list(m), delta, level=True)
        per_motif += int(lv.sum())
    comined = sum(cnt.values())
    shared = sum((mult[p] - 1) * cnt[p] for p in mult)
    assert per_motif - comined == shared
    assert shared > 0 and any(v > 1 for v in mult.values())


@pytest.mark.parametrize("delta", [5, 12])
def test_partition_identity_908_connected(oracle_mod, delta):
    """The 68 connected 3-edge and 840 connected 4-edge motifs on <= 4
    vertices partition the delta-window triples and quadruples whose union is
    connected, spans <= 4 vertices and has no self-loop (each such tuple has
    exactly one first-appearance form); counted by an independent enumerator
    over edge subsets."""
    three = [m for m in W.enumerate_motifs(3, 4, connected=False) if _union_connected(m)]
    four = [m for m in W.enumerate_motifs(4, 4, connected=False) if _union_connected(m)]
    assert (len(three), len(four)) == (68, 840)
    rng = np.random.default_rng(55)
    s, d, t = tiny_graph(rng, 5, 34, 30, self_loops=True)
    o = np.lexsort((np.arange(len(t)), t))
    s, d, t = s[o], d[o], t[o]
    og = oracle_mod.OracleGraph(s, d, t, 5)
    for k, ms in ((3, three), (4, four)):
        tuples = 0
        for c in itertools.combinations(range(len(t)), k):
            ts = t[list(c)]
            if not np.all(ts[1:] > ts[:-1]) or ts[-1] - ts[0] > delta:
                continue
            pairs = [(int(s[i]), int(d[i])) for i in c]
            if any(a == b for a, b in pairs) or len({x for e in pairs for x in e}) > 4:
                continue
            tuples += _union_connected(pairs)
        got = sum(og.count(list(m), delta) for m in ms)
        assert got == tuples and tuples > 0, (k, got, tuples)


@pytest.mark.parametrize("mutant", [5, 6])
def test_log_pins_catch_planted_mistakes(oracle_mod, mutant):
    """Mistakes that leave every count intact but corrupt a log (window entries
    logged after the structural filter; partial matches logged before it) are
    caught by the brute-force log pins."""
    rng = np.random.default_rng(301)
    n = 5
    s, d, t = tiny_graph(rng, n, 11, 8, self_loops=True)
    og = oracle_mod.OracleGraph(s, d, t, n, mutant=mutant)
    caught = False
    for m in _window_motifs()[:40]:
        tot, lv, wr = og.count(list(m), 3, level=True, windows_per_root=True)
        assert tot == brute.count(s, d, t, m, 3)        # counts stay right
        want_w = np.array(brute.window_entries(s, d, t, m, 3), dtype=np.uint64)
        want_l = [[brute.count(s, d, t, m[:j + 1], 3, roots=[r]) for j in range(len(m))]
                  for r in range(len(s))]
        caught |= not np.array_equal(wr, want_w) or lv.tolist() != want_l
    assert caught
