"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact
uint64 counts on tiny, medium and configuration-shaped graphs, sampled roots
of the full-size benchmark graph, schedule independence, search statistics
and edge cases."""
import sys

import numpy as np
import pytest

from paper_2507_14813_amd import api, workloads as W
from oracle import OracleGraph, brute
from conftest import edges_of, tiny_graph

pytestmark = pytest.mark.gpu
BIG = 10 ** 12


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    api.lib()
    return torch


def gpu_count(s, d, t, n, motifs, delta, **kw):
    say("count", "E=%d" % len(s), "V=%d" % n, "motifs=%d" % len(motifs), "delta=%d" % delta, kw)
    g = api.Graph(s, d, t, n)
    tr = api.Tree(motifs, delta)
    return api.count(g, tr, **kw)


def oracle_counts(og, motifs, delta, roots=None):
    return np.array([og.count(m, delta, roots=roots) for m in motifs], dtype=np.uint64)


def test_golden_examples(golden_examples, oracle_mod):
    for ex in golden_examples:
        s, d, t, n = edges_of(ex)
        by_delta = {}
        for c in ex["cases"]:
            by_delta.setdefault(c["delta"], []).append(c)
        for delta, cases in by_delta.items():
            motifs = [[tuple(e) for e in c["motif"]] for c in cases]
            want = [c["count"] for c in cases]
            for mode in ("comine", "per_motif"):
                got = gpu_count(s, d, t, n, motifs, delta, mode=mode)
                assert got.tolist() == want, (ex["name"], delta, mode)


def _tiny_motifs():
    ms = []
    for k in (1, 2, 3):
        ms += W.enumerate_motifs(k, 2 * k, connected=False)
    rng = np.random.default_rng(7)
    four = W.enumerate_motifs(4, 5, connected=False)
    ms += [four[i] for i in rng.choice(len(four), 40, replace=False)]
    five = W.enumerate_motifs(5, 6, connected=False)
    ms += [five[i] for i in rng.choice(len(five), 40, replace=False)]
    return ms


@pytest.mark.parametrize("seed", range(4))
def test_tiny_random_graphs(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 8))
    s, d, t = tiny_graph(rng, n, int(rng.integers(6, 15)), 10, self_loops=bool(seed % 2))
    og = OracleGraph(s, d, t, n)
    ms = _tiny_motifs()
    for delta in (0, 1, 3, 5, BIG):
        want = oracle_counts(og, ms, delta)
        got = gpu_count(s, d, t, n, ms, delta)
        assert np.array_equal(got, want), delta


def _medium(seed=1, E=4000, V=40, tmax=600, self_loops=True):
    rng = np.random.default_rng(seed)
    s, d, t = tiny_graph(rng, V, E, tmax, self_loops=self_loops)
    ms = (W.random_extension_motifs(30, (2, 3, 4, 5), 6, seed)
          + [m for m in W.enumerate_motifs(3, 6, connected=False) if max(max(e) for e in m) >= 3][:20])
    return s, d, t, V, ms


@pytest.mark.parametrize("delta", [7, 40])
def test_medium_graph_all_modes(delta):
    s, d, t, n, ms = _medium()
    og = OracleGraph(s, d, t, n)
    want = oracle_counts(og, ms, delta)
    assert want.sum() > 0
    g = api.Graph(s, d, t, n)
    tr = api.Tree(ms, delta)
    say("medium", delta)
    assert np.array_equal(api.count(g, tr), want)
    assert np.array_equal(api.count(g, tr, mode="per_motif"), want)
    for blocks, chunk, queues, ls in ((1, 64, 0, 0), (3, 128, 1, -1), (0, 1024, 3, 7),
                                      (0, 64, 8, 1000), (9, 192, 0, 1)):
        say("schedule", blocks, chunk, queues, ls)
        assert np.array_equal(api.count(g, tr, blocks=blocks, chunk=chunk, queues=queues,
                                        leaf_scan=ls), want)
    roots = np.arange(5, len(s), 7)
    say("roots subset")
    assert np.array_equal(api.count(g, tr, roots=roots), oracle_counts(og, ms, delta, roots))


@pytest.mark.parametrize("kmax", [3, 4])
def test_medium_graph_leaf_parents(kmax):
    # trees of up to four edges count batches of leaf parents (nodes whose
    # children all end a motif) one partial match per lane, with groups of
    # lanes sharing each short window and the whole wave taking long ones
    s, d, t, n, ms = _medium(seed=2)
    ms = [m for m in ms if len(m) <= kmax]
    og = OracleGraph(s, d, t, n)
    g = api.Graph(s, d, t, n)
    for delta in (7, 40, 200):
        want = oracle_counts(og, ms, delta)
        tr = api.Tree(ms, delta)
        say("leaf parents", kmax, delta)
        for blocks, chunk, queues, ls in ((0, 64, 0, 0), (1, 64, 0, 1), (0, 128, 3, 5),
                                          (0, 64, 8, 17), (2, 192, 1, 1000)):
            assert np.array_equal(api.count(g, tr, blocks=blocks, chunk=chunk, queues=queues,
                                            leaf_scan=ls), want), (delta, ls)
        tm = api.Tree(ms, [3, delta, 2 * delta])
        want_m = np.stack([oracle_counts(og, ms, x) for x in (3, delta, 2 * delta)])
        assert np.array_equal(api.count(g, tm), want_m), delta


def test_closing_edges_from_hub_out_lists():
    # three-edge motifs whose last edge leaves the second-edge vertex x for a
    # root vertex (x -> a, x -> b): a lane may count those edges in the root's
    # in-lists instead of x's out-list, whichever is shorter.  Hubs with long
    # out-lists or long in-lists make either choice happen, and the three
    # windows put the in-list suffixes below and above 16 entries.
    rng = np.random.default_rng(11)
    n, e = 400, 24000
    s = rng.integers(0, n, e)
    d = rng.integers(0, n, e)
    hub_out = rng.random(e) < 0.25
    s[hub_out] = rng.integers(0, 3, hub_out.sum())
    hub_in = rng.random(e) < 0.15
    d[hub_in] = rng.integers(3, 5, hub_in.sum())
    keep = s != d
    s, d = s[keep].astype(np.int32), d[keep].astype(np.int32)
    t = np.sort(rng.integers(0, 30000, len(s))).astype(np.int64)
    ms = W.enumerate_motifs(3, 3, connected=False)
    og = OracleGraph(s, d, t, n)
    g = api.Graph(s, d, t, n)
    for delta in (6, 60, 400, 1500):
        want = oracle_counts(og, ms, delta)
        assert want.sum() > 0
        tr = api.Tree(ms, delta)
        for ls in (0, 5, 256):
            say("hub closing edges", delta, ls)
            assert np.array_equal(api.count(g, tr, leaf_scan=ls), want), (delta, ls)
        say("hub closing edges, epochs", delta)
        assert np.array_equal(api.count(g, tr, epoch_idle=50), want), delta


def test_three_edge_trees_with_a_four_vertex_prefix():
    # depth-3 kernels keep three vertices per level-2 partial match; a tree
    # whose two-edge prefix spans four vertices (and goes deeper) runs on the
    # depth-4 kernel, in every mode and in batches
    s, d, t, n, _ = _medium(seed=3)
    og = OracleGraph(s, d, t, n)
    g = api.Graph(s, d, t, n)
    conn = W.enumerate_motifs(3, 3)
    wide = [m for m in W.enumerate_motifs(3, 4, connected=False)
            if len({v for e in m[:2] for v in e}) == 4][:12]
    assert wide
    for ms, kdepth in ((conn, 3), (conn + wide, 4)):
        for delta in (7, 40):
            say("four-vertex prefix", kdepth, delta)
            want = oracle_counts(og, ms, delta)
            tr = api.Tree(ms, delta)
            assert np.array_equal(api.count(g, tr), want), (kdepth, delta)
            assert np.array_equal(api.count(g, tr, mode="per_motif"), want)
            c, st = api.count(g, tr, stats=True)
            assert np.array_equal(c, want)
            assert np.array_equal(api.count(g, tr, epoch_idle=50), want)
            tm = api.Tree(ms, [3, delta])
            want_m = np.stack([oracle_counts(og, ms, 3), want])
            assert np.array_equal(api.count(g, tm), want_m)
            b = api.Batch([g], [tr], item_roots=64)
            assert b.info()["depth"] == kdepth
            assert np.array_equal(b.count()[0], want)


def test_epochs_hand_on_leftovers_exactly():
    # an epoch ends as soon as a few waves are idle: the busy waves write what
    # is left of their root-level windows as contexts, and later launches
    # search them; no candidate is searched twice or skipped
    s, d, t, n, ms = _medium(seed=3)
    og = OracleGraph(s, d, t, n)
    g = api.Graph(s, d, t, n)
    carried = 0
    for kmax in (3, 5):
        mm = [m for m in ms if len(m) <= kmax]
        for delta in (60, 200):
            want = oracle_counts(og, mm, delta)
            tr = api.Tree(mm, delta)
            for pct, epochs, blocks, chunk in ((1, 16, 0, 64), (1, 3, 0, 64), (1, 2, 4, 128),
                                               (50, 16, 2, 64), (100, 4, 1, 64)):
                say("epochs", kmax, delta, pct, epochs, blocks)
                log = np.zeros(epochs, np.int64)
                got = api.count(g, tr, epoch_idle=pct, max_epochs=epochs, epoch_contexts=log,
                                blocks=blocks, chunk=chunk)
                assert np.array_equal(got, want), (kmax, delta, pct, epochs, blocks, log)
                assert log[-1] == 0
                carried += int(log.sum())
            tm = api.Tree(mm, [7, delta, 3 * delta])
            want_m = np.stack([oracle_counts(og, mm, x) for x in (7, delta, 3 * delta)])
            assert np.array_equal(api.count(g, tm, epoch_idle=1), want_m), delta
    assert carried > 0   # some epochs did end early and hand work on
    with pytest.raises(api.MayuraError):
        api.count(g, tr, epoch_idle=5, stats=True)
    with pytest.raises(api.MayuraError):
        api.count(g, tr, epoch_idle=101)


@pytest.mark.parametrize("seed", range(3))
def test_multi_window_tiny(seed):
    """One search for several windows equals the oracle at every window, on
    tiny graphs with forced ties, every motif with k <= 3 and sampled four-
    and five-edge motifs, in co-mining and per-motif mode."""
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(3, 8))
    s, d, t = tiny_graph(rng, n, int(rng.integers(8, 16)), 10, self_loops=seed == 1)
    og = OracleGraph(s, d, t, n)
    ms = _tiny_motifs()
    windows = [5, 0, BIG, 3, 1, 3]
    want = np.stack([oracle_counts(og, ms, w) for w in windows])
    g = api.Graph(s, d, t, n)
    tr = api.Tree(ms, windows)
    say("multi-window tiny", seed)
    assert np.array_equal(api.count(g, tr), want)
    assert np.array_equal(api.count(g, tr, mode="per_motif"), want)


def test_multi_window_medium_every_path():
    """Several windows on a medium graph through each leaf-counting path
    (lane-counted, wave-counted, expanded), with statistics equal to a plain
    search at the largest window, in a batch, and without allocation."""
    s, d, t, n, ms = _medium(seed=2, E=6000, V=30, tmax=900)
    windows = [40, 7, 19, 0]
    og = OracleGraph(s, d, t, n)
    want = np.stack([oracle_counts(og, ms, w) for w in windows])
    g = api.Graph(s, d, t, n)
    tr = api.Tree(ms, windows)
    for ls in (0, 1, 4, -1):
        say("multi-window medium leaf_scan", ls)
        assert np.array_equal(api.count(g, tr, leaf_scan=ls), want), ls
    _, st = api.count(g, tr, stats=True)
    _, st1 = api.count(g, api.Tree(ms, max(windows)), stats=True)
    assert st == st1
    roots = np.arange(1, len(s), 3)
    want_r = np.stack([oracle_counts(og, ms, w, roots) for w in windows])
    assert np.array_equal(api.count(g, tr, roots=roots), want_r)
    say("multi-window batch")
    single = api.Tree(ms[:7], 11)
    b = api.Batch([g, g], [tr, single], item_roots=128)
    for _ in range(2):
        a, c = b.count()
        assert np.array_equal(a, want) and np.array_equal(c, oracle_counts(og, ms[:7], 11))
    say("multi-window noalloc")
    assert np.array_equal(api.count_noalloc(g, tr), want)


def _records(motif, edges):
    return sorted((int(m),) + tuple(int(x) for x in e if x >= 0) for m, e in zip(motif, edges))


@pytest.mark.parametrize("seed", range(3))
def test_enumeration_equals_brute_force(seed):
    """Every match written out by the search equals the brute-force list of
    the definition on tiny graphs (ties, self-loops, unsorted input), for
    every motif with k <= 3 and sampled four- and five-edge motifs; the
    hand-listed matches of Example A come out as listed."""
    rng = np.random.default_rng(600 + seed)
    n = int(rng.integers(3, 7))
    s, d, t = tiny_graph(rng, n, int(rng.integers(8, 13)), 8, self_loops=seed != 1)
    perm = rng.permutation(len(s))
    s, d, t = s[perm], d[perm], t[perm]
    ms = _tiny_motifs()[::3] + [[(0, 1), (2, 3)], [(0, 1), (0, 1)]]
    g = api.Graph(s, d, t, n)
    for delta in (0, 4, BIG):
        say("enumerate tiny", seed, delta)
        tr = api.Tree(ms + [ms[0]], delta)           # a duplicate motif
        motif, edges = api.enumerate_matches(g, tr)
        want = sorted((i,) + tup for i, m in enumerate(ms) for tup in brute.matches(s, d, t, m, delta))
        assert _records(motif, edges) == want


def test_enumeration_golden_and_medium(golden_examples):
    A = golden_examples[0]
    s, d, t, n = edges_of(A)
    cases = [c for c in A["cases"] if "matches" in c]
    g = api.Graph(s, d, t, n)
    tr = api.Tree([[tuple(e) for e in c["motif"]] for c in cases], 30)
    motif, edges = api.enumerate_matches(g, tr)
    assert _records(motif, edges) == sorted((i,) + tuple(x) for i, c in enumerate(cases)
                                            for x in c["matches"])
    # medium graph: as many records per motif as the oracle counts, every one
    # a match, no record twice
    s, d, t, n, ms = _medium(seed=5, E=3000, V=25, tmax=500)
    og = OracleGraph(s, d, t, n)
    want = oracle_counts(og, ms, 20)
    g = api.Graph(s, d, t, n)
    say("enumerate medium")
    motif, edges = api.enumerate_matches(g, api.Tree(ms, 20))
    # a duplicate motif's matches are reported under its first occurrence
    first = {}
    exp = np.zeros(len(ms), np.uint64)
    for i, m in enumerate(ms):
        if tuple(map(tuple, m)) not in first:
            first[tuple(map(tuple, m))] = i
            exp[i] = want[i]
    assert len(first) < len(ms)
    assert np.array_equal(np.bincount(motif, minlength=len(ms)).astype(np.uint64), exp)
    recs = _records(motif, edges)
    assert len(set(recs)) == len(recs)
    rng = np.random.default_rng(1)
    for i in rng.choice(len(recs), min(len(recs), 3000), replace=False):
        m, *es = recs[i]
        assert brute.is_match([(int(s[x]), int(d[x]), int(t[x])) for x in es], ms[m], 20)
    with pytest.raises(api.MayuraError, match="MG_EUNSUPPORTED"):
        api.enumerate_matches(g, api.Tree(ms, [5, 20]))


def test_autotuner_and_its_cache(tmp_path):
    """mg_tune picks settings by timing, appends them to its cache and reads
    them back without timing; counts with the tuned settings equal the
    oracle's."""
    s, d, t, n, ms = _medium(seed=4, E=30000, V=200, tmax=20000)
    og = OracleGraph(s, d, t, n)
    want = oracle_counts(og, ms, 300)
    g = api.Graph(s, d, t, n)
    tr = api.Tree(ms, 300)
    cache = str(tmp_path / "tune.jsonl")
    say("tune")
    r = api.tune(g, tr, cache=cache)
    assert r["from_cache"] == 0 and r["trials"] >= 10 and r["ms"] <= r["default_ms"]
    assert r["chunk"] % 64 == 0 and 1 <= r["queues"] <= 8 and r["leaf_scan"] > 0
    r2 = api.tune(g, tr, cache=cache)
    assert r2["from_cache"] == 1 and r2["trials"] == 0
    assert {k: r2[k] for k in ("blocks", "chunk", "queues", "leaf_scan")} == \
        {k: r[k] for k in ("blocks", "chunk", "queues", "leaf_scan")}
    assert len(open(cache).read().splitlines()) == 1
    kw = {k: r[k] for k in ("blocks", "chunk", "queues", "leaf_scan")}
    assert np.array_equal(api.count(g, tr, **kw), want)
    # another tree is another key
    r3 = api.tune(g, api.Tree(ms[:5], 300), cache=cache)
    assert r3["from_cache"] == 0 and len(open(cache).read().splitlines()) == 2


def test_stop_and_resume():
    """A count stopped by a chunk budget and resumed from its cursor until
    done sums to the oracle's counts and statistics, on every root and on a
    root subset; a stop flag set before the call searches nothing and leaves
    the cursor where it was."""
    import torch
    s, d, t, n, ms = _medium(seed=3, E=20000, V=60)
    delta = 25
    og = OracleGraph(s, d, t, n)
    g = api.Graph(s, d, t, n)
    tr = api.Tree(ms, delta)
    want = oracle_counts(og, ms, delta)
    _, want_st = api.count(g, tr, stats=True)
    stop = torch.zeros(1, dtype=torch.int32, device="cuda")
    pinned = torch.zeros(1, dtype=torch.int32).pin_memory()
    for roots, budget, queues in ((None, 5, 0), (None, 1, 3), (np.arange(3, len(s), 5), 2, 8)):
        say("resume", "roots" if roots is not None else "all", budget, queues)
        exp = want if roots is None else oracle_counts(og, ms, delta, roots)
        cur = api.Cursor()
        total = np.zeros(len(ms), np.uint64)
        st_total = {}
        calls = 0
        while not cur.done:
            flag = pinned if calls % 2 else stop
            before = sum(cur.head)
            c, st = api.count(g, tr, roots=roots, queues=queues, max_chunks=budget,
                              stop=flag.data_ptr(), cursor=cur, stats=True)
            total += c
            for k, v in st.items():
                st_total[k] = st_total.get(k, 0) + v
            calls += 1
            # every call with a budget searches at least one chunk, at most `budget`
            assert before < sum(cur.head) <= before + 64 * budget
            if calls == 2:
                # a raised flag: nothing is searched and the cursor stays
                heads = list(cur.head)
                stop.fill_(1)
                torch.cuda.synchronize()
                c0 = api.count(g, tr, roots=roots, queues=queues, stop=stop.data_ptr(),
                               cursor=cur)
                assert int(c0.sum()) == 0 and list(cur.head) == heads and not cur.done
                stop.fill_(0)
                torch.cuda.synchronize()
        assert calls > 2
        assert np.array_equal(total, exp)
        if roots is None:
            assert st_total == want_st
    # a cursor is tied to its count's roots, chunk and queues
    cur = api.Cursor()
    api.count(g, tr, max_chunks=1, cursor=cur)
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        api.count(g, tr, chunk=128, cursor=cur)
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        api.count(g, tr, mode="per_motif", max_chunks=1)


def _trie_expectations(og, motifs, delta):
    """Search statistics the co-mining search must produce, derived from the
    oracle's per-motif counts and window logs: each distinct prefix is matched
    once, each (prefix, list) pair opens one window per match of the prefix."""
    def canon(m):
        lab = {}
        out = []
        for u, v in m:
            for x in (u, v):
                if x not in lab:
                    lab[x] = len(lab)
            out.append((lab[u], lab[v]))
        return tuple(out)

    prefixes = set()
    for m in motifs:
        c = canon(m)
        for j in range(1, len(c) + 1):
            prefixes.add(c[:j])
    kids = {}
    for p in prefixes:
        if len(p) > 1:
            kids.setdefault(p[:-1], []).append(p)
    cnt = {p: og.count(list(p), delta) for p in prefixes}
    st = dict(win_list=0, win_all=0, ent_list=0, ent_all=0, push=0, credit=0)
    for p in prefixes:
        if len(p) > 1:
            st["credit"] += cnt[p]
            if p in kids:
                st["push"] += cnt[p]
        if p not in kids:
            continue
        nv = 1 + max(max(e) for e in p)
        groups = {}
        for c in kids[p]:
            u, v = c[-1]
            key = ("out", u) if u < nv else (("in", v) if v < nv else ("all", 0))
            groups.setdefault(key, c)
        for key, c in groups.items():
            _, wins = og.count(list(c), delta, windows=True)
            name = "all" if key[0] == "all" else "list"
            st["win_" + name] += cnt[p]
            st["ent_" + name] += int(wins[len(p)])
    return st


def test_search_statistics_match_oracle():
    # per-vertex lists on the GPU leave self-loops out (they never match) while
    # the oracle scans them, so window sizes are compared on a loop-free graph
    s, d, t, n, ms = _medium(seed=3, E=2500, self_loops=False)
    og = OracleGraph(s, d, t, n)
    want = _trie_expectations(og, ms, 30)
    g = api.Graph(s, d, t, n)
    tr = api.Tree(ms, 30)
    say("stats")
    counts, st = api.count(g, tr, stats=True)
    assert np.array_equal(counts, oracle_counts(og, ms, 30))
    assert st["roots"] == int((s != d).sum())
    for k, v in want.items():
        assert st[k] == v, (k, st[k], v)
    # every way of counting leaf windows (lane, whole wave, candidate expansion)
    # gives the same statistics
    for ls in (1, 4, -1):
        say("stats, leaf_scan", ls)
        c2, st2 = api.count(g, tr, stats=True, leaf_scan=ls)
        assert np.array_equal(c2, counts) and st2 == st, ls


def _root_cost_expectation(og, motifs, delta, n_edges, src, dst):
    """Per-root search cost of co-mining from the oracle's per-root window
    logs: 1 for the root plus, for every distinct prefix p with children and
    every list its children scan, the window entries under that root."""
    def canon(m):
        lab, out = {}, []
        for u, v in m:
            for x in (u, v):
                lab.setdefault(x, len(lab))
            out.append((lab[u], lab[v]))
        return tuple(out)
    prefixes = {c[:j] for m in motifs for c in [canon(m)] for j in range(1, len(c) + 1)}
    kids = {}
    for p in prefixes:
        if len(p) > 1:
            kids.setdefault(p[:-1], []).append(p)
    o = np.lexsort((np.arange(n_edges), og_times(og)))
    cost = (src[o] != dst[o]).astype(np.uint64)
    for p, cs in kids.items():
        nv = 1 + max(max(e) for e in p)
        seen = set()
        for c in cs:
            u, v = c[-1]
            key = ("out", u) if u < nv else (("in", v) if v < nv else ("all", 0))
            if key in seen:
                continue
            seen.add(key)
            _, wr = og.count(list(c), delta, windows_per_root=True)
            cost += wr[:, len(p)]
    return cost


def og_times(og):
    return og.t_sorted


def test_per_root_cost_log_matches_oracle():
    # loop-free graph: the oracle's lists keep self-loop edges, the GPU's do not
    s, d, t, n, ms = _medium(seed=4, E=3000, self_loops=False)
    o = np.lexsort((np.arange(len(t)), t))
    og = OracleGraph(s, d, t, n)
    og.t_sorted = t[o]
    g = api.Graph(s, d, t, n)
    say("root cost log")
    for delta in (9, 35):
        tr = api.Tree(ms, delta)
        counts, cost = api.count(g, tr, root_cost=True)
        assert np.array_equal(counts, oracle_counts(og, ms, delta))
        want = _root_cost_expectation(og, ms, delta, len(s), s, d)
        assert np.array_equal(cost, want), delta
        # per-motif mode logs the sum of the per-motif searches
        _, cpm = api.count(g, tr, mode="per_motif", root_cost=True)
        assert (cpm >= cost).all() and cpm.sum() > cost.sum()


def test_batch_equals_single_counts_and_oracle(gpu):
    """Jobs of uneven size and depth (one graph shared by two jobs) in one
    launch; every replay of the captured step matches the single counts and
    the oracle, with eager work between replays."""
    rng = np.random.default_rng(12)
    graphs, trees, want = [], [], []
    for j in range(7):
        E = int(rng.integers(50, 3000))
        n = int(rng.integers(5, 60))
        s, d, t = tiny_graph(rng, n, E, int(rng.integers(50, 2000)), self_loops=True)
        ms = W.random_extension_motifs(int(rng.integers(2, 12)), (1, 2, 3, 4), 5, 50 + j)
        delta = int(rng.integers(0, 200))
        og = OracleGraph(s, d, t, n)
        g = api.Graph(s, d, t, n)
        graphs.append(g)
        trees.append(api.Tree(ms, delta))
        want.append(oracle_counts(og, ms, delta))
        if j == 2:   # same graph, second motif group
            ms2 = [[(0, 1), (1, 0)], [(0, 1), (1, 2), (2, 0)], [(5, 6)]]
            graphs.append(g)
            trees.append(api.Tree(ms2, delta + 7))
            want.append(oracle_counts(og, ms2, delta + 7))
    single = [api.count(g, tr) for g, tr in zip(graphs, trees)]
    for a, b in zip(single, want):
        assert np.array_equal(a, b)
    for kw in (dict(), dict(item_roots=64), dict(item_roots=192, use_graph=False)):
        say("batch", kw)
        b = api.Batch(graphs, trees, **kw)
        for rep in range(3):
            got = b.count()
            for a, w in zip(got, want):
                assert np.array_equal(a, w), (kw, rep)
            x = gpu.arange(1000, device="cuda").sum()      # eager work between replays
            gpu.cuda.synchronize()
            assert int(x) == 499500
        info = b.info()
        assert info["graph_captured"] == (0 if kw.get("use_graph") is False else 1)
        assert info["n_jobs"] == len(graphs) and info["item_roots"] % 64 == 0
        b.close()
    say("one-shot batch")
    for kw in (dict(), dict(item_roots=128)):
        for a, w in zip(api.count_batch(graphs, trees, **kw), want):
            assert np.array_equal(a, w), kw


@pytest.mark.parametrize("depth", [1, 2, 3, 5])
def test_batch_every_depth(depth):
    """Batches whose deepest tree has 1, 2, 3 or 5 edges (each depth is its own
    kernel instantiation with its own per-wave LDS layout)."""
    rng = np.random.default_rng(30 + depth)
    graphs, trees, want = [], [], []
    for j in range(3):
        n = int(rng.integers(6, 40))
        s, d, t = tiny_graph(rng, n, int(rng.integers(200, 2500)), 400, self_loops=True)
        ks = tuple(range(1, depth + 1))
        ms = W.random_extension_motifs(6, ks, 6, 300 + 10 * depth + j)
        if j == 0:
            ms = ms + [tuple([(0, 1)] + [(1, 0), (0, 1)] * 2)[:depth]]
        delta = int(rng.integers(10, 120))
        og = OracleGraph(s, d, t, n)
        graphs.append(api.Graph(s, d, t, n))
        trees.append(api.Tree(ms, delta))
        want.append(oracle_counts(og, ms, delta))
    say("batch depth", depth)
    b = api.Batch(graphs, trees, item_roots=64)
    assert b.info()["depth"] == depth
    for _ in range(2):
        for a, w in zip(b.count(), want):
            assert np.array_equal(a, w)


def test_config1_full():
    wl = W.make_config(1)
    s, d, t, n = wl.graphs[0]
    og = OracleGraph(s, d, t, n)
    ms, delta = wl.motif_sets[0], wl.deltas[0]
    want = oracle_counts(og, ms, delta)
    assert np.array_equal(gpu_count(s, d, t, n, ms, delta), want)
    assert np.array_equal(gpu_count(s, d, t, n, ms, delta, mode="per_motif"), want)


@pytest.mark.parametrize("k,scale", [(2, 0.01), (4, 0.002), (5, 0.0005)])
def test_config_minis(k, scale):
    wl = W.make_config(k, scale=scale)
    s, d, t, n = wl.graphs[0]
    og = OracleGraph(s, d, t, n)
    ms = wl.motif_sets[0]
    g = api.Graph(s, d, t, n)
    for delta in wl.deltas:
        want = oracle_counts(og, ms, delta)
        tr = api.Tree(ms, delta)
        say("config", k, scale, delta)
        assert np.array_equal(api.count(g, tr), want), (k, delta)


def test_edge_cases(oracle_mod):
    ms = [[(0, 1)], [(0, 1), (1, 2)], [(0, 1), (2, 3), (1, 2)]]
    # empty graph
    say("empty graph")
    assert gpu_count(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64), 3,
                     ms, 5).tolist() == [0, 0, 0]
    # only self-loops
    say("self-loops only")
    z = np.array([0, 1, 1], np.int32)
    assert gpu_count(z, z, np.array([1, 2, 3]), 2, ms, 5).tolist() == [0, 0, 0]
    rng = np.random.default_rng(5)
    s, d, t = tiny_graph(rng, 9, 300, 40, self_loops=True)
    og = OracleGraph(s, d, t, 9)
    g = api.Graph(s, d, t, 9)
    # no roots
    say("no roots")
    assert api.count(g, api.Tree(ms, 5), roots=np.zeros(0, np.int64)).tolist() == [0, 0, 0]
    # self-loop roots are never searched
    say("root cost of self-loops")
    _, cost = api.count(g, api.Tree(ms, 5), root_cost=True)
    o = np.lexsort((np.arange(len(t)), t))
    assert (cost[(s[o] == d[o])] == 0).all() and (cost[(s[o] != d[o])] >= 1).all()
    # depth-1 tree, duplicates with other labels
    say("depth 1 and duplicates")
    got = api.count(g, api.Tree([[(0, 1)], [(4, 2)]], 3))
    assert got.tolist() == [int((s != d).sum())] * 2
    dup = [[(0, 1), (1, 2), (2, 0)], [(5, 6), (6, 7), (7, 5)], [(0, 1), (1, 0)]]
    got = api.count(g, api.Tree(dup, 8))
    assert got[0] == got[1] == og.count(dup[0], 8) and got[2] == og.count(dup[2], 8)
    # window 0 and an unbounded window
    for delta in (0, BIG, 2 ** 63 - 1):
        say("delta", delta)
        assert np.array_equal(api.count(g, api.Tree(ms, delta)), oracle_counts(og, ms, delta))
    # unsorted input is sorted stably by the library
    perm = rng.permutation(len(s))
    say("unsorted input")
    got = gpu_count(s[perm], d[perm], t[perm], 9, ms, 6)
    og2 = OracleGraph(s[perm], d[perm], t[perm], 9)
    assert np.array_equal(got, oracle_counts(og2, ms, 6))


def test_device_input_graph(gpu):
    """Edges handed over in device memory (MG_DEVICE_INPUT) give the same graph
    and counts as host arrays, sorted or not."""
    rng = np.random.default_rng(9)
    s, d, t = tiny_graph(rng, 20, 2000, 300, self_loops=True)
    ms = W.random_extension_motifs(10, (2, 3, 4), 5, 9)
    og = OracleGraph(s, d, t, 20)
    want = oracle_counts(og, ms, 30)
    tr = api.Tree(ms, 30)
    for perm in (np.arange(len(s)), rng.permutation(len(s))):
        say("device input")
        g = api.Graph(*(gpu.from_numpy(np.ascontiguousarray(x[perm])).cuda() for x in (s, d, t)), 20)
        assert g.info()["n_edges"] == len(s) and g.info()["self_loops"] == int((s == d).sum())
        assert np.array_equal(api.count(g, tr), want)
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        bad = gpu.from_numpy(np.array([0, 25], np.int32)).cuda()
        api.Graph(bad, bad.flip(0), gpu.zeros(2, dtype=gpu.int64, device="cuda"), 20)


def test_wide_time_span_uses_64bit_times():
    rng = np.random.default_rng(8)
    s, d, t = tiny_graph(rng, 12, 600, 80, self_loops=False)
    t = t * (2 ** 30) + 5          # span > 2^32
    ms = W.random_extension_motifs(12, (2, 3, 4), 5, 2)
    og = OracleGraph(s, d, t, 12)
    g = api.Graph(s, d, t, 12)
    assert g.info()["time_bytes"] == 8
    for delta in (3 * 2 ** 30, 20 * 2 ** 30):
        say("64-bit times", delta)
        assert np.array_equal(api.count(g, api.Tree(ms, delta)), oracle_counts(og, ms, delta))


def test_invalid_arguments():
    say("invalid arguments")
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        api.Graph(np.array([0, 5], np.int32), np.array([1, 1], np.int32), np.array([1, 2]), 3)
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        api.Graph(np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([5, 2]), 3,
                  sorted_by_t=True)
    g = api.Graph(np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1, 2]), 3)
    tr = api.Tree([[(0, 1), (1, 2)]], 5)
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        api.count(g, tr, roots=np.array([0, 2]))
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        api.count(g, tr, chunk=100)
    with pytest.raises(api.MayuraError, match="MG_EINVAL"):
        api.count(g, tr, queues=9)
    assert api.count(g, tr).tolist() == [1]
