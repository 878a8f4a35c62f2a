"""The learned root-cost scheduler: MFMA MLP numerics against a CPU FP32
reference on the same BF16-rounded weights, features against a NumPy
recomputation, the training step's update direction, loss decrease, held-out
rank correlation, and exact counts under the learned schedule."""
import sys

import numpy as np
import pytest

from paper_2507_14813_amd import api, workloads as W
from oracle import OracleGraph
from conftest import tiny_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    return torch


def bf16(x):
    """Round to BF16 (nearest even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def unpack(P):
    o = 0
    W1 = P[o:o + 2048].reshape(32, 64); o += 2048
    b1 = P[o:o + 64]; o += 64
    W2 = P[o:o + 4096].reshape(64, 64); o += 4096
    b2 = P[o:o + 64]; o += 64
    W3 = P[o:o + 4096].reshape(64, 64); o += 4096
    b3 = P[o:o + 64]; o += 64
    W4 = P[o:o + 64]; o += 64
    return W1, b1, W2, b2, W3, b3, W4, P[o]


def mlp_ref(P, F):
    """Forward pass with the kernel's precision: BF16 inputs to every product,
    wide accumulation, FP32 bias and ReLU."""
    W1, b1, W2, b2, W3, b3, W4, b4 = [np.asarray(a, np.float64) for a in unpack(P)]
    X = np.zeros((len(F), 32)); X[:, :16] = F
    h1 = np.maximum(bf16(X).astype(np.float64) @ bf16(W1) + b1, 0)
    h2 = np.maximum(bf16(h1).astype(np.float64) @ bf16(W2) + b2, 0)
    h3 = np.maximum(bf16(h2).astype(np.float64) @ bf16(W3) + b3, 0)
    return bf16(h3).astype(np.float64) @ bf16(W4) + b4, (X, h1, h2, h3)


def test_mlp_forward_matches_cpu_reference():
    rng = np.random.default_rng(0)
    m = api.Model(seed=3)
    P = m.weights()
    P[2048:2112] = rng.normal(0, 0.1, 64)          # non-zero biases
    P[-1] = 1.5
    m.set_weights(P)
    F = rng.uniform(0, 1, (1000, 16)).astype(np.float32)
    say("mlp forward")
    got = m.predict(F)
    want, _ = mlp_ref(P, F)
    err = np.abs(got - want)
    assert np.median(err) < 1e-3 * (1 + np.median(np.abs(want)))
    assert np.all(err <= 0.02 + 0.02 * np.abs(want)), err.max()


def test_training_step_matches_reference_gradients():
    """One Adam step from zero moments moves every weight by ~lr against the
    sign of its gradient, and the gradient read back from Adam's moments
    equals, element by element, a CPU reference of the backward pass with the
    kernel's BF16 roundings."""
    rng = np.random.default_rng(1)
    m = api.Model(seed=5)
    P0 = m.weights()
    F = rng.uniform(0, 1, (32, 16)).astype(np.float32)
    y = rng.uniform(0, 4, 32).astype(np.float32)
    lr = 1e-3
    say("train one step")
    m.train(F, y, epochs=1, lr=lr, seed=0)
    P1 = m.weights()
    W1, b1, W2, b2, W3, b3, W4, b4 = [np.asarray(a, np.float64) for a in unpack(P0)]
    pred, (X, h1, h2, h3) = mlp_ref(P0, F)
    h1, h2, h3 = [bf16(h).astype(np.float64) for h in (h1, h2, h3)]
    dout = 2 * (pred - y) / 32
    g = {}
    g["W4"] = h3.T @ dout
    g["b4"] = np.array([dout.sum()])
    dz3 = bf16(np.where(h3 > 0, np.outer(dout, bf16(W4)), 0)).astype(np.float64)
    dz2 = bf16(np.where(h2 > 0, dz3 @ bf16(W3).T, 0)).astype(np.float64)
    dz1 = bf16(np.where(h1 > 0, dz2 @ bf16(W2).T, 0)).astype(np.float64)
    g["W3"], g["b3"] = h2.T @ dz3, dz3.sum(0)
    g["W2"], g["b2"] = h1.T @ dz2, dz2.sum(0)
    g["W1"], g["b1"] = (bf16(X).astype(np.float64).T @ dz1)[:16], dz1.sum(0)
    p0 = dict(zip(("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"), unpack(P0)))
    p1 = dict(zip(("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"), unpack(P1)))
    p0["W1"], p1["W1"] = p0["W1"][:16], p1["W1"][:16]
    agree = total = 0
    for k, gr in g.items():
        d = (np.asarray(p1[k], np.float64) - np.asarray(p0[k], np.float64)).reshape(-1)
        gr = gr.reshape(-1)
        big = np.abs(gr) > 1e-3 * np.abs(gr).max()
        agree += int((np.sign(d[big]) == -np.sign(gr[big])).sum())
        total += int(big.sum())
        assert np.all(np.abs(d) <= 1.01 * lr + 1e-7)
    assert total > 1000 and agree >= 0.97 * total, (agree, total)
    assert np.all(P1[16 * 64:32 * 64] == 0)          # padding rows of W1 stay zero
    # the gradient itself, element by element: after one step from fresh
    # moments Adam's first moment is (1 - beta1) * g and its second
    # (1 - beta2) * g^2
    m1, m2 = m.moments()
    m1d = dict(zip(("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"), unpack(m1)))
    m2d = dict(zip(("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"), unpack(m2)))
    m1d["W1"], m2d["W1"] = m1d["W1"][:16], m2d["W1"][:16]
    one_b1 = float(np.float32(1) - np.float32(0.9))
    one_b2 = float(np.float32(1) - np.float32(0.999))
    for k, gr in g.items():
        gr = gr.reshape(-1)
        got = np.asarray(m1d[k], np.float64).reshape(-1) / one_b1
        scale = np.abs(gr).max()
        # BF16 operands (8-bit mantissa) and FP32 accumulation in another
        # order: a relative L2 error of 2 % and no element off by more than
        # 5 % of the layer's largest gradient
        rel = np.linalg.norm(got - gr) / np.linalg.norm(gr)
        assert rel < 0.02, (k, rel)
        assert np.all(np.abs(got - gr) <= 0.05 * scale), (k, np.abs(got - gr).max(), scale)
        sq = np.asarray(m2d[k], np.float64).reshape(-1) / one_b2
        assert np.allclose(sq, got ** 2, rtol=1e-3, atol=1e-12 * scale ** 2), k


def test_features_match_numpy():
    rng = np.random.default_rng(2)
    s, d, t = tiny_graph(rng, 30, 4000, 3000, self_loops=True)
    g = api.Graph(s, d, t, 30)
    tr = api.Tree(W.CONFIG1_MOTIFS, 40)
    say("features")
    f = api.root_features(g, tr)
    o = np.lexsort((np.arange(len(t)), t))
    s, d, t = s[o], d[o], t[o]
    loop = s == d
    deg_o = np.bincount(s[~loop], minlength=30)
    deg_i = np.bincount(d[~loop], minlength=30)
    ts = {}
    for v in range(30):
        ts[("o", v)] = t[(s == v) & ~loop]
        ts[("i", v)] = t[(d == v) & ~loop]
    L = lambda x: np.log1p(np.asarray(x, np.float64)) / 16
    win = lambda arr, a: np.searchsorted(arr, a + 40, "right") - np.searchsorted(arr, a, "right")
    want = np.zeros((len(s), 16))
    for r in range(len(s)):
        a, b, tt = s[r], d[r], t[r]
        if a == b:
            continue
        want[r, :4] = L([deg_o[a], deg_i[a], deg_o[b], deg_i[b]])
        want[r, 4:8] = L([win(ts[("o", a)], tt), win(ts[("o", b)], tt),
                          win(ts[("i", a)], tt), win(ts[("i", b)], tt)])
        want[r, 8] = L(win(t, tt))
        want[r, 9], want[r, 10], want[r, 11] = 3 / 8, np.log1p(4) / 8, 1
    assert np.allclose(f, want, atol=1e-5)


def _cost_data(cfg, scale, seed_shift=0):
    wl = W.make_config(cfg, scale=scale)
    s, d, t, n = wl.graphs[0]
    g = api.Graph(s, d, t, n)
    tr = api.Tree(wl.motif_sets[0], wl.deltas[0])
    counts, cost = api.count(g, tr, root_cost=True)
    f = api.root_features(g, tr)
    live = cost > 0
    return g, tr, counts, f[live], np.log1p(cost[live]).astype(np.float32)


def test_training_learns_and_generalises():
    say("cost data")
    _, _, _, f_tr, y_tr = _cost_data(2, 0.004)
    m = api.Model(seed=0)
    say("train")
    loss = m.train(f_tr, y_tr, epochs=6, lr=2e-3, seed=1)
    assert loss[-1] < 0.5 * loss[0], loss
    # held out: a larger graph of the same family (another size, same recipe)
    _, _, _, f_te, y_te = _cost_data(2, 0.006)
    pred = m.predict(f_te)
    rank = lambda x: np.argsort(np.argsort(x))
    rho = np.corrcoef(rank(pred), rank(y_te))[0, 1]
    assert rho > 0.6, rho


def test_learned_schedule_counts_are_exact():
    rng = np.random.default_rng(4)
    s, d, t = tiny_graph(rng, 40, 5000, 700, self_loops=True)
    ms = W.random_extension_motifs(25, (2, 3, 4, 5), 6, 11)
    og = OracleGraph(s, d, t, 40)
    g = api.Graph(s, d, t, 40)
    m = api.Model(seed=9)
    for delta in (15, 60):
        tr = api.Tree(ms, delta)
        want = np.array([og.count(x, delta) for x in ms], dtype=np.uint64)
        for sample in (0, 1, 4, 64):
            say("learned schedule", delta, "sample", sample)
            assert np.array_equal(api.count(g, tr, model=m, sample=sample), want)
        _, cost = api.count(g, tr, root_cost=True)
        f = api.root_features(g, tr)
        live = cost > 0
        m.train(f[live], np.log1p(cost[live]).astype(np.float32), epochs=3, lr=2e-3)
        assert np.array_equal(api.count(g, tr, model=m), want)
        # adversarial predictions: the trained costs in reverse order (the output
        # layer negated), and one huge cost for every root
        w = m.weights()
        inv = w.copy()
        inv[-(64 + 1):] *= -1.0
        flat = w.copy()
        flat[-(64 + 1):-1] = 0.0
        flat[-1] = 30.0
        for bad in (inv, flat):
            say("adversarial model", delta)
            assert np.array_equal(api.count(g, tr, model=api.Model(weights=bad)), want)
    wl = W.make_config(2, scale=0.01)
    s, d, t, n = wl.graphs[0]
    g = api.Graph(s, d, t, n)
    tr = api.Tree(wl.motif_sets[0], wl.deltas[0])
    say("learned schedule config-2 mini")
    assert np.array_equal(api.count(g, tr, model=m), api.count(g, tr))
    for bad in (-1, 3, 128):
        with pytest.raises(api.MayuraError):
            api.count(g, tr, model=m, sample=bad)


def test_learned_batch_counts_are_exact():
    rng = np.random.default_rng(6)
    graphs, trees, want = [], [], []
    for j in range(5):
        n = int(rng.integers(8, 50))
        s, d, t = tiny_graph(rng, n, int(rng.integers(100, 4000)), int(rng.integers(100, 3000)),
                             self_loops=True)
        ms = W.random_extension_motifs(int(rng.integers(3, 10)), (2, 3, 4), 5, 70 + j)
        delta = int(rng.integers(5, 150))
        og = OracleGraph(s, d, t, n)
        graphs.append(api.Graph(s, d, t, n))
        trees.append(api.Tree(ms, delta))
        want.append(np.array([og.count(x, delta) for x in ms], dtype=np.uint64))
    m = api.Model(seed=4)
    say("learned batch")
    b = api.Batch(graphs, trees, model=m)
    assert b.info()["learned"] == 1
    for _ in range(3):
        for a, w in zip(b.count(), want):
            assert np.array_equal(a, w)


def _steep_model(scale=40.0):
    """A model whose prediction grows steeply with the root's whole-list window
    count (feature 8), so that a few segments are predicted to carry most of
    the cost and their roots are split into parts."""
    m = api.Model(seed=0)
    P = np.zeros_like(m.weights())
    P[8 * 64 + 0] = 1.0                       # W1[8][0]
    P[2048 + 64 + 0] = 1.0                    # W2[0][0]
    P[2048 + 64 + 4096 + 64 + 0] = 1.0        # W3[0][0]
    P[2048 + 64 + 2 * (4096 + 64)] = scale    # W4[0]
    m.set_weights(P)
    return m


def test_learned_split_roots_are_exact():
    """Heavy segments become per-root items and heavy roots become parts of
    their first-level candidates: counts, search statistics and the per-root
    cost log stay those of the plain schedule."""
    rng = np.random.default_rng(12)
    # a dense burst (600 edges in 30 time units) inside a sparse background:
    # the burst's roots have long whole-list windows, the rest short ones
    s1, d1, t1 = tiny_graph(rng, 40, 600, 30, self_loops=True)
    s2, d2, t2 = tiny_graph(rng, 40, 6000, 200_000, self_loops=True)
    s, d, t = np.concatenate([s1, s2]), np.concatenate([d1, d2]), np.concatenate([t1, t2 + 1000])
    ms = W.random_extension_motifs(20, (2, 3, 4), 5, 21)
    og = OracleGraph(s, d, t, 40)
    g = api.Graph(s, d, t, 40)
    m = _steep_model()
    for delta in (20, 90):
        tr = api.Tree(ms, delta)
        # the schedule this model makes really splits roots
        pred = m.predict(api.root_features(g, tr))
        live = api.root_features(g, tr)[:, 11] > 0
        c = np.where(live, np.exp(np.clip(pred, 0, 40)), 0.0)
        seg = np.add.reduceat(c, np.arange(0, len(c), 64))
        tot = seg.sum()
        heavy = (seg > 8 * tot / len(seg)) & (seg > tot / 32768)
        assert heavy.any() and (seg[heavy] / 64 > tot / 32768).any()
        want = np.array([og.count(x, delta) for x in ms], dtype=np.uint64)
        for sample in (1, 8):
            say("split roots", delta, sample)
            assert np.array_equal(api.count(g, tr, model=m, sample=sample), want)
        _, st_plain = api.count(g, tr, stats=True)
        _, st_learn = api.count(g, tr, stats=True, model=m, sample=1)
        assert st_plain == st_learn
        _, rc_plain = api.count(g, tr, root_cost=True)
        _, rc_learn = api.count(g, tr, root_cost=True, model=m, sample=1)
        assert np.array_equal(rc_plain, rc_learn)


def test_learned_batch_split_roots_are_exact():
    """The batch schedule from the steep model: heavy segments of the burst
    graph go first as single roots in parts, the rest in time order."""
    rng = np.random.default_rng(13)
    s1, d1, t1 = tiny_graph(rng, 40, 600, 30, self_loops=True)
    s2, d2, t2 = tiny_graph(rng, 40, 6000, 200_000, self_loops=True)
    burst = (np.concatenate([s1, s2]), np.concatenate([d1, d2]), np.concatenate([t1, t2 + 1000]))
    plain = tiny_graph(rng, 30, 3000, 5000, self_loops=True)
    graphs, trees, want = [], [], []
    for j, ((s, d, t), n) in enumerate([(burst, 40), (plain, 30), (burst, 40)]):
        ms = W.random_extension_motifs(12, (2, 3, 4), 5, 40 + j)
        delta = (20, 50, 90)[j]
        og = OracleGraph(s, d, t, n)
        graphs.append(api.Graph(s, d, t, n))
        trees.append(api.Tree(ms, delta))
        want.append(np.array([og.count(x, delta) for x in ms], dtype=np.uint64))
    say("learned batch, split roots")
    b = api.Batch(graphs, trees, model=_steep_model())
    assert b.info()["learned"] == 1
    for _ in range(3):
        for a, w in zip(b.count(), want):
            assert np.array_equal(a, w)
