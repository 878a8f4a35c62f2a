"""Seeded synthetic inputs: temporal graphs and motif sets.

This module only draws inputs.  It holds none of the counting arithmetic and is
the one piece of code shared by the oracle-side tests and the HIP path.

The paper evaluates on five real temporal graphs (its dataset table in the
evaluation-methodology section: 1.1M-66M vertices, temporal/static edge ratios
of 1.5-3.4, windows from milliseconds to one day) and on motif groups that are
only drawn in a figure.  Neither is available, so every workload here is a
seeded synthetic stand-in with that shape:

* ``uniform_graph``  -- src/dst uniform, no self-loops, integer timestamps
  uniform in ``[0, t_max)``, stably sorted by time.
* ``powerlaw_graph`` -- directed Chung-Lu degrees (Pareto weights with tail
  exponent ``gamma - 1``, capped at ``sqrt(E)``), per-source bursty timestamps
  (Pareto burst sizes, exponential gaps inside a burst) and destination reuse
  inside a burst, stably sorted by time.

Motif sets are ordered edge sequences written in first-appearance labelling:
edge 1 is ``(0, 1)`` and every newly seen vertex takes the next free id,
source before destination.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "uniform_graph",
    "powerlaw_graph",
    "extension_options",
    "enumerate_motifs",
    "random_extension_motifs",
    "Workload",
    "make_config",
    "CONFIG1_MOTIFS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# graphs
# --------------------------------------------------------------------------
def uniform_graph(n_nodes: int, n_edges: int, t_max: int, seed: int):
    """Uniform random directed temporal graph.

    src, dst ~ U{0..n_nodes-1} with dst redrawn while it equals src; t ~
    U{0..t_max-1}; edges stably sorted by t.  Returns (src int32, dst int32,
    t int64).
    """
    rng = _rng(seed)
    src = rng.integers(0, n_nodes, n_edges, dtype=np.int64)
    dst = rng.integers(0, n_nodes, n_edges, dtype=np.int64)
    bad = dst == src
    while bad.any():
        dst[bad] = rng.integers(0, n_nodes, int(bad.sum()), dtype=np.int64)
        bad = dst == src
    t = rng.integers(0, t_max, n_edges, dtype=np.int64)
    order = np.argsort(t, kind="stable")
    return (src[order].astype(np.int32), dst[order].astype(np.int32),
            t[order].astype(np.int64))


def _pareto_weights(rng, n, gamma, cap):
    u = rng.random(n)
    u = np.maximum(u, 1e-300)
    w = u ** (-1.0 / (gamma - 1.0))
    return np.minimum(w, cap)


def _draw_from_weights(rng, w, n, progress=None):
    """n i.i.d. draws of indices with probability proportional to w (the
    lookup runs in pieces, reporting each to ``progress``)."""
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    x = rng.random(n)
    idx = np.empty(n, dtype=np.int64)
    step = 1 << 24
    for a in range(0, n, step):
        idx[a:a + step] = np.searchsorted(cdf, x[a:a + step], side="right")
        if progress and n > step:
            progress("weighted draws %d/%d" % (min(n, a + step), n))
    return np.minimum(idx, len(w) - 1)


def powerlaw_graph(n_nodes: int, n_edges: int, gamma: float, span: int,
                   seed: int, gamma_in: float | None = None,
                   burst_alpha: float = 1.5, gap_mean: float = 30.0,
                   reuse_p: float = 0.5, burst_cap: int | None = None, progress=None):
    """Heavy-tailed bursty directed temporal graph (seeded).

    Recipe (a reading: the paper gives only the dataset statistics):

    1. Out- and in-weights are i.i.d. Pareto, ``w = U**(-1/(gamma-1))``
       capped at ``sqrt(n_edges)``.  Out-degrees are one multinomial draw of
       ``n_edges`` over the out-weights; edges are laid out grouped by source.
    2. Each source's edges are cut into bursts: burst lengths come from one
       stream of ``ceil(Pareto(x_m=1, burst_alpha))`` sizes (at most
       ``burst_cap`` when given) over the source-grouped edge order, and every
       source starts a new burst.
    3. A burst starts at ``U[0, span)``; inside it the gaps are
       ``Exp(gap_mean)``; ``t = floor(start + offset)`` clipped to
       ``[0, span)``.
    4. Every edge draws a fresh destination proportional to the in-weights
       (redrawn while it equals the source); inside a burst an edge reuses the
       previous edge's destination with probability ``reuse_p``.
    5. All edges are stably sorted by t.

    Returns (src int32, dst int32, t int64).  ``progress``, when given, is
    called with the name of each finished stage (large graphs take minutes).
    """
    say = progress or (lambda _msg: None)
    rng = _rng(seed)
    gamma_in = gamma if gamma_in is None else gamma_in
    cap = math.sqrt(n_edges)
    w_out = _pareto_weights(rng, n_nodes, gamma, cap)
    w_in = _pareto_weights(rng, n_nodes, gamma_in, cap)
    w_in = w_in[rng.permutation(n_nodes)]

    deg = rng.multinomial(n_edges, w_out / w_out.sum()).astype(np.int64)
    src = np.repeat(np.arange(n_nodes, dtype=np.int64), deg)
    E = n_edges
    say("degrees")

    # burst boundaries: a global Pareto size stream plus every source start
    sizes = []
    total = 0
    while total < E:
        s = np.ceil(np.maximum(rng.random(max(1024, E // 2)), 1e-300)
                    ** (-1.0 / burst_alpha)).astype(np.int64)
        if burst_cap is not None:
            np.minimum(s, burst_cap, out=s)
        sizes.append(s)
        total += int(s.sum())
    sizes = np.concatenate(sizes)
    bounds = np.cumsum(sizes)
    bounds = bounds[bounds < E]
    start_flag = np.zeros(E, dtype=bool)
    start_flag[0] = True
    start_flag[bounds] = True
    node_start = np.cumsum(deg)[:-1]
    node_start = node_start[node_start < E]
    start_flag[node_start] = True
    burst_id = np.cumsum(start_flag) - 1
    n_bursts = int(burst_id[-1]) + 1 if E else 0
    say("bursts")

    # timestamps
    bstart = rng.integers(0, span, n_bursts, dtype=np.int64).astype(np.float64)
    gaps = rng.exponential(gap_mean, E)
    gaps[start_flag] = 0.0
    c = np.cumsum(gaps)
    first_idx = np.flatnonzero(start_flag)
    offset = c - c[first_idx][burst_id]
    t = np.floor(bstart[burst_id] + offset).astype(np.int64)
    np.clip(t, 0, span - 1, out=t)
    say("timestamps")

    # destinations
    fresh = _draw_from_weights(rng, w_in, E, say)
    bad = fresh == src
    while bad.any():
        fresh[bad] = _draw_from_weights(rng, w_in, int(bad.sum()))
        bad = fresh == src
    reuse = rng.random(E) < reuse_p
    reuse[start_flag] = False
    idx = np.where(reuse, 0, np.arange(E, dtype=np.int64))
    np.maximum.accumulate(idx, out=idx)
    dst = fresh[idx]
    say("destinations")

    order = np.argsort(t, kind="stable")
    say("time order")
    return (src[order].astype(np.int32), dst[order].astype(np.int32),
            t[order].astype(np.int64))


# --------------------------------------------------------------------------
# motifs
# --------------------------------------------------------------------------
def extension_options(motif, max_nodes: int, connected: bool = True):
    """All edges that may follow ``motif`` in first-appearance labelling.

    With ``connected`` the new edge touches an existing vertex (prefix
    connected); otherwise an edge between two new vertices is allowed too.
    """
    nv = 1 + max(max(u, v) for u, v in motif)
    opts = [(x, y) for x in range(nv) for y in range(nv) if x != y]
    if nv < max_nodes:
        opts += [(x, nv) for x in range(nv)] + [(nv, x) for x in range(nv)]
    if not connected and nv + 1 < max_nodes:
        opts.append((nv, nv + 1))
    return opts


def enumerate_motifs(k: int, max_nodes: int, connected: bool = True):
    """Every k-edge motif on <= max_nodes vertices, in first-appearance form.

    ``connected=True`` gives the prefix-connected ones (every edge touches an
    earlier one); ``connected=False`` gives all of them.
    """
    out = []

    def rec(m):
        if len(m) == k:
            out.append(tuple(m))
            return
        for e in extension_options(m, max_nodes, connected):
            rec(m + [e])

    rec([(0, 1)])
    return out


def random_extension_motifs(n: int, k_choices, max_nodes: int, seed: int):
    """``n`` distinct prefix-connected motifs from seeded extension walks."""
    rng = _rng(seed)
    seen, out = set(), []
    tries = 0
    while len(out) < n and tries < 100000:
        tries += 1
        k = int(rng.choice(k_choices))
        m = [(0, 1)]
        while len(m) < k:
            opts = extension_options(m, max_nodes, True)
            m.append(opts[int(rng.integers(0, len(opts)))])
        m = tuple(m)
        if m not in seen:
            seen.add(m)
            out.append(m)
    return out


# config 1's group: the path A->B, B->C and its three 3-edge extensions
CONFIG1_MOTIFS = [
    ((0, 1), (1, 2)),
    ((0, 1), (1, 2), (2, 0)),
    ((0, 1), (1, 2), (2, 3)),
    ((0, 1), (1, 2), (2, 1)),
]


@dataclass
class Workload:
    name: str
    graphs: list = field(default_factory=list)   # [(src, dst, t, n_nodes)]
    motif_sets: list = field(default_factory=list)  # one motif list per graph
    deltas: list = field(default_factory=list)   # one delta per graph (or per tree)
    note: str = ""


def make_config(k: int, scale: float = 1.0, progress=None) -> Workload:
    """The five synthetic workloads; ``scale`` shrinks edge and node counts;
    ``progress`` is passed to the graph generator."""
    def sc(x):
        return max(16, int(round(x * scale)))

    if k == 1:
        V, E = sc(2000), sc(20000)
        g = uniform_graph(V, E, 1_000_000, seed=1)
        return Workload("uniform V=%d E=%d delta=10000, 4 path motifs" % (V, E),
                        [(*g, V)], [list(CONFIG1_MOTIFS)], [10_000])
    if k == 2:
        V, E = sc(1_000_000), sc(20_000_000)
        g = powerlaw_graph(V, E, 2.1, 30_000_000, seed=2, progress=progress)
        return Workload(
            "powerlaw V=%d E=%d gamma=2.1 span=3e7 delta=3600, 36 motifs" % (V, E),
            [(*g, V)], [enumerate_motifs(3, 3)], [3600])
    if k == 3:
        rng = _rng(3)
        graphs, msets, deltas = [], [], []
        for gi in range(64):
            E = int(round(math.exp(rng.uniform(math.log(1e4), math.log(2e6)))))
            gam = float(rng.uniform(1.9, 2.5))
            dl = int(rng.choice([600, 3600, 86400]))
            nm = int(rng.integers(4, 25))
            E = sc(E)
            V = max(16, E // 10)
            # burst sizes capped at 64, as for config 4 (day-long windows over
            # uncapped Pareto bursts explode combinatorially)
            g = powerlaw_graph(V, E, gam, 30_000_000, seed=3000 + gi, burst_cap=64)
            graphs.append((*g, V))
            msets.append(random_extension_motifs(nm, (2, 3, 4), 5, 3000 + gi))
            deltas.append(dl)
        return Workload("64 powerlaw graphs, E log-uniform 1e4-2e6", graphs,
                        msets, deltas)
    if k == 4:
        V, E = sc(5_000_000), sc(50_000_000)
        # burst sizes capped at 64 (calibration: uncapped Pareto bursts make a
        # few roots explode combinatorially for 4-edge motifs; with the cap the
        # top 1% of roots still hold most of the work)
        g = powerlaw_graph(V, E, 1.8, 30_000_000, seed=4, burst_cap=64, progress=progress)
        ms = enumerate_motifs(3, 4) + enumerate_motifs(4, 4)
        return Workload(
            "powerlaw V=%d E=%d gamma=1.8 delta=7200, 756 motifs" % (V, E),
            [(*g, V)], [ms], [7200])
    if k == 5:
        V, E = sc(20_000_000), sc(200_000_000)
        # burst sizes capped at 32 (5-edge motifs, windows up to 6 hours)
        g = powerlaw_graph(V, E, 2.0, 100_000_000, seed=5, burst_cap=32, progress=progress)
        ms = (random_extension_motifs(16, (3,), 5, 51)
              + random_extension_motifs(16, (4,), 5, 52)
              + random_extension_motifs(16, (5,), 5, 53))
        return Workload(
            "powerlaw V=%d E=%d gamma=2.0 span=1e8, 48 motifs, delta sweep" % (V, E),
            [(*g, V)], [ms], [900, 3600, 21600])
    raise ValueError("config must be 1..5")
