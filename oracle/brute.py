"""Brute-force counter: the definition of a delta-temporal motif match, written
out directly (paper, section 2.1).  TEST INFRASTRUCTURE ONLY; tiny inputs.

A match of M = ((u_1,v_1),...,(u_k,v_k)) is a tuple of k edges with strictly
increasing timestamps, last minus first <= delta, and an injective vertex map
phi with phi(u_j) = src and phi(v_j) = dst for every j.  Every k-subset of the
edges is tried; a tuple with strictly increasing t is a subset listed in time
order, so subsets cover every candidate exactly once.
"""
from __future__ import annotations

import itertools


def is_match(edges, motif, delta):
    """edges: k (src, dst, t) triples in the order they are matched."""
    ts = [e[2] for e in edges]
    if any(not (a < b) for a, b in zip(ts, ts[1:])):
        return False
    if ts[-1] - ts[0] > delta:
        return False
    phi = {}
    for (s, d, _), (u, v) in zip(edges, motif):
        for mv, gv in ((u, s), (v, d)):
            if mv in phi and phi[mv] != gv:
                return False
            phi[mv] = gv
    return len(set(phi.values())) == len(phi)   # injective


def count(src, dst, t, motif, delta, roots=None):
    """Number of matches; ``roots`` restricts the first edge (positions in the
    stably time-sorted list)."""
    order = sorted(range(len(t)), key=lambda i: (int(t[i]), i))
    E = [(int(src[i]), int(dst[i]), int(t[i])) for i in order]
    k = len(motif)
    allowed = None if roots is None else set(int(r) for r in roots)
    c = 0
    for comb in itertools.combinations(range(len(E)), k):
        if allowed is not None and comb[0] not in allowed:
            continue
        if is_match([E[i] for i in comb], motif, delta):
            c += 1
    return c


def _sorted_edges(src, dst, t):
    order = sorted(range(len(t)), key=lambda i: (int(t[i]), i))
    return [(int(src[i]), int(dst[i]), int(t[i])) for i in order]


def partial_matches(E, motif, delta, root):
    """Every match of ``motif`` whose first edge is position ``root`` of the
    time-sorted edge list E, as a list of edge-position tuples (the definition
    applied to every subset of later edges)."""
    k = len(motif)
    out = []
    later = range(root + 1, len(E))
    for rest in itertools.combinations(later, k - 1):
        tup = (root,) + rest
        if is_match([E[i] for i in tup], motif, delta):
            out.append(tup)
    return out


def window_entries(src, dst, t, motif, delta):
    """Per root and per motif edge j >= 1: the number of list entries with
    t_prev < t <= t_first + delta summed over the matches of the first j edges
    from that root, where the list is chosen by the rule the oracle reads into
    Algorithm 1: the out-edges of the graph vertex bound to u_j if u_j is
    bound, else the in-edges of the vertex bound to v_j if v_j is bound, else
    every edge.  Lists hold every edge, self-loops included.  Returns an
    (n_edges x k) list of lists (column 0 stays 0)."""
    E = _sorted_edges(src, dst, t)
    k = len(motif)
    out = [[0] * k for _ in E]
    for r in range(len(E)):
        for j in range(1, k):
            for tup in partial_matches(E, motif[:j], delta, r):
                phi = {}
                for i, (u, v) in zip(tup, motif[:j]):
                    phi[u], phi[v] = E[i][0], E[i][1]
                t_prev, t_first = E[tup[-1]][2], E[tup[0]][2]
                u, v = motif[j]
                if u in phi:
                    lst = [e for e in E if e[0] == phi[u]]
                elif v in phi:
                    lst = [e for e in E if e[1] == phi[v]]
                else:
                    lst = E
                out[r][j] += sum(1 for e in lst if t_prev < e[2] <= t_first + delta)
    return out


def matches(src, dst, t, motif, delta):
    """Every match as a tuple of the caller's edge indices (the motif's edges
    in order), sorted: the definition applied to every k-subset of edges, as
    count does, with the edges listed instead of counted."""
    order = sorted(range(len(t)), key=lambda i: (int(t[i]), i))
    E = [(int(src[i]), int(dst[i]), int(t[i])) for i in order]
    out = []
    for comb in itertools.combinations(range(len(E)), len(motif)):
        if is_match([E[i] for i in comb], motif, delta):
            out.append(tuple(order[i] for i in comb))
    return sorted(out)
