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
