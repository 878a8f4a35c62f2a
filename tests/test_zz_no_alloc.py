"""mg_count_noalloc (the count for callers that cannot allocate device memory)
against mg_count: the same counts and statistics, bit for bit, on two calls
in a row with a smaller input the second time, and no device allocation
during the call."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2507_14813_amd import api, workloads as W
from conftest import tiny_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def _raw_noalloc(g, tr, n_motifs, stats=False):
    """The entry point called directly through the C ABI."""
    L = api.lib()
    o = api.CountOpts()
    L.mg_count_opts_init(ctypes.byref(o))
    st = np.zeros(len(api.STAT_NAMES), np.uint64)
    if stats:
        o.stats = st.ctypes.data
    out = np.zeros(n_motifs, np.uint64)
    rc = L.mg_count_noalloc(g.handle, tr.handle, ctypes.byref(o), out.ctypes.data)
    assert rc == 0, L.mg_last_error()
    return out, st


def test_noalloc_matches_mg_count():
    import torch
    assert torch.cuda.is_available()
    rng = np.random.default_rng(11)
    big = W.make_config(2, scale=0.02)
    s, d, t, n = big.graphs[0]
    cases = [(s, d, t, n, big.motif_sets[0], big.deltas[0])]
    s2, d2, t2 = tiny_graph(rng, 30, 3000, 2000, self_loops=True)
    cases.append((s2, d2, t2, 30, W.random_extension_motifs(12, (2, 3, 4), 5, 4), 90))
    for s_, d_, t_, n_, ms, delta in cases:
        say("noalloc", "E=%d" % len(s_), "motifs=%d" % len(ms), "delta=%d" % delta)
        g = api.Graph(s_, d_, t_, n_)
        tr = api.Tree(ms, delta)
        with pytest.raises(api.MayuraError, match="MG_EINVAL"):
            api.count_noalloc(g, tr)            # no device tables yet
        want, want_st = api.count(g, tr, stats=True)
        torch.cuda.synchronize()
        before = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        got, st = _raw_noalloc(g, tr, len(ms), stats=True)
        got2 = api.count_noalloc(g, tr, chunk=128, queues=3)
        torch.cuda.synchronize()
        after = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        assert after == before
        assert np.array_equal(got, want) and np.array_equal(got2, want)
        assert {k: int(v) for k, v in zip(api.STAT_NAMES, st)} == want_st
        with pytest.raises(api.MayuraError, match="MG_EINVAL"):
            api.count_noalloc(g, tr, chunk=100)
