"""The multi-GPU design, simulated on the CPU (no second GPU exists here):
roots are sharded by time range, shard g holds the time slab [T_g, T_{g+1} +
delta] of the edge list and searches its own roots (t in [T_g, T_{g+1})) with
the CPU backend, and one sum all-reduce (gloo, two processes) of the count
vectors gives the unsharded count, which the oracle fixes."""
import os
import socket

import numpy as np
import pytest

from paper_2507_14813_amd import api, workloads as W
from oracle import OracleGraph

DELTA = 3600
MOTIFS = [[(0, 1), (1, 2)], [(0, 1), (1, 2), (2, 0)], [(0, 1), (1, 0), (0, 2)],
          [(0, 1), (2, 1), (1, 3)], [(0, 1), (0, 2), (0, 3), (3, 1)]]


def _graph():
    s, d, t = W.powerlaw_graph(2000, 30000, 2.1, 300_000, seed=77)
    return s, d, np.asarray(t, np.int64), 2000


def _bounds(t, n_shards):
    # time boundaries with equal root counts
    q = np.quantile(t, np.linspace(0, 1, n_shards + 1)).astype(np.int64)
    q[0], q[-1] = t.min(), t.max() + 1
    return q


def shard_counts(s, d, t, n, bounds, shards):
    total = np.zeros(len(MOTIFS), np.uint64)
    for gi in shards:
        lo, hi = bounds[gi], bounds[gi + 1]
        idx = np.flatnonzero((t >= lo) & (t <= hi + DELTA))   # the shard's time slab
        g = api.Graph(s[idx], d[idx], t[idx], n, sorted_by_t=True, host_only=True)
        roots = np.flatnonzero(t[idx] < hi)                   # its roots, in slab positions
        total += api.count_cpu(g, api.Tree(MOTIFS, DELTA), roots=roots)
    return total


def _rank(rank, world, port, n_shards, out):
    import torch
    import torch.distributed as dist
    os.environ.update(MASTER_ADDR="127.0.0.1", MASTER_PORT=str(port))
    dist.init_process_group("gloo", rank=rank, world_size=world)
    s, d, t, n = _graph()
    bounds = _bounds(t, n_shards)
    mine = shard_counts(s, d, t, n, bounds, range(rank, n_shards, world))
    v = torch.from_numpy(mine.astype(np.int64))
    dist.all_reduce(v, op=dist.ReduceOp.SUM)
    if rank == 0:
        out.put(v.numpy().astype(np.uint64).tolist())
    dist.destroy_process_group()


def test_time_sharded_counts_sum_to_the_whole():
    s, d, t, n = _graph()
    og = OracleGraph(s, d, t, n)
    want = np.array([og.count(m, DELTA) for m in MOTIFS], np.uint64)
    og.close()
    assert want.sum() > 0
    for n_shards in (1, 3, 7):
        got = shard_counts(s, d, t, n, _bounds(t, n_shards), range(n_shards))
        assert np.array_equal(got, want), n_shards


def test_shards_over_two_processes_all_reduce():
    import torch.multiprocessing as mp
    with socket.socket() as sk:
        sk.bind(("127.0.0.1", 0))
        port = sk.getsockname()[1]
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    procs = [ctx.Process(target=_rank, args=(r, 2, port, 4, q)) for r in range(2)]
    for p in procs:
        p.start()
    got = np.array(q.get(timeout=300), np.uint64)
    for p in procs:
        p.join(timeout=120)
        assert p.exitcode == 0
    s, d, t, n = _graph()
    og = OracleGraph(s, d, t, n)
    want = np.array([og.count(m, DELTA) for m in MOTIFS], np.uint64)
    og.close()
    assert np.array_equal(got, want)
