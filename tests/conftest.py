import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP path)")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def golden_examples():
    with open(os.path.join(GOLDEN, "examples.json")) as f:
        return json.load(f)["examples"]


def edges_of(ex):
    e = np.array(ex["edges"], dtype=np.int64).reshape(-1, 3)
    return (e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.int64),
            int(ex["n_nodes"]))


def tiny_graph(rng, n_nodes, n_edges, t_max, self_loops=False):
    """Small random temporal graph with many tied timestamps."""
    s = rng.integers(0, n_nodes, n_edges)
    d = rng.integers(0, n_nodes, n_edges)
    if not self_loops:
        d = np.where(d == s, (d + 1) % n_nodes, d)
    t = rng.integers(0, t_max + 1, n_edges)
    return s.astype(np.int32), d.astype(np.int32), t.astype(np.int64)
