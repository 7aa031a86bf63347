"""The library's host-side aggregation (fo_mdsc_aggregate_graph, no GPU) against the oracle's,
bit for bit, on mesh graphs and hand-made graphs, and its argument checks."""
import os
import re

import numpy as np
import pytest

from fo_inputs import config0_slab, ellipse_mesh, ExtrudedMesh, structured_box
from oracle import mdsc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2204_04321_amd", "libfo_stokes.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _csr(nbrs):
    ptr = np.zeros(len(nbrs) + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(l) for l in nbrs])
    idx = np.array([w for l in nbrs for w in l], dtype=np.int32)
    return ptr, idx


def _graphs():
    rng = np.random.default_rng(0)
    out = {}
    xy, tri = ellipse_mesh(700, 50e3, 30e3, rng)
    out["ellipse_wedge"] = mdsc.plane_graph(ExtrudedMesh("wedge", xy, tri, np.ones(len(xy)), np.ones(len(xy)),
                                                         np.ones(len(xy)), np.linspace(0, 1, 3)))
    m, _ = config0_slab()
    out["slab_hex"] = mdsc.plane_graph(m)
    xy, cells, sig = structured_box(9, 7, 2, 1.0, 1.0, elem="wedge")
    out["box_wedge"] = mdsc.plane_graph(ExtrudedMesh("wedge", xy, cells, np.ones(len(xy)), np.ones(len(xy)),
                                                     np.ones(len(xy)), sig))
    # random symmetric graph with isolated vertices sprinkled in
    n = 300
    adj = [set([v]) for v in range(n)]
    for _ in range(500):
        a, b = rng.integers(0, n, 2)
        if a % 7 and b % 7:
            adj[a].add(int(b))
            adj[b].add(int(a))
    out["random_isolated"] = [sorted(s) for s in adj]
    out["all_isolated"] = [[v] for v in range(21)]
    return out


@pytest.mark.parametrize("name", ["ellipse_wedge", "slab_hex", "box_wedge", "random_isolated", "all_isolated"])
def test_aggregation_matches_the_oracle(name):
    from paper_2204_04321_amd import aggregate_graph
    nbrs = _graphs()[name]
    # every level of the hierarchy, as the preconditioner builds it
    while True:
        want, n_want = mdsc.aggregate(nbrs)
        got, n_got = aggregate_graph(*_csr(nbrs))
        assert n_got == n_want and np.array_equal(got, want), name
        if len(nbrs) <= mdsc.COARSEST_MAX:
            break
        nbrs = mdsc.coarse_graph(nbrs, want, n_want)


def test_aggregation_rejects_malformed_graphs():
    from paper_2204_04321_amd import aggregate_graph
    from paper_2204_04321_amd._lib import FoError
    bad = {
        "missing from its own list": ([0, 1, 2], [1, 0]),
        "sorted": ([0, 2, 4], [1, 0, 0, 1]),
        "out of range": ([0, 2, 4], [0, 5, 0, 1]),
        "empty list": ([0, 1, 1], [0]),
        "ptr[0]": ([1, 2, 3], [0, 0, 1]),
    }
    for msg, (ptr, idx) in bad.items():
        with pytest.raises(FoError, match=re.escape(msg)):
            aggregate_graph(np.array(ptr), np.array(idx))


def test_icesheet_aggregation_matches_the_oracle():
    """The ice-sheet configuration's base graph (125k vertices): every level bit for bit."""
    from fo_inputs import config1_icesheet
    from paper_2204_04321_amd import aggregate_graph
    m, _ = config1_icesheet()
    nbrs = mdsc.plane_graph(m)
    sizes = []
    while len(nbrs) > mdsc.COARSEST_MAX:
        want, n_want = mdsc.aggregate(nbrs)
        got, n_got = aggregate_graph(*_csr(nbrs))
        assert n_got == n_want and np.array_equal(got, want), len(nbrs)
        sizes.append(len(nbrs))
        nbrs = mdsc.coarse_graph(nbrs, want, n_want)
    assert sizes[0] == m.n_verts and len(sizes) >= 3
