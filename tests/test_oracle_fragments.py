"""Pins of the oracle's fragment labelling (connected components of the alive
springs, labelled by their smallest node id; detached = no node anchored at
t = 0) against independent facts: scipy's connected components, a brute-force
transitive closure, and hand-built graphs."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle as O
from paper_1302_3663_amd import synth


def min_id_labels(n, ij, alive):
    """Component labels from scipy, renamed to the smallest member id."""
    e = np.asarray(alive, bool)
    A = sp.coo_matrix((np.ones(e.sum()), (ij[0][e], ij[1][e])), shape=(n, n))
    k, lab = connected_components(A, directed=False)
    smallest = np.full(k, n)
    np.minimum.at(smallest, lab, np.arange(n))
    return smallest[lab], k


def closure_labels(n, ij, alive):
    """Brute force: reachability by repeated squaring of the adjacency."""
    R = np.eye(n, dtype=bool)
    for e in np.nonzero(np.asarray(alive, bool))[0]:
        R[ij[0][e], ij[1][e]] = R[ij[1][e], ij[0][e]] = True
    for _ in range(int(np.ceil(np.log2(max(n, 2)))) + 1):
        R = (R.astype(np.int64) @ R.astype(np.int64)) > 0
    return np.array([np.nonzero(R[s])[0].min() for s in range(n)])


def test_hand_built_graphs():
    # a chain 0-1-2-3 cut in the middle, an isolated node, a triangle 5-6-7
    ij = np.array([[0, 1, 2, 5, 6, 5], [1, 2, 3, 6, 7, 7]])
    alive = np.array([1, 0, 1, 1, 1, 1])
    anchored = np.array([0, 0, 0, 1, 0, 0, 0, 0])
    lab, nf, nd = O.fragments(ij, alive, anchored)
    assert lab.tolist() == [0, 0, 2, 2, 4, 5, 5, 5]
    assert nf == 4
    assert nd == 3          # only {2, 3} holds an anchored node
    # all springs broken: every node its own fragment
    lab, nf, nd = O.fragments(ij, np.zeros(6), np.zeros(8))
    assert lab.tolist() == list(range(8)) and nf == 8 and nd == 8


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_against_scipy_and_closure(seed):
    rng = np.random.default_rng(seed)
    n, m = 60, 90
    ij = np.sort(rng.integers(0, n, size=(2, m)), axis=0)
    ij = ij[:, ij[0] != ij[1]]
    alive = rng.random(ij.shape[1]) < 0.6
    anchored = (rng.random(n) < 0.1).astype(np.uint8)
    lab, nf, nd = O.fragments(ij, alive, anchored)
    ref, k = min_id_labels(n, ij, alive)
    assert np.array_equal(lab, ref) and nf == k
    assert np.array_equal(lab, closure_labels(n, ij, alive))
    detached = sum(1 for r in np.unique(lab) if not anchored[lab == r].any())
    assert nd == detached


def test_workload_graph_against_scipy():
    case = synth.tube_3d(seed=2)
    ij = case["ij"]
    n = case["X"].shape[1]
    rng = np.random.default_rng(5)
    alive = rng.random(ij.shape[1]) < 0.1       # heavy breakage: many fragments, some detached
    lab, nf, nd = O.fragments(ij, alive, O.anchored_nodes(dict(attach_axis=1, attach_dist=0.02), case["X"]))
    ref, k = min_id_labels(n, ij, alive)
    assert np.array_equal(lab, ref) and nf == k and nf > 10 and 0 < nd < nf
