"""Pins of the oracle's greedy coloring (Alg. 'Graph Coloring', App. A)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import GOLDEN
import synth
from oracle import assemble as AS, hierarchy as H


def _graph(n, edges):
    e = np.array(edges).reshape(-1, 2)
    r = np.concatenate([np.arange(n), e[:, 0], e[:, 1]])
    c = np.concatenate([np.arange(n), e[:, 1], e[:, 0]])
    S = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    S.sort_indices()
    return S


def _cases():
    with open(os.path.join(GOLDEN, "coloring_greedy.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"][:25])
def test_hand_worked(case):
    col, nc = H.coloring(_graph(case["n"], case["edges"]))
    assert col.tolist() == case["colors"]
    assert nc == max(case["colors"]) + 1


def _valid(A, col):
    C = A.tocoo()
    off = C.row != C.col
    return np.all(col[C.row[off]] != col[C.col[off]])


def test_mesh_coloring_valid_deterministic():
    V, F = synth.small_icosphere(4, seed=1)
    A, _, _ = AS.system(V, F, 1e-3)
    col, nc = H.coloring(A)
    col2, nc2 = H.coloring(A)
    assert np.array_equal(col, col2) and nc == nc2
    assert _valid(A, col)
    maxdeg = int(np.diff(A.indptr).max()) - 1
    assert nc <= maxdeg + 1
    assert set(np.unique(col)) == set(range(nc))


def test_explicit_zero_entries_count_as_edges():
    # the square's diagonal has cotan weight exactly 0 but is a structural edge
    V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], dtype=float)
    F = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    L = AS.laplacian(V, F)
    assert L[0, 2] == 0.0
    col, _ = H.coloring(L)
    assert col[0] != col[2]
