"""Pins of the oracle's A = M + t L assembly (closed forms, invariants)."""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN
import synth
from oracle import assemble as AS


def _golden():
    with open(os.path.join(GOLDEN, "cotan_closed_forms.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"][:30])
def test_closed_form_triangles(case):
    V = np.array(case["V"])
    F = np.array(case["F"], dtype=np.int32)
    L = AS.laplacian(V, F)
    np.testing.assert_allclose(L.toarray(), np.array(case["L_dense"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(AS.mass(V, F), np.array(case["M_diag"]), rtol=1e-15)
    if "structural_nnz" in case:
        assert L.nnz == case["structural_nnz"]


def test_invariants_icosphere():
    V, F = synth.small_icosphere(3, seed=7, sigma=0.02)
    A, L, m = AS.system(V, F, 1e-2)
    n = len(V)
    assert abs(L @ np.ones(n)).max() < 1e-13
    assert abs(L - L.T).max() == 0.0
    ev = np.linalg.eigvalsh(L.toarray())
    assert ev.min() >= -1e-12 * abs(ev).max()
    assert abs(m.sum() - AS.face_areas(V, F).sum()) < 1e-13
    assert np.linalg.eigvalsh(A.toarray()).min() > 0
    assert A.nnz == n + 2 * len(AS.edge_list(F))


def test_sphere_area_converges():
    areas = [AS.mass(*synth.icosphere_subdiv(lv)).sum() for lv in (2, 4, 6)]
    err = [abs(a - 4 * np.pi) for a in areas]
    assert err[0] > err[1] > err[2] and err[2] < 2e-3 * 4 * np.pi


def test_flat_linear_precision():
    V, F = synth.flat_disc(12, seed=3, jitter=0.15)
    L = AS.laplacian(V, F)
    interior = (np.abs(np.abs(V[:, 0]) - 1) > 1e-12) & (np.abs(np.abs(V[:, 1]) - 1) > 1e-12)
    for X in (V[:, 0], V[:, 1], 2 * V[:, 0] - 3 * V[:, 1] + 1):
        assert abs((L @ X)[interior]).max() < 1e-13


def test_edge_weights_and_mass_scale():
    V, F = synth.small_icosphere(2, seed=2)
    E = AS.edge_list(F)
    rng = np.random.default_rng(0)
    w = rng.uniform(0.5, 2.0, len(E))
    Lw = AS.laplacian(V, F, edge_weights=w, edges=E)
    L = AS.laplacian(V, F)
    for e in rng.choice(len(E), 20, replace=False):
        i, j = E[e]
        assert abs(Lw[i, j] - w[e] * L[i, j]) < 1e-15
    assert abs(Lw @ np.ones(len(V))).max() < 1e-13
    s = rng.uniform(0.5, 1.5, len(V))
    A, _, m = AS.system(V, F, 0.1, mass_scale=s)
    np.testing.assert_allclose(A.diagonal(), s * m + 0.1 * L.diagonal(), rtol=1e-14)
