"""Pins of the oracle's adjoint gradients: dense-solve reference and central
finite differences with relative steps."""
import numpy as np
import pytest

import synth
from oracle import assemble as AS, grad as G, hierarchy as H, vcycle as VC


@pytest.fixture(scope="module")
def heat():
    w = synth.workload_c4(level=3)
    V, F = w["V"], w["F"]
    A, L, m = AS.system(V, F, w["t"])
    Ps, _, _ = H.prolongations(V, F, n_levels=3)
    return w, A, L, m, Ps


def test_mg_grads_match_dense(heat):
    w, A, L, m, Ps = heat
    S = VC.Solver(Ps, A)
    got = G.mg_grads(S, L, m, w["b"], w["w"][:, None], 1e-14)
    ref = G.dense_grads(A, L, m, w["b"], w["w"])
    for key in ("db", "ds"):
        assert np.linalg.norm(got[key] - ref[key]) / np.linalg.norm(ref[key]) < 1e-11
    assert abs(got["dt"] - ref["dt"]) / abs(ref["dt"]) < 1e-11


def test_fd_dt_and_ds(heat):
    w, A, L, m, Ps = heat
    t = w["t"]
    S = VC.Solver(Ps, A)
    ref = G.mg_grads(S, L, m, w["b"], w["w"][:, None], 1e-14)

    def loss(tt, s):
        Ak, _, _ = AS.system(w["V"], w["F"], tt, mass_scale=s)
        S.set_values(Ak)
        u, _, _ = S.solve(w["b"], 1e-14, 200)
        return float(w["w"] @ u[:, 0])

    ones = np.ones(len(m))
    h = 1e-6 * t
    fd = (loss(t + h, ones) - loss(t - h, ones)) / (2 * h)
    assert abs(fd - ref["dt"]) / abs(ref["dt"]) < 1e-6
    rng = np.random.default_rng(0)
    for i in list(w["sources"][:3]) + list(rng.choice(len(m), 3, replace=False)):
        e = np.zeros(len(m))
        e[i] = 1e-6
        fd = (loss(t, ones + e) - loss(t, ones - e)) / 2e-6
        assert abs(fd - ref["ds"][i]) <= 1e-6 * max(abs(ref["ds"][i]), 1e-3 * abs(ref["ds"]).max())
    S.set_values(A)
