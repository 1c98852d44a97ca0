"""Host-side checks of libsmg (no GPU): the C ABI loads and exports every
declared symbol; the host precompute (successive self-parameterization,
coloring) matches the oracle's independent implementation."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import ROOT
import synth
from oracle import assemble as AS, hierarchy as OH


def _declared():
    src = open(os.path.join(ROOT, "include", "smg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_2104_13755_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.SIGNATURES) >= set(names)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2104_13755_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def _p_matrix(cols, w, shape):
    n = len(cols)
    m = w > 0
    return sp.csr_matrix((w[m], (np.repeat(np.arange(n), 3).reshape(n, 3)[m], cols[m])), shape=shape)


@pytest.mark.parametrize("mesh", ["icosphere", "torus", "disc", "heightfield", "torus-100k"])
def test_precompute_matches_oracle(mesh):
    from paper_2104_13755_amd.solver import Hierarchy
    rng = np.random.default_rng(8)
    if mesh == "icosphere":
        V, F = synth.small_icosphere(4, seed=12, sigma=0.01)
    elif mesh == "torus":
        V, F = synth.torus_grid(80, 30, 1.0, 0.3, rng, jitter=0.2)
    elif mesh == "torus-100k":
        V, F = synth.torus_grid(400, 250, 1.0, 0.3, rng, jitter=0.2)
    elif mesh == "disc":
        V, F = synth.flat_disc(45, 39, seed=6, jitter=0.1)
    else:
        V, F = synth.disc_grid(50, 47, rng, 0.1, height=lambda x, y: 0.1 * np.sin(3 * x) * np.cos(2 * y))
    h = Hierarchy.build(V, F, n_levels=4)
    Ps, _, st = OH.prolongations(V, F, n_levels=4)
    assert h.sizes == [len(V)] + [P.shape[1] for P in Ps]
    for l, P in enumerate(Ps):
        c, w = h.prolongation(l)
        Pp = _p_matrix(c, w, P.shape)
        assert ((Pp != 0) != (P != 0)).nnz == 0
        assert abs(Pp - P).max() < 1e-12
        s = h.stats(l)
        for key in ("collapses", "interior", "one_boundary", "b_case1", "b_case2", "b_case3"):
            assert s[key] == st[l][key]


@pytest.mark.parametrize("collapses", ["interior", "straight"])
def test_flat_closed_form_product(collapses):
    """Product SSP on the flat disc with interior-only collapses, and with
    boundary-edge collapses on the straight sides too, reproduces linear
    functions exactly (the planar closed form), picks the third boundary case
    for every boundary collapse, and equals the oracle's P under the same
    restriction (structure, values to 1e-12)."""
    from paper_2104_13755_amd.solver import Hierarchy
    V, F = synth.flat_disc(32, seed=11, jitter=0.1)
    h = Hierarchy.build(V, F, n_levels=2, collapses=collapses)
    c, w = h.prolongation(0)
    Vc_ref, _, Pc, Pw, st = OH.native.ssp_level(V, F, OH.next_target(len(V)), collapses)
    P = _p_matrix(c, w, (len(V), h.sizes[1]))
    assert abs(P @ Vc_ref[:, :2] - V[:, :2]).max() < 1e-13
    s = h.stats(0)
    assert s["b_case1"] == s["b_case2"] == s["one_boundary"] == 0
    assert (s["b_case3"] > 20) == (collapses == "straight")
    for key in ("collapses", "interior", "b_case3"):
        assert s[key] == st[key]
    mask = Pw > 0
    rows = np.repeat(np.arange(len(V)), 3).reshape(-1, 3)[mask]
    Po = sp.csr_matrix((Pw[mask], (rows, Pc[mask])), shape=P.shape)
    assert ((P != 0) != (Po != 0)).nnz == 0 and abs(P - Po).max() < 1e-12


def test_hierarchy_save_load_round_trip(tmp_path):
    """smg_hier_save / smg_hier_load through the C ABI: sizes, every P_l and
    the decimation statistics come back bitwise; hierarchies without
    positions too; a truncated, altered or foreign file is refused."""
    import ctypes
    from paper_2104_13755_amd import _lib as L
    from paper_2104_13755_amd.solver import Hierarchy
    rng = np.random.default_rng(4)
    V, F = synth.disc_grid(40, 37, rng, 0.1, height=lambda x, y: 0.1 * np.sin(3 * x))
    h = Hierarchy.build(V, F, n_levels=4)
    path = tmp_path / "hier.smg"
    h.save(path)
    g = Hierarchy.load(path)
    assert g.sizes == h.sizes
    for l in range(h.num_levels - 1):
        c0, w0 = h.prolongation(l)
        c1, w1 = g.prolongation(l)
        assert np.array_equal(c0, c1) and np.array_equal(w0, w1)
        assert h.stats(l) == g.stats(l)
    # a hierarchy given as prolongations (no positions) round-trips as well
    e = Hierarchy.from_prolongations(h.sizes, *zip(*[h.prolongation(l) for l in range(h.num_levels - 1)]))
    e.save(tmp_path / "ext.smg")
    e2 = Hierarchy.load(tmp_path / "ext.smg")
    assert e2.sizes == h.sizes and np.array_equal(e2.prolongation(2)[1], h.prolongation(2)[1])
    lib = L.load()
    raw = path.read_bytes()
    bad = {"truncated": raw[:-9], "altered": raw[:100] + bytes([raw[100] ^ 1]) + raw[101:],
           "foreign": b"NOTAHIER" + raw[8:], "trailing": raw + b"x"}
    for name, data in bad.items():
        q = tmp_path / (name + ".smg")
        q.write_bytes(data)
        out = ctypes.c_void_p()
        st = lib.smg_hier_load(str(q).encode(), ctypes.byref(out))
        assert st == -1 and not out.value, name
    assert lib.smg_hier_load(str(tmp_path / "missing.smg").encode(), ctypes.byref(ctypes.c_void_p())) == -1


def test_coloring_matches_oracle():
    from paper_2104_13755_amd.solver import color_pattern
    V, F = synth.small_icosphere(4, seed=2)
    A, _, _ = AS.system(V, F, 1e-2)
    Ps, _, _ = OH.prolongations(V, F, n_levels=3)
    A1 = OH.galerkin(A, Ps[0])
    for M in (A, A1):
        col_o, nc_o = OH.coloring(M)
        col_p, nc_p = color_pattern(M.indptr, M.indices)
        assert nc_o == nc_p and np.array_equal(col_o, col_p)


def test_coloring_matches_hand_worked_cases():
    """The library's greedy coloring against the colorings worked out by hand
    from App. A's algorithm (the same fixtures that pin the oracle)."""
    import json
    from conftest import GOLDEN
    from paper_2104_13755_amd.solver import color_pattern
    with open(os.path.join(GOLDEN, "coloring_greedy.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        n = case["n"]
        e = np.array(case["edges"]).reshape(-1, 2)
        r = np.concatenate([np.arange(n), e[:, 0], e[:, 1]])
        c = np.concatenate([np.arange(n), e[:, 1], e[:, 0]])
        S = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
        S.sort_indices()
        col, nc = color_pattern(S.indptr, S.indices)
        assert np.asarray(col).tolist() == case["colors"], case["name"]
        assert nc == max(case["colors"]) + 1


def test_pattern_helpers_reject_bad_input():
    import ctypes
    from paper_2104_13755_amd import _lib as L
    from paper_2104_13755_amd._lib import SmgError
    from paper_2104_13755_amd.solver import color_pattern, mesh_pattern
    V, F = synth.flat_disc(6, seed=1)
    Fb = F.copy()
    Fb[2, 1] = -1
    with pytest.raises(SmgError, match="out of range"):
        mesh_pattern(len(V), Fb)
    rp, ci = mesh_pattern(len(V), F)
    lib = L.load()
    small = np.zeros(len(ci) - 1, dtype=np.int32)
    nnz = ctypes.c_int32(len(small))
    r = np.zeros(len(V) + 1, dtype=np.int32)
    F32 = np.ascontiguousarray(F, dtype=np.int32)
    st = lib.smg_mesh_pattern(len(V), F32.ctypes.data, len(F), r.ctypes.data, small.ctypes.data, ctypes.byref(nnz))
    assert st == -1 and "capacity" in lib.smg_last_error().decode()
    cb = ci.copy()
    cb[3] = len(V)
    with pytest.raises(SmgError, match="out of range"):
        color_pattern(rp, cb)


def test_mesh_pattern_matches_oracle():
    from paper_2104_13755_amd.solver import mesh_pattern
    V, F = synth.flat_disc(17, 23, seed=1)
    rp, ci = mesh_pattern(len(V), F)
    ip, ii = AS.pattern(len(V), F)
    assert np.array_equal(rp, ip) and np.array_equal(ci, ii)


def test_precompute_rejects_bad_input():
    from paper_2104_13755_amd.solver import Hierarchy
    from paper_2104_13755_amd._lib import SmgError
    V, F = synth.flat_disc(8, seed=0)
    Fb = F.copy()
    Fb[0, 0] = len(V) + 5
    with pytest.raises(SmgError, match="out of range"):
        Hierarchy.build(V, Fb, n_levels=2)
    Fd = F.copy()
    Fd[3, 2] = Fd[3, 0]
    with pytest.raises(SmgError, match="repeats a vertex"):
        Hierarchy.build(V, Fd, n_levels=2)
    Vn = V.copy()
    Vn[5, 1] = np.nan
    with pytest.raises(SmgError, match="non-finite"):
        Hierarchy.build(Vn, F, n_levels=2)


def test_solver_create_rejects_bad_pattern_before_any_device_call():
    """The level-0 pattern is checked on the host first (these calls never
    reach the HIP runtime)."""
    import ctypes
    from paper_2104_13755_amd import _lib as L
    from paper_2104_13755_amd.solver import Hierarchy, mesh_pattern
    V, F = synth.flat_disc(10, seed=1)
    h = Hierarchy.build(V, F, n_levels=2)
    rp, ci = mesh_pattern(len(V), F)
    lib = L.load()
    cases = []
    r = rp.copy(); r[0] = 1; cases.append((r, ci, "rowptr"))
    r = rp.copy(); r[3] = r[2] - 1; cases.append((r, ci, "monotone"))
    c = ci.copy(); c[5] = len(V); cases.append((rp, c, "out of range"))
    c = ci.copy(); c[rp[4]], c[rp[4] + 1] = c[rp[4] + 1], c[rp[4]]; cases.append((rp, c, "ascending"))
    for r, c, msg in cases:
        r = np.ascontiguousarray(r, dtype=np.int32)
        c = np.ascontiguousarray(c, dtype=np.int32)
        out = ctypes.c_void_p()
        st = lib.smg_solver_create(0, h._h, r.ctypes.data, c.ctypes.data, None, ctypes.byref(out))
        assert st == -1 and not out.value, msg
        assert msg in lib.smg_last_error().decode()


def test_solver_create_rejects_an_oversized_coarsest_level():
    """A coarsest level above the dense factorization's limit (16384 rows)
    is refused on the host, before any allocation or device call."""
    import ctypes
    from paper_2104_13755_amd import _lib as L
    from paper_2104_13755_amd.solver import Hierarchy
    n = 16385
    h = Hierarchy.from_prolongations([n], [], [])
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    lib = L.load()
    out = ctypes.c_void_p()
    st = lib.smg_solver_create(0, h._h, rp.ctypes.data, ci.ctypes.data, None, ctypes.byref(out))
    assert st == -1 and not out.value
    assert "16384" in lib.smg_last_error().decode()


def test_external_prolongations_are_validated():
    from paper_2104_13755_amd.solver import Hierarchy
    from paper_2104_13755_amd._lib import SmgError
    cols = np.array([[0, 1, -1], [1, -1, -1], [0, 1, -1], [1, 0, -1]], dtype=np.int32)
    w = np.array([[0.5, 0.5, 0], [1, 0, 0], [0.25, 0.75, 0], [0.6, 0.4, 0]])
    h = Hierarchy.from_prolongations([4, 2], [cols], [w])
    c, ww = h.prolongation(0)
    assert np.array_equal(c, cols) and np.array_equal(ww, w)
    for bad_c, bad_w, msg in [(cols, np.where(cols >= 0, -0.5, 0.0), "out of range"),
                              (np.where(cols == 1, 2, cols).astype(np.int32), w, "out of range"),
                              (cols, np.where(cols >= 0, np.inf, 0.0), "out of range"),
                              (cols, np.vstack([w[:3], np.zeros(3)]), "no positive weight")]:
        with pytest.raises(SmgError, match=msg):
            Hierarchy.from_prolongations([4, 2], [bad_c], [bad_w])
    with pytest.raises(SmgError, match="empty level"):
        Hierarchy.from_prolongations([0], [], [])
    with pytest.raises(SmgError, match="bad level"):
        h.prolongation(1)


def _host_dirichlet(h, A, known):
    """smg_hier_dirichlet + smg_dirichlet_pattern, called straight through the
    C ABI (both are host-only)."""
    import ctypes
    from paper_2104_13755_amd import _lib as L
    from paper_2104_13755_amd.solver import Hierarchy
    lib = L.load()
    n = A.shape[0]
    kn = np.ascontiguousarray(known, dtype=np.uint8)
    uidx = np.zeros(n, dtype=np.int32)
    nu = ctypes.c_int32()
    hh = ctypes.c_void_p()
    L.check(lib.smg_hier_dirichlet(h._h, kn.ctypes.data, ctypes.byref(hh), uidx.ctypes.data, ctypes.byref(nu)),
            "hier_dirichlet")
    rp = np.ascontiguousarray(A.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.indices, dtype=np.int32)
    urp = np.zeros(n + 1, dtype=np.int32)
    uci = np.zeros(len(ci), dtype=np.int32)
    nu2, nnz = ctypes.c_int32(), ctypes.c_int32()
    L.check(lib.smg_dirichlet_pattern(n, rp.ctypes.data, ci.ctypes.data, kn.ctypes.data, urp.ctypes.data,
                                      uci.ctypes.data, ctypes.byref(nu2), ctypes.byref(nnz)), "dirichlet_pattern")
    assert nu2.value == nu.value
    return Hierarchy(hh), uidx[:nu.value], urp[:nu.value + 1], uci[:nnz.value]


@pytest.mark.parametrize("which", ["none", "rim", "random60", "random85"])
def test_dirichlet_host_reduction_matches_oracle(which):
    """App. B on the host: the unknowns, the reduced hierarchy (P_{u:}, zero
    columns removed level by level) and the A_uu pattern equal the oracle's,
    bitwise."""
    from oracle import dirichlet as DR
    from paper_2104_13755_amd.solver import Hierarchy
    V, F = synth.flat_disc(31, 27, seed=5, jitter=0.1)
    n = len(V)
    A, _, _ = AS.system(V, F, 1e-2)
    A = A.tocsr()
    Ps, _, _ = OH.prolongations(V, F, n_levels=4)
    cols, ws = [], []
    for P in Ps:
        P = P.tocsr()
        c = -np.ones((P.shape[0], 3), dtype=np.int32)
        w = np.zeros((P.shape[0], 3))
        cnt = np.diff(P.indptr)
        for s in range(3):
            m = cnt > s
            c[m, s] = P.indices[P.indptr[:-1][m] + s]
            w[m, s] = P.data[P.indptr[:-1][m] + s]
        cols.append(c)
        ws.append(w)
    h = Hierarchy.from_prolongations([n] + [P.shape[1] for P in Ps], cols, ws)
    rng = np.random.default_rng(17)
    if which == "none":
        known = np.zeros(n, bool)
    elif which == "rim":
        known = np.zeros(n, bool)
        known[np.argsort(np.linalg.norm(V[:, :2], axis=1))[-n // 8:]] = True
    else:
        known = rng.uniform(size=n) < (0.6 if which == "random60" else 0.85)
    hr, u, urp, uci = _host_dirichlet(h, A, known)
    Auu, _, u_ref = DR.reduce(A, np.zeros(n), known, np.zeros(n))
    Pr = DR.prolongations(Ps, known)
    assert np.array_equal(u, u_ref)
    assert np.array_equal(urp, Auu.indptr) and np.array_equal(uci, Auu.indices)
    assert hr.sizes == [len(u)] + [P.shape[1] for P in Pr]
    for l, P in enumerate(Pr):
        Pp = _p_matrix(*hr.prolongation(l), P.shape)
        assert ((Pp != 0) != (P != 0)).nnz == 0, l
        assert abs(Pp - P).max() == 0.0, l


def test_dirichlet_all_known_is_an_error():
    from paper_2104_13755_amd._lib import SmgError
    from paper_2104_13755_amd.solver import Hierarchy
    V, F = synth.flat_disc(12, seed=2)
    A, _, _ = AS.system(V, F, 1e-2)
    h = Hierarchy.build(V, F, n_levels=2)
    with pytest.raises(SmgError):
        _host_dirichlet(h, A.tocsr(), np.ones(len(V), bool))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message (before
    touching any GPU)."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


@pytest.mark.parametrize("mesh", ["icosphere", "disc", "heightfield"])
def test_host_assembly_matches_oracle(mesh):
    """smg_pre_assemble (faces scattered one by one) against the oracle's
    cotangent Laplacian and lumped mass (vectorised numpy), on closed and
    bounded meshes: 1e-13 of the largest entry; bad input is refused."""
    import ctypes
    from paper_2104_13755_amd import _lib as L
    from paper_2104_13755_amd.solver import host_assemble
    rng = np.random.default_rng(8)
    if mesh == "icosphere":
        V, F = synth.small_icosphere(4, seed=3, sigma=0.01)
    elif mesh == "disc":
        V, F = synth.flat_disc(40, seed=4, jitter=0.1)
    else:
        V, F = synth.disc_grid(40, 38, rng, 0.1, height=lambda x, y: 0.1 * np.sin(3 * x) * np.cos(2 * y))
    rp, ci, lv, m = host_assemble(V, F)
    _, Lo, mo = AS.system(V, F, 1.0)
    assert np.array_equal(rp, Lo.indptr) and np.array_equal(ci, Lo.indices)
    assert abs(lv - Lo.data).max() < 1e-13 * abs(Lo.data).max()
    assert abs(m - mo).max() < 1e-15 * mo.max()
    lib = L.load()
    Fb = np.ascontiguousarray(F.copy(), dtype=np.int32)
    Fb[3, 1] = len(V)
    out_l, out_m = np.zeros(len(ci)), np.zeros(len(V))
    Vc = np.ascontiguousarray(V)
    assert lib.smg_pre_assemble(Vc.ctypes.data, len(V), Fb.ctypes.data, len(F), rp.ctypes.data, ci.ctypes.data,
                                out_l.ctypes.data, out_m.ctypes.data) == -1
    rp2 = rp.copy()
    rp2[0] = 1
    assert lib.smg_pre_assemble(Vc.ctypes.data, len(V), np.ascontiguousarray(F, dtype=np.int32).ctypes.data, len(F),
                                rp2.ctypes.data, ci.ctypes.data, out_l.ctypes.data, out_m.ctypes.data) == -1
