"""Host logic of the device hierarchy, checked on the CPU: build_levels()
(coloring, color-major permutation, sliced-ELL storage, restriction, and the
two symbolic Galerkin plans of Eq. gca) is compiled with a small driver that
replays both plans row by row as the device does, from A_0 in the library's
storage, and decodes every level back to natural CSR.  Each level must equal
the oracle's P_l^T A_l P_l (all of its nonzeros inside the symbolic pattern,
values to rounding), and each color class must be an independent set.  The
sliced-ELL layout of the per-color launches and the one-workgroup tail's
record layout are checked the same way: one Gauss-Seidel sweep replayed from
each (ascending and descending color order) must equal the oracle's
multicolor sweep on that level; the restriction and prolongation layouts
must give P^T r and x + P e."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import ROOT
import synth
from oracle import assemble as AS, hierarchy as OH, vcycle as OV

CSRC = os.path.join(ROOT, "paper_2104_13755_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host", "galerkin_plan_driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path_factory.mktemp("plans") / "driver"
    subprocess.run([cxx, "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC, DRIVER,
                    os.path.join(CSRC, "hier.cpp"), "-o", str(exe)], check=True, capture_output=True, timeout=180)
    return str(exe)


def _ell3(P):
    P = P.tocsr()
    n = P.shape[0]
    cols = -np.ones((n, 3), dtype=np.int32)
    w = np.zeros((n, 3))
    cnt = np.diff(P.indptr)
    for s in range(3):
        m = cnt > s
        cols[m, s] = P.indices[P.indptr[:-1][m] + s]
        w[m, s] = P.data[P.indptr[:-1][m] + s]
    return cols, w


def _run(driver, tmp_path, A, Ps, lpr, sort_rows, xb, ecs):
    sizes = [A.shape[0]] + [P.shape[1] for P in Ps]
    A = A.tocsr()
    A.sort_indices()
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        np.array([len(sizes), lpr, sort_rows], dtype=np.int32).tofile(f)
        np.array(sizes, dtype=np.int32).tofile(f)
        for P in Ps:
            c, w = _ell3(P)
            c.tofile(f)
            w.tofile(f)
        np.array([A.nnz], dtype=np.int32).tofile(f)
        A.indptr.astype(np.int32).tofile(f)
        A.indices.astype(np.int32).tofile(f)
        A.data.astype(np.float64).tofile(f)
        for x0, b in xb:
            x0.astype(np.float64).tofile(f)
            b.astype(np.float64).tofile(f)
        for e in ecs:
            e.astype(np.float64).tofile(f)
    r = subprocess.run([driver, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(out, "rb").read()
    o, levels = 0, []
    for n in sizes:
        nnz, ncol = np.frombuffer(raw, np.int32, 2, o)
        o += 8
        ptr = np.frombuffer(raw, np.int32, n + 1, o); o += 4 * (n + 1)
        idx = np.frombuffer(raw, np.int32, nnz, o); o += 4 * nnz
        val = np.frombuffer(raw, np.float64, nnz, o); o += 8 * nnz
        col = np.frombuffer(raw, np.int32, n, o); o += 4 * n
        levels.append((sp.csr_matrix((val, idx, ptr), shape=(n, n)), int(ncol), col))
    sweeps = []
    for n in sizes[:-1]:
        grp, nuni = (int(v) for v in np.frombuffer(raw, np.int32, 2, o))
        o += 8
        xa = np.frombuffer(raw, np.float64, n, o); o += 8 * n
        xd = np.frombuffer(raw, np.float64, n, o); o += 8 * n
        ya = np.frombuffer(raw, np.float64, n, o); o += 8 * n
        yd = np.frombuffer(raw, np.float64, n, o); o += 8 * n
        sweeps.append((grp, nuni, xa, xd, ya, yd))
    transfers = []
    for n, nc in zip(sizes[:-1], sizes[1:]):
        rc = np.frombuffer(raw, np.float64, nc, o); o += 8 * nc
        xp = np.frombuffer(raw, np.float64, n, o); o += 8 * n
        transfers.append((rc, xp))
    assert o == len(raw)
    return levels, sweeps, transfers


def _meshes():
    rng = np.random.default_rng(21)
    yield "icosphere", synth.small_icosphere(4, seed=5, sigma=0.01), 3
    yield "torus", synth.torus_grid(64, 24, 1.0, 0.3, rng, jitter=0.2), 4
    yield "disc", synth.flat_disc(41, 37, seed=3, jitter=0.1), 4


@pytest.mark.parametrize("lpr,sort_rows", [(0, 4096), (1, 0), (8, 100000), (2, 4096)])
def test_plans_replay_to_the_oracle_galerkin(driver, tmp_path, lpr, sort_rows):
    uniform = 0
    for name, (V, F), nl in _meshes():
        A, _, _ = AS.system(V, F, 1e-2)
        Ps, _, _ = OH.prolongations(V, F, n_levels=nl)
        rng = np.random.default_rng(77)
        xb = [(rng.uniform(-1, 1, P.shape[0]), rng.uniform(-1, 1, P.shape[0])) for P in Ps]
        ecs = [rng.uniform(-1, 1, P.shape[1]) for P in Ps]
        levels, sweeps, transfers = _run(driver, tmp_path, A, Ps, lpr, sort_rows, xb, ecs)
        for l, (rc, xp) in enumerate(transfers):
            ro = Ps[l].T @ xb[l][0]
            assert abs(rc - ro).max() <= 1e-14 * abs(ro).max(), (name, l)
            xo = xb[l][0] + Ps[l] @ ecs[l]
            assert abs(xp - xo).max() <= 1e-14 * abs(xo).max(), (name, l)
        O = OV.Solver(Ps, A)
        uniform += sum(sw[1] for sw in sweeps)
        for l, (grp, _, xa, xd, ya, yd) in enumerate(sweeps):
            assert grp in (1, 2, 4)
            for desc, xg in ((False, xa), (True, xd), (False, ya), (True, yd)):
                xo = O.relax(l, xb[l][0][:, None].copy(), xb[l][1][:, None], 1, descending=desc)[:, 0]
                assert abs(xg - xo).max() <= 1e-12 * abs(xo).max(), (name, l, desc)
        Al = A.tocsr()
        for l, (G, ncol, col) in enumerate(levels):
            if l > 0:
                Al = OH.galerkin(Al, Ps[l - 1]).tocsr()
            scale = abs(Al).max()
            # every oracle nonzero lies in the symbolic pattern; values agree everywhere on it
            inside = sp.csr_matrix((np.ones(G.nnz), G.indices, G.indptr), shape=G.shape)
            outside = abs(Al) - abs(Al).multiply(inside)
            assert outside.nnz == 0 or abs(outside).max() == 0.0, (name, l)
            diff = G - Al
            assert abs(diff).max() <= 1e-13 * scale, (name, l, abs(diff).max() / scale)
            if l + 1 < len(levels):
                # colors: 0..ncol-1, no edge of the pattern inside one color
                assert col.min() == 0 and col.max() == ncol - 1
                rows = np.repeat(np.arange(G.shape[0]), np.diff(G.indptr))
                off = rows != G.indices
                assert not np.any(col[rows[off]] == col[G.indices[off]]), (name, l)
            else:
                assert (col == -1).all()
    assert uniform > 0   # colors of uniform width were replayed through their own offsets
