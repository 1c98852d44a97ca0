"""Seeded workload recipes (meshes, scalars and random right-hand-side data).

Each recipe returns a dict.  Right-hand sides that involve the mass matrix
(``b = M u``) are returned as the random factor ``u`` together with
``rhs_kind``; the consumer applies its own mass matrix.
Draw order within a recipe: positions noise, then fields / weights, then RHS.
"""
import math
import numpy as np

from .meshes import (icosphere_subdiv, icosphere_freq, torus_grid, disc_grid,
                     mean_edge_length, edges_of)


def _radial_noise(V, rng, sigma):
    xi = rng.normal(0.0, 1.0, size=len(V))
    return V * (1.0 + sigma * xi)[:, None]


def small_icosphere(level, seed=0, sigma=0.01):
    rng = np.random.default_rng(seed)
    V, F = icosphere_subdiv(level)
    if sigma > 0:
        V = _radial_noise(V, rng, sigma)
    return V, F


def flat_disc(nx, ny=None, seed=0, jitter=0.1):
    rng = np.random.default_rng(seed)
    return disc_grid(nx, nx if ny is None else ny, rng, jitter)


def workload_c1():
    """Icosphere, 5 subdivisions (10,242 vertices), radial noise 0.01,
    A = M + 1e-3 L, b = M u with u ~ U[-1,1], 3 levels, rtol 1e-10."""
    rng = np.random.default_rng(1)
    V, F = icosphere_subdiv(5)
    V = _radial_noise(V, rng, 0.01)
    u = rng.uniform(-1.0, 1.0, size=(len(V), 1))
    return dict(name="icosphere-L5", V=V, F=F, t=1e-3, u=u, rhs_kind="mass",
                n_levels=3, rtol=1e-10)


def workload_c2(a=1000, b=1000):
    """Torus grid a x b (default 1,000,000 vertices), R = 1, r = 0.3, jitter
    0.2 grid spacings in parameter space, A = M + 1e-2 L, b = M X with X the
    vertex coordinates (3 RHS), 7 levels, rtol 1e-8."""
    rng = np.random.default_rng(2)
    V, F = torus_grid(a, b, 1.0, 0.3, rng, jitter=0.2)
    return dict(name=f"torus-{a}x{b}", V=V, F=F, t=1e-2, u=V.copy(),
                rhs_kind="mass", n_levels=7, rtol=1e-8)


def _c3_mesh(rng, kind, N):
    if kind == 0:  # noisy icosphere
        nu = max(2, int(round(math.sqrt((N - 2) / 10.0))))
        V, F = icosphere_freq(nu)
        V = _radial_noise(V, rng, 0.3 * mean_edge_length(V, F))
        return "icosphere", V, F
    if kind == 1:  # torus, a/b = R/r = 10/3
        bb = max(3, int(round(math.sqrt(N * 3.0 / 10.0))))
        aa = max(3, int(round(N / bb)))
        V, F = torus_grid(aa, bb, 1.0, 0.3, rng, jitter=0.2)
        return "torus", V, F
    s = max(3, int(round(math.sqrt(N))))
    V, F = disc_grid(s, s, rng, jitter=0.1)
    return "disc", V, F


def workload_c3(count=64, nmin=20000, nmax=300000, seed=3):
    """``count`` meshes of sizes U[nmin, nmax]: noisy icospheres, tori and flat
    discs (natural Neumann boundary); t ~ logU[1e-4, 1e-1]; 1-3 RHS per mesh,
    b ~ U[-1,1]; levels by the coarsest >= 500 rule; rtol 1e-8."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        N = int(rng.integers(nmin, nmax + 1))
        kind = int(rng.integers(0, 3))
        t = float(10.0 ** rng.uniform(-4.0, -1.0))
        k = int(rng.integers(1, 4))
        name, V, F = _c3_mesh(rng, kind, N)
        bvec = rng.uniform(-1.0, 1.0, size=(len(V), k))
        out.append(dict(name=name, V=V, F=F, t=t, b=bvec, rhs_kind="direct",
                        n_levels=0, rtol=1e-8))
    return out


def workload_c4(level=8, seed=4):
    """Heat step on a noisy icosphere (``level`` subdivisions; 8 gives 655,362
    vertices, 4 gives the 2,562-vertex subcase): radial noise 0.3 mean edge
    lengths, t = (mean edge length)^2, b = unit impulses at 16 distinct seeded
    sources, loss weights w ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    V, F = icosphere_subdiv(level)
    V = _radial_noise(V, rng, 0.3 * mean_edge_length(V, F))
    h = mean_edge_length(V, F)
    src = rng.choice(len(V), size=16, replace=False)
    w = rng.normal(0.0, 1.0, size=len(V))
    b = np.zeros((len(V), 1))
    b[src, 0] = 1.0
    return dict(name=f"icosphere-L{level}", V=V, F=F, t=h * h, b=b, w=w,
                sources=np.sort(src), rhs_kind="direct", n_levels=0, rtol=1e-8)


def _c5_height(x, y):
    return 0.1 * np.sin(3.0 * x) * np.cos(2.0 * y)


def workload_c5_mesh(nx=1415, ny=1414, seed=5):
    """Height-field disc z = 0.1 sin(3x) cos(2y) on a jittered nx x ny grid
    (2,000,810 vertices by default), b = M u with u ~ U[-1,1], 8 levels."""
    rng = np.random.default_rng(seed)
    V, F = disc_grid(nx, ny, rng, jitter=0.1, height=_c5_height)
    u = rng.uniform(-1.0, 1.0, size=(len(V), 1))
    return dict(name=f"disc-{nx}x{ny}", V=V, F=F, u=u, rhs_kind="mass",
                n_levels=8, rtol=1e-8, edges=edges_of(F))


def workload_c5_frame(mesh, k, seed=5):
    """Frame ``k``: per-edge weights w_e = 2^(sin(a x_e + phi) cos(b y_e + psi))
    at edge midpoints (values in [0.5, 2]) for the canonical edge list
    ``mesh['edges']`` (sorted, i < j), and t_k ~ logU[1e-3, 1e-1]."""
    rng = np.random.default_rng((seed, 1000 + k))
    a, bb = rng.uniform(1.0, 6.0, size=2)
    phi, psi = rng.uniform(0.0, 2.0 * np.pi, size=2)
    t = float(10.0 ** rng.uniform(-3.0, -1.0))
    E = mesh["edges"]
    V = mesh["V"]
    xm = 0.5 * (V[E[:, 0], 0] + V[E[:, 1], 0])
    ym = 0.5 * (V[E[:, 0], 1] + V[E[:, 1], 1])
    w = np.exp2(np.sin(a * xm + phi) * np.cos(bb * ym + psi))
    return dict(t=t, w=w)
