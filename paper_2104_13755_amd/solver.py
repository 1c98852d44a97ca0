"""Python binding of libsmg: argument marshalling only.

Every step of the solve (assembly, Galerkin, Cholesky, relaxation, residual,
transfers, norms) runs in the library's HIP kernels; torch supplies device
memory and the current stream.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L

_c = ctypes.c_void_p


def _np_ptr(a):
    return a.ctypes.data_as(_c)


def _t_ptr(t):
    return _c(t.data_ptr()) if t is not None else None


def _stream():
    return _c(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t, shape=None, device=None, dtype=torch.float64, name="tensor"):
    """Check a tensor before its pointer crosses the ABI: a contiguous CUDA
    tensor of `dtype` (on `device` if given) with exactly `shape`."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name}: on cuda:{t.device.index}, the solver is on cuda:{device}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def mesh_pattern(n, F):
    """CSR pattern {diagonal} U {mesh edges} (int32 rowptr, cols)."""
    lib = L.load()
    F = np.ascontiguousarray(F, dtype=np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    nnz = ctypes.c_int32(0)
    L.check(lib.smg_mesh_pattern(n, _np_ptr(F), len(F), _np_ptr(rowptr), None, ctypes.byref(nnz)), "mesh_pattern")
    cols = np.zeros(nnz.value, dtype=np.int32)
    L.check(lib.smg_mesh_pattern(n, _np_ptr(F), len(F), _np_ptr(rowptr), _np_ptr(cols), ctypes.byref(nnz)), "mesh_pattern")
    return rowptr, cols


def host_assemble(V, F, rowptr=None, cols=None):
    """Cotangent Laplacian values (CSR order of the mesh pattern) and lumped
    mass on the host (smg_pre_assemble).  Returns (rowptr, cols, L_vals, M)."""
    lib = L.load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    if rowptr is None:
        rowptr, cols = mesh_pattern(len(V), F)
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    lv = np.zeros(len(cols))
    m = np.zeros(len(V))
    L.check(lib.smg_pre_assemble(_np_ptr(V), len(V), _np_ptr(F), len(F), _np_ptr(rowptr), _np_ptr(cols),
                                 _np_ptr(lv), _np_ptr(m)), "pre_assemble")
    return rowptr, cols, lv, m


def color_pattern(rowptr, cols):
    """Greedy coloring of a CSR pattern's off-diagonal graph (host)."""
    lib = L.load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    n = len(rowptr) - 1
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = lib.smg_color_pattern(n, _np_ptr(rowptr), _np_ptr(cols), _np_ptr(out))
    if nc < 0:
        L.check(nc, "color_pattern")
    return out[:n], nc


_COLLAPSES = {"all": L.SMG_COLLAPSE_ALL, "interior": L.SMG_COLLAPSE_INTERIOR,
              "straight": L.SMG_COLLAPSE_STRAIGHT}


class Hierarchy:
    """Host-side prolongations P_1..P_H (owned by libsmg)."""

    def __init__(self, handle):
        self._h = handle
        self._lib = L.load()

    @classmethod
    def build(cls, V, F, n_levels=0, min_coarse=500, collapses="all"):
        """Precompute P_1..P_H from the mesh alone (Sec. 4, successive
        self-parameterization; host).  V: n x 3 float64, F: m x 3 int32.
        n_levels = 0 keeps decimating by 1/4 while the next level has at
        least min_coarse vertices (Sec. 5 defaults).  collapses: "all" (the
        method), or the test restrictions "interior" (both endpoints
        interior) and "straight" (those plus boundary edges on straight
        boundary runs)."""
        lib = L.load()
        V = np.ascontiguousarray(V, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.int32)
        o = L.PreOpts(int(n_levels), int(min_coarse), _COLLAPSES[collapses])
        h = _c()
        L.check(lib.smg_pre_build(_np_ptr(V), len(V), _np_ptr(F), len(F), ctypes.byref(o), ctypes.byref(h)), "pre_build")
        return cls(h)

    @classmethod
    def from_prolongations(cls, sizes, pcols, pws):
        """Wrap prolongations computed elsewhere: level l is sizes[l] x 3 ELL
        (pcols[l] int32 with -1 for unused slots, pws[l] float64 >= 0)."""
        lib = L.load()
        sizes = np.ascontiguousarray(sizes, dtype=np.int32)
        pcols = [np.ascontiguousarray(p, dtype=np.int32) for p in pcols]
        pws = [np.ascontiguousarray(p, dtype=np.float64) for p in pws]
        nl = len(sizes)
        arr_c = (_c * max(1, nl - 1))(*[_np_ptr(p) for p in pcols])
        arr_w = (_c * max(1, nl - 1))(*[_np_ptr(p) for p in pws])
        h = _c()
        L.check(lib.smg_hier_from_prolongations(nl, _np_ptr(sizes), arr_c, arr_w, ctypes.byref(h)), "hier_from_prolongations")
        return cls(h)

    @property
    def num_levels(self):
        return self._lib.smg_hier_num_levels(self._h)

    @property
    def sizes(self):
        return [self._lib.smg_hier_level_size(self._h, l) for l in range(self.num_levels)]

    def prolongation(self, l):
        n = self.sizes[l]
        cols = np.zeros((n, 3), dtype=np.int32)
        w = np.zeros((n, 3), dtype=np.float64)
        L.check(self._lib.smg_hier_get_prolongation(self._h, l, _np_ptr(cols), _np_ptr(w)), "get_prolongation")
        return cols, w

    def save(self, path):
        """Write the hierarchy (smg_hier_save: versioned binary file with a
        checksum): the precompute depends on the geometry only, so a saved
        hierarchy serves every later system on the same mesh."""
        L.check(self._lib.smg_hier_save(self._h, str(path).encode()), "hier_save")

    @classmethod
    def load(cls, path):
        """Hierarchy from a file written by save() (smg_hier_load)."""
        lib = L.load()
        h = _c()
        L.check(lib.smg_hier_load(str(path).encode(), ctypes.byref(h)), "hier_load")
        return cls(h)

    def stats(self, l):
        s = np.zeros(8)
        L.check(self._lib.smg_hier_stats(self._h, l, _np_ptr(s)), "hier_stats")
        keys = ["collapses", "fails", "interior", "one_boundary", "b_case1", "b_case2", "b_case3", "max_clamp"]
        return {k: (float(v) if k == "max_clamp" else int(v)) for k, v in zip(keys, s)}

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.smg_hier_free(self._h)
            self._h = None


class DirichletSystem:
    """Dirichlet conditions (App. B): the reduced system A_uu x_u = b_u - A_uk x_k
    on the unknowns, with its hierarchy (P_{u:} at the finest transfer, zero
    columns removed).  `known`: boolean per vertex (natural order)."""

    def __init__(self, hier, rowptr, cols, known):
        lib = L.load()
        self._lib = lib
        n = len(rowptr) - 1
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        kn = np.ascontiguousarray(np.asarray(known, dtype=bool).astype(np.uint8))
        if len(kn) != n:
            raise ValueError("known must have one flag per row")
        uidx = np.zeros(n, dtype=np.int32)
        nu = ctypes.c_int32()
        h = _c()
        L.check(lib.smg_hier_dirichlet(hier._h, _np_ptr(kn), ctypes.byref(h), _np_ptr(uidx), ctypes.byref(nu)),
                "hier_dirichlet")
        self.hier = Hierarchy(h)
        self.unknown = uidx[:nu.value].copy()
        urp = np.zeros(n + 1, dtype=np.int32)
        uci = np.zeros(max(1, len(cols)), dtype=np.int32)
        nu2, nnz = ctypes.c_int32(), ctypes.c_int32()
        L.check(lib.smg_dirichlet_pattern(n, _np_ptr(rowptr), _np_ptr(cols), _np_ptr(kn), _np_ptr(urp), _np_ptr(uci),
                                          ctypes.byref(nu2), ctypes.byref(nnz)), "dirichlet_pattern")
        self.u_rowptr = urp[:nu2.value + 1].copy()
        self.u_cols = uci[:nnz.value].copy()
        dev = "cuda"
        self._d = [torch.tensor(a, device=dev) for a in (self.unknown, rowptr, cols, kn, self.u_rowptr)]
        self.n = n

    def reduce(self, a_vals, x, b):
        """(A_uu values on (u_rowptr, u_cols), b_u - A_uk x_k); x and b are n x k
        (the known entries of x are the prescribed values)."""
        x2 = x if x.dim() == 2 else x.unsqueeze(1)
        b2 = b if b.dim() == 2 else b.unsqueeze(1)
        k = b2.shape[1]
        uv = torch.empty(len(self.u_cols), dtype=torch.float64, device=a_vals.device)
        rhs = torch.empty((len(self.unknown), k), dtype=torch.float64, device=a_vals.device)
        ui, rp, ci, kn, urp = self._d
        L.check(self._lib.smg_dirichlet_reduce(len(self.unknown), _t_ptr(ui), _t_ptr(rp), _t_ptr(ci),
                                               _t_ptr(_dev_f64(a_vals)), _t_ptr(kn), _t_ptr(_dev_f64(x2.contiguous())),
                                               _t_ptr(_dev_f64(b2.contiguous())), k, _t_ptr(urp), _t_ptr(uv),
                                               _t_ptr(rhs), _stream()), "dirichlet_reduce")
        return uv, (rhs if b.dim() == 2 else rhs[:, 0])


class TorchAllocator:
    """A library context whose device buffers come from torch's caching
    allocator (smg_ctx_create with caller functions): solver and batch
    buffers then show in torch's memory statistics and are reused by it
    once the solver is destroyed.  Keep it alive while its solvers live
    (each Solver made with it holds a reference)."""

    def __init__(self, device=0):
        self._lib = L.load()
        self.device = int(device)
        self.live = {}                       # pointer -> bytes, for statistics
        self._alloc = L.ALLOC_FN(self._take)
        self._free = L.FREE_FN(self._give)
        h = _c()
        L.check(self._lib.smg_ctx_create(self.device, self._alloc, self._free, None, ctypes.byref(h)), "ctx_create")
        self._ctx = h

    def _take(self, nbytes, user):
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                   torch.cuda.current_stream(self.device))
        except Exception:
            return None
        self.live[p] = int(nbytes)
        return p

    def _give(self, p, nbytes, user):
        self.live.pop(p, None)
        torch.cuda.caching_allocator_delete(p)

    @property
    def bytes_in_use(self):
        return sum(self.live.values())

    def __del__(self):
        if getattr(self, "_ctx", None):
            self._lib.smg_ctx_destroy(self._ctx)
            self._ctx = None


PRECISION = {"fp64": L.SMG_FP64, "fp32ir": L.SMG_FP32_IR}
SMOOTHER = {"gs": L.SMG_SMOOTH_GS, "jacobi": L.SMG_SMOOTH_JACOBI}


class Solver:
    """Device-resident multigrid solver of one mesh."""

    def __init__(self, hier, rowptr, cols, device=0, mu_pre=2, mu_post=2, faces=None,
                 tail_rows=0, lanes_per_row=None, allocator=None, team_level=0, team_size=0):
        """Upload a hierarchy for the level-0 CSR pattern (rowptr, cols: host
        int32, diagonal present, columns ascending).  Builds colorings,
        layouts and the symbolic Galerkin plans; `faces` enables assemble().
        tail_rows / lanes_per_row are launch shapes (0 = defaults).
        allocator: a TorchAllocator to take the device buffers from torch's
        caching allocator (default: the library's hipMalloc)."""
        self._lib = L.load()
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        self.rowptr, self.cols = rowptr, cols
        self.n = len(rowptr) - 1
        self.nnz = len(cols)
        self.device = device
        lpr = list(lanes_per_row or [])
        o = L.Opts(int(mu_pre), int(mu_post), int(tail_rows),
                   (ctypes.c_int32 * 16)(*(lpr + [0] * (16 - len(lpr)))), int(team_level), int(team_size))
        h = _c()
        self.allocator = allocator
        if allocator is not None:
            if allocator.device != device:
                raise ValueError("the allocator's device differs from the solver's")
            L.check(self._lib.smg_solver_create_ctx(allocator._ctx, hier._h, _np_ptr(rowptr), _np_ptr(cols),
                                                    ctypes.byref(o), ctypes.byref(h)), "solver_create")
        else:
            L.check(self._lib.smg_solver_create(device, hier._h, _np_ptr(rowptr), _np_ptr(cols), ctypes.byref(o),
                                                ctypes.byref(h)), "solver_create")
        self._s = h
        if faces is not None:
            F = np.ascontiguousarray(faces, dtype=np.int32)
            L.check(self._lib.smg_solver_attach_mesh(self._s, _np_ptr(F), len(F)), "attach_mesh")

    def __del__(self):
        if getattr(self, "_s", None):
            self._lib.smg_solver_destroy(self._s)
            self._s = None

    # ---- argument checks (every pointer is checked before the C call) ---
    def _level(self, l, smoothed=False, transfer=False):
        nl = self.num_levels
        if not (0 <= int(l) < nl):
            raise ValueError(f"level {l} out of range 0..{nl - 1}")
        if (smoothed or transfer) and int(l) == nl - 1:
            raise ValueError(f"level {l} is the coarsest level")
        return int(l)

    def _vecs(self, n, *named):
        """Each (name, tensor) must be an n x k float64 CUDA tensor on the
        solver's device, contiguous, with one k (1..4) for all; returns k."""
        k = None
        for name, t in named:
            if not isinstance(t, torch.Tensor) or t.dim() != 2:
                raise ValueError(f"{name}: expected an n x k tensor")
            k = t.shape[1] if k is None else k
            _dev_f64(t, (n, k), self.device, name=name)
        if not 1 <= k <= 4:
            raise ValueError(f"k = {k} right-hand sides; 1..4 supported")
        return k

    # ---- structure ------------------------------------------------------
    @property
    def num_levels(self):
        return self._lib.smg_num_levels(self._s)

    def level_size(self, l):
        return self._lib.smg_level_size(self._s, l)

    def level_nnz(self, l):
        return self._lib.smg_level_nnz(self._s, l)

    def colors(self, l):
        n = self.level_size(l)
        out = np.zeros(max(n, 1), dtype=np.int32)
        nc = self._lib.smg_level_colors(self._s, l, _np_ptr(out))
        return out[:n], nc

    def level_matrix(self, l):
        import scipy.sparse as sp
        n, nnz = self.level_size(l), self.level_nnz(l)
        rp = np.zeros(n + 1, dtype=np.int32)
        ci = np.zeros(nnz, dtype=np.int32)
        v = np.zeros(nnz, dtype=np.float64)
        L.check(self._lib.smg_get_level_matrix(self._s, l, _np_ptr(rp), _np_ptr(ci), _np_ptr(v)), "get_level_matrix")
        return sp.csr_matrix((v, ci, rp), shape=(n, n))

    def coarse_factor(self):
        n = self.level_size(self.num_levels - 1)
        G = np.zeros(n * n, dtype=np.float64)
        L.check(self._lib.smg_get_coarse_factor(self._s, _np_ptr(G)), "get_coarse_factor")
        return G.reshape(n, n).T.copy()   # column-major -> row-major

    # ---- values ---------------------------------------------------------
    def assemble(self, V, t, mass_scale=None, edge_w=None, want_l=False, want_mass=False):
        """A = M + t L on the device from vertex positions V (n x 3 float64):
        cotangent Laplacian and lumped mass (optional per-vertex mass scales
        and per-edge float32 weights).  Returns (a, l, m): values of A on the
        solver's pattern, of L if want_l, the lumped mass if want_mass."""
        _dev_f64(V, (self.n, 3), self.device, name="V")
        if mass_scale is not None:
            _dev_f64(mass_scale, (self.n,), self.device, name="mass_scale")
        if edge_w is not None:
            _dev_f64(edge_w, ((self.nnz - self.n) // 2,), self.device, torch.float32, name="edge_w")
        dev = V.device
        a = torch.empty(self.nnz, dtype=torch.float64, device=dev)
        lv = torch.empty(self.nnz, dtype=torch.float64, device=dev) if want_l else None
        m = torch.empty(self.n, dtype=torch.float64, device=dev) if want_mass else None
        L.check(self._lib.smg_assemble(self._s, _t_ptr(V), float(t),
                                       _t_ptr(mass_scale), _t_ptr(edge_w), _t_ptr(a), _t_ptr(lv),
                                       _t_ptr(m), _stream()), "assemble")
        return a, lv, m

    def set_values(self, a_vals):
        """New values of A_0 on the pattern: every Galerkin level
        A_{l+1} = P_l^T A_l P_l and the coarsest factor are recomputed on the
        device (Alg. "Galerkin Surface Multigrid Solver")."""
        L.check(self._lib.smg_set_values(self._s, _t_ptr(_dev_f64(a_vals, (self.nnz,), self.device, name="a_vals")),
                                         _stream()), "set_values")

    # ---- solve ----------------------------------------------------------
    def solve(self, b, rtol=1e-8, max_cycles=100, precision="fp64", fixed_cycles=0,
              use_graph=False, raise_on_error=True, timed=False):
        """V-cycles from x = 0 until every column's relative residual is at most
        rtol (or exactly fixed_cycles).  b: n or n x k (k <= 4) float64 on the
        device.  precision "fp32ir" runs FP32 cycles inside FP64 iterative
        refinement.  use_graph replays each cycle from a captured hipGraph:
        the same iterates bit for bit, one host call per cycle instead of one
        per launch (faster wherever the host enqueues a launch more slowly
        than the device runs it).  Returns (x, info) with info cycles,
        rel_res, ms and ms_phase (device ms per phase of Tab. "profile":
        prepare = the last value refresh, and with timed=True relax,
        transfer, norm, other)."""
        b2 = b if b.dim() == 2 else b.unsqueeze(1)
        b2 = b2.contiguous()
        k = self._vecs(self.n, ("b", b2))
        x = torch.empty_like(b2)
        p = L.SolveParams(float(rtol), int(max_cycles), PRECISION[precision], int(fixed_cycles), int(bool(use_graph)),
                          int(bool(timed)))
        info = L.SolveInfo()
        st = self._lib.smg_solve(self._s, _t_ptr(b2), _t_ptr(x), k, ctypes.byref(p), ctypes.byref(info), _stream())
        if raise_on_error:
            L.check(st, "solve")
        out = dict(status=st, cycles=info.cycles, rel_res=list(info.rel_res)[:k], ms=info.ms,
                   ms_phase=dict(zip(L.PHASES, list(info.ms_phase))))
        return (x if b.dim() == 2 else x[:, 0]), out

    def split_prepare(self, q_vals, m_vals):
        """Keep the Galerkin levels of two level-0 matrices (values on the
        solver's pattern) for split_combine (App. E linearity)."""
        q = _dev_f64(q_vals, (self.nnz,), self.device, name="q_vals")
        m = _dev_f64(m_vals, (self.nnz,), self.device, name="m_vals")
        L.check(self._lib.smg_split_prepare(self._s, _t_ptr(q), _t_ptr(m), _stream()), "split_prepare")

    def split_combine(self, a, b):
        """Values a Q + b M on every level without assembly or Galerkin products."""
        L.check(self._lib.smg_split_combine(self._s, float(a), float(b), _stream()), "split_combine")

    def set_smoother(self, kind="gs", omega=0.0):
        """Relaxation for every later call: "gs" (multicolor Gauss-Seidel)
        or "jacobi" (damped Jacobi; omega > 0 on every level, omega <= 0 per
        level from the largest eigenvalue estimate of D^{-1} A)."""
        L.check(self._lib.smg_set_smoother(self._s, SMOOTHER[kind], float(omega)), "set_smoother")

    def jacobi_omega(self, level):
        w = ctypes.c_double()
        L.check(self._lib.smg_get_jacobi_omega(self._s, int(level), ctypes.byref(w)), "jacobi_omega")
        return w.value

    def pcg(self, b, rtol=1e-8, max_iters=100, precision="fp64", fixed_iters=0, raise_on_error=True):
        """Conjugate gradients preconditioned by one symmetric V-cycle
        (smg_pcg_solve); returns (x, info) with info["iterations"]."""
        b2 = b if b.dim() == 2 else b.unsqueeze(1)
        b2 = b2.contiguous()
        k = self._vecs(self.n, ("b", b2))
        x = torch.empty_like(b2)
        p = L.SolveParams(float(rtol), int(max_iters), PRECISION[precision], int(fixed_iters), 0, 0)
        info = L.SolveInfo()
        st = self._lib.smg_pcg_solve(self._s, _t_ptr(b2), _t_ptr(x), k, ctypes.byref(p), ctypes.byref(info), _stream())
        if raise_on_error:
            L.check(st, "pcg")
        out = dict(status=st, iterations=info.cycles, rel_res=list(info.rel_res)[:k], ms=info.ms)
        return (x if b.dim() == 2 else x[:, 0]), out

    def vcycle(self, b, x, precision="fp64"):
        """One cycle updating x in place: a V-cycle (Alg. "V-cycle"), or with
        "fp32ir" one refinement step (FP64 residual, FP32 V-cycle on it
        scaled by its column max, FP64 update)."""
        k = self._vecs(self.n, ("b", b), ("x", x))
        L.check(self._lib.smg_vcycle(self._s, PRECISION[precision], _t_ptr(b), _t_ptr(x), k, _stream()), "vcycle")
        return x

    # ---- single steps (level-natural numbering) ------------------------
    # precision "fp32ir" runs the FP32 kernels of the inner cycles on the
    # inputs rounded to FP32 (results returned in float64).
    def residual(self, l, b, x, precision="fp64"):
        """r = b - A_l x on level l."""
        l = self._level(l, smoothed=True)
        k = self._vecs(self.level_size(l), ("b", b), ("x", x))
        r = torch.empty_like(b)
        L.check(self._lib.smg_residual(self._s, l, PRECISION[precision], _t_ptr(b), _t_ptr(x), _t_ptr(r), k,
                                       _stream()), "residual")
        return r

    def smooth(self, l, b, x, sweeps, precision="fp64"):
        """`sweeps` relaxation sweeps of the current smoother on level l, in place."""
        l = self._level(l, smoothed=True)
        k = self._vecs(self.level_size(l), ("b", b), ("x", x))
        L.check(self._lib.smg_smooth(self._s, l, PRECISION[precision], _t_ptr(b), _t_ptr(x), k, int(sweeps),
                                     _stream()), "smooth")
        return x

    def restrict(self, l, r, precision="fp64"):
        """P_l^T r: level l to level l + 1."""
        l = self._level(l, transfer=True)
        k = self._vecs(self.level_size(l), ("r", r))
        rc = torch.empty((self.level_size(l + 1), k), dtype=torch.float64, device=r.device)
        L.check(self._lib.smg_restrict(self._s, l, PRECISION[precision], _t_ptr(r), _t_ptr(rc), k, _stream()),
                "restrict")
        return rc

    def prolong_add(self, l, e, x, precision="fp64"):
        """x += P_l e: level l + 1 to level l, in place."""
        l = self._level(l, transfer=True)
        k = self._vecs(self.level_size(l), ("x", x))
        if self._vecs(self.level_size(l + 1), ("e", e)) != k:
            raise ValueError("e and x need the same number of columns")
        L.check(self._lib.smg_prolong_add(self._s, l, PRECISION[precision], _t_ptr(e), _t_ptr(x), k, _stream()),
                "prolong_add")
        return x

    def coarse_solve(self, b, precision="fp64"):
        """x = A_H^{-1} b on the coarsest level (dense Cholesky factor)."""
        k = self._vecs(self.level_size(self.num_levels - 1), ("b", b))
        x = torch.empty_like(b)
        L.check(self._lib.smg_coarse_solve(self._s, PRECISION[precision], _t_ptr(b), _t_ptr(x), k, _stream()),
                "coarse_solve")
        return x

    # ---- steps of the one-workgroup tail (smg_tail_step) ---------------
    def tail_first(self, k, precision="fp64"):
        """Finest level the one-workgroup tail covers (num_levels - 1: none)."""
        return self._lib.smg_tail_first_level(self._s, PRECISION[precision], int(k))

    def _tail(self, l, step, a, a2, out, k, sweeps, precision):
        L.check(self._lib.smg_tail_step(self._s, l, step, PRECISION[precision], _t_ptr(a), _t_ptr(a2), _t_ptr(out),
                                        k, int(sweeps), _stream()), "tail_step")
        return out

    def tail_relax(self, l, b, x, sweeps, precision="fp64"):
        """|sweeps| Gauss-Seidel sweeps in the tail's code, in place on x
        (colors descending if sweeps < 0)."""
        l = self._level(l, smoothed=True)
        k = self._vecs(self.level_size(l), ("b", b), ("x", x))
        return self._tail(l, L.SMG_TAIL_RELAX, b, None, x, k, sweeps, precision)

    def tail_residual(self, l, b, x, precision="fp64"):
        l = self._level(l, smoothed=True)
        k = self._vecs(self.level_size(l), ("b", b), ("x", x))
        return self._tail(l, L.SMG_TAIL_RESIDUAL, b, x, torch.empty_like(b), k, 0, precision)

    def tail_restrict(self, l, r, precision="fp64"):
        l = self._level(l, transfer=True)
        k = self._vecs(self.level_size(l), ("r", r))
        out = torch.empty((self.level_size(l + 1), k), dtype=torch.float64, device=r.device)
        return self._tail(l, L.SMG_TAIL_RESTRICT, r, None, out, k, 0, precision)

    def tail_prolong(self, l, e, x, precision="fp64"):
        l = self._level(l, transfer=True)
        k = self._vecs(self.level_size(l), ("x", x))
        if self._vecs(self.level_size(l + 1), ("e", e)) != k:
            raise ValueError("e and x need the same number of columns")
        return self._tail(l, L.SMG_TAIL_PROLONG, e, None, x, k, 0, precision)

    def tail_coarse(self, b, precision="fp64"):
        l = self.num_levels - 1
        k = self._vecs(self.level_size(l), ("b", b))
        return self._tail(l, L.SMG_TAIL_COARSE, b, None, torch.empty_like(b), k, 0, precision)

    # ---- per-launch timing --------------------------------------------
    # "gs_group": one event pair around each relaxation call's launches
    PROF = {"gs": 0, "residual": 1, "restrict": 2, "prolong": 3, "coarse": 4, "galerkin": 5, "gs_group": 0x100}

    def profile_enable(self, kind, level=0):
        L.check(self._lib.smg_profile_enable(self._s, self.PROF[kind] if kind else -1, level), "profile_enable")

    def launch_floor(self, kind, level, launches=2000):
        """Launches of kind "empty", "chain" (index load, dependent load,
        store) or "chain_rw" (the chain gathering what the previous launch
        wrote) with level `level`'s widest color grid, queued ahead of the
        device: (device µs from one launch to the next, host µs to enqueue
        one)."""
        us, host = ctypes.c_double(0.0), ctypes.c_double(0.0)
        L.check(self._lib.smg_launch_floor(self._s, {"empty": 0, "chain": 1, "chain_rw": 2}[kind], int(level),
                                           int(launches),
                                           _stream(), ctypes.byref(us), ctypes.byref(host)), "launch_floor")
        return us.value, host.value

    def profile_read(self):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        by = ctypes.c_double(0.0)
        L.check(self._lib.smg_profile_read(self._s, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)), "profile_read")
        return dict(ms=ms.value, launches=n.value, bytes=by.value)

    # ---- adjoint helpers ----------------------------------------------
    def spmv_dot(self, l_vals, lam, u):
        """lam^T L u over the level-0 pattern (one column)."""
        _dev_f64(l_vals, (self.nnz,), self.device, name="l_vals")
        lam = lam.reshape(self.n) if lam.numel() == self.n else lam
        u = u.reshape(self.n) if u.numel() == self.n else u
        _dev_f64(lam, (self.n,), self.device, name="lam")
        _dev_f64(u, (self.n,), self.device, name="u")
        out = ctypes.c_double(0.0)
        L.check(self._lib.smg_spmv_dot(self._s, _t_ptr(l_vals), _t_ptr(lam), _t_ptr(u), ctypes.byref(out), _stream()),
                "spmv_dot")
        return out.value

    def mass_grad(self, lam, m, u):
        """-lam_i m_i u_i per vertex."""
        for name, t in (("lam", lam), ("m", m), ("u", u)):
            _dev_f64(t, (self.n,), self.device, name=name)
        out = torch.empty_like(lam)
        L.check(self._lib.smg_mass_grad(self._s, _t_ptr(lam), _t_ptr(m), _t_ptr(u), _t_ptr(out), _stream()),
                "mass_grad")
        return out
