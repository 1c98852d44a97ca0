// C ABI of libsmg (see include/smg.h): host precompute entry points, device
// solver construction, hierarchy refresh (Galerkin + coarsest Cholesky), the
// V-cycle driver and the FP64 / FP32-in-FP64-refinement solve loops.
#include "smg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hier.h"
#include "kernels.h"
#include "runtime.h"

using namespace smg;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;
// levels with at most this many rows (and all coarser ones) form the
// one-workgroup LDS tail unless the caller chooses otherwise
static constexpr int kTailRowsDefault = 4096;
// largest coarsest level factored densely: 16384^2 doubles = 2 GiB per copy
static constexpr int kCoarsestMax = 16384;
// The LDS tail runs one workgroup per right-hand side (columns are
// independent solves): each holds one value per row in LDS and the columns
// proceed on different compute units at once.
constexpr bool kTailPerColumn = true;
// Whole-level passes (residual, CG product, restriction) on levels with at
// least this many rows take their slices region by region.  Workgroups are
// dealt to the 8 XCDs in turn and the kernels renumber them (xcd_block) so
// that each XCD works through a contiguous eighth of the wavefront indices;
// in color-major slice order that eighth is about one color spread over the
// whole mesh, whose gathers reach all of x.  The order below lists, for
// x = 0..7, the x-th eighth (a Morton range) of every color, so the eighth
// an XCD takes is one region of the mesh in every color.
static constexpr int kRegionOrderRows = 65536;
static std::vector<int32_t> region_order(const std::vector<int32_t> &bounds, int total) {
    std::vector<int32_t> out;
    if (bounds.size() < 2 || bounds.front() != 0 || bounds.back() != total) return out;
    out.reserve((size_t)total);
    for (int x = 0; x < 8; ++x)
        for (size_t c = 0; c + 1 < bounds.size(); ++c) {
            const int64_t b0 = bounds[c], len = (int64_t)bounds[c + 1] - b0;
            for (int64_t i = b0 + len * x / 8; i < b0 + len * (x + 1) / 8; ++i) out.push_back((int32_t)i);
        }
    if ((int)out.size() != total) out.clear();   // bounds were not a partition
    return out;
}

namespace smg {
smg_status fail(smg_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}
}  // namespace smg

#define HIPCHK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(SMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" const char *smg_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *smg_status_string(smg_status st) {
    switch (st) {
    case SMG_OK: return "ok";
    case SMG_ERR_INVALID_ARG: return "invalid argument";
    case SMG_ERR_OOM: return "out of memory";
    case SMG_ERR_HIP: return "HIP runtime error";
    case SMG_ERR_NOT_SPD: return "coarsest matrix not positive definite";
    case SMG_ERR_NO_CONVERGENCE: return "no convergence within the cycle cap";
    case SMG_ERR_NONFINITE: return "non-finite value";
    case SMG_ERR_STATE: return "call out of order";
    case SMG_ERR_PRECOMPUTE: return "hierarchy precompute failed";
    default: return "unknown status";
    }
}

// ------------------------------------------------------- host precompute
struct smg_hier_s {
    HierHost H;
};

// Zero-column removal (App. B): drop coarse vertices that receive no weight
// from the level above, and the matching rows of the next prolongation (a
// removal can leave further zero columns below, so levels go in order).
static void compact_zero_columns(HierHost &H) {
    for (int l = 0; l + 1 < H.nlev; ++l) {
        const int nc = H.sizes[l + 1];
        std::vector<char> used(nc, 0);
        for (size_t e = 0; e < H.pcols[l].size(); ++e)
            if (H.pcols[l][e] >= 0 && H.pw[l][e] > 0.0) used[H.pcols[l][e]] = 1;
        std::vector<int32_t> newid(nc, -1);
        int cnt = 0;
        for (int a = 0; a < nc; ++a) if (used[a]) newid[a] = cnt++;
        if (cnt == nc) continue;
        for (auto &c : H.pcols[l]) if (c >= 0) c = newid[c];
        if (l + 1 < (int)H.X.size() && H.X[l + 1].size() == 3 * (size_t)nc) {
            std::vector<double> Xc;
            for (int a = 0; a < nc; ++a)
                if (used[a]) Xc.insert(Xc.end(), H.X[l + 1].begin() + 3 * a, H.X[l + 1].begin() + 3 * a + 3);
            H.X[l + 1] = std::move(Xc);
        }
        if (l + 2 < H.nlev) {
            std::vector<int32_t> pc2;
            std::vector<double> pw2;
            for (int a = 0; a < nc; ++a)
                if (used[a])
                    for (int q = 0; q < 3; ++q) { pc2.push_back(H.pcols[l + 1][3 * a + q]); pw2.push_back(H.pw[l + 1][3 * a + q]); }
            H.pcols[l + 1] = std::move(pc2);
            H.pw[l + 1] = std::move(pw2);
        }
        H.sizes[l + 1] = cnt;
    }
}

extern "C" smg_status smg_pre_build(const double *V, int32_t n, const int32_t *F, int32_t m,
                                    const smg_pre_opts *opts, smg_hier *out) {
    if (!V || !F || !out || n < 3 || m < 1) return fail(SMG_ERR_INVALID_ARG, "smg_pre_build: bad arguments");
    for (int64_t i = 0; i < 3 * (int64_t)m; ++i)
        if (F[i] < 0 || F[i] >= n) return fail(SMG_ERR_INVALID_ARG, "smg_pre_build: face index out of range");
    for (int64_t f = 0; f < m; ++f)
        if (F[3 * f] == F[3 * f + 1] || F[3 * f + 1] == F[3 * f + 2] || F[3 * f] == F[3 * f + 2])
            return fail(SMG_ERR_INVALID_ARG, "smg_pre_build: face " + std::to_string(f) + " repeats a vertex");
    for (int64_t i = 0; i < 3 * (int64_t)n; ++i)
        if (!std::isfinite(V[i])) return fail(SMG_ERR_INVALID_ARG, "smg_pre_build: non-finite vertex coordinate");
    const int min_coarse = (opts && opts->min_coarse > 0) ? opts->min_coarse : 500;
    const int collapses = opts ? opts->collapses : SMG_COLLAPSE_ALL;
    if (collapses < SMG_COLLAPSE_ALL || collapses > SMG_COLLAPSE_STRAIGHT)
        return fail(SMG_ERR_INVALID_ARG, "smg_pre_build: unknown collapse set");
    int nlev = opts ? opts->n_levels : 0;
    auto target = [](int nn) { return (int)std::floor(nn / 4.0 + 0.5); };
    if (nlev <= 0) {
        nlev = 1;
        for (int nn = n; target(nn) >= min_coarse; nn = target(nn)) ++nlev;
    }
    auto h = std::make_unique<smg_hier_s>();
    h->H.nlev = nlev;
    h->H.sizes.push_back(n);
    std::vector<double> X(V, V + 3 * (size_t)n);
    h->H.X.push_back(X);
    std::vector<int32_t> Fv(F, F + 3 * (size_t)m);
    for (int l = 0; l + 1 < nlev; ++l) {
        LevelOut lo;
        const int rc = ssp_decimate_level(X, Fv, target((int)(X.size() / 3)), collapses, lo);
        if (rc != 0) return fail(SMG_ERR_PRECOMPUTE, "successive self-parameterization failed at level " + std::to_string(l));
        h->H.pcols.push_back(std::move(lo.pcols));
        h->H.pw.push_back(std::move(lo.pw));
        std::array<double, 8> st;
        std::copy(lo.stats, lo.stats + 8, st.begin());
        h->H.stats.push_back(st);
        X = std::move(lo.X);
        Fv = std::move(lo.F);
        h->H.sizes.push_back((int)(X.size() / 3));
        h->H.X.push_back(X);
    }
    compact_zero_columns(h->H);
    *out = h.release();
    return SMG_OK;
}

extern "C" smg_status smg_hier_from_prolongations(int32_t n_levels, const int32_t *sizes,
                                                  const int32_t *const *p_cols,
                                                  const double *const *p_w, smg_hier *out) {
    if (n_levels < 1 || !sizes || !out || (n_levels > 1 && (!p_cols || !p_w)))
        return fail(SMG_ERR_INVALID_ARG, "smg_hier_from_prolongations: bad arguments");
    if (sizes[0] < 1) return fail(SMG_ERR_INVALID_ARG, "empty level");
    auto h = std::make_unique<smg_hier_s>();
    h->H.nlev = n_levels;
    h->H.sizes.assign(sizes, sizes + n_levels);
    for (int l = 0; l + 1 < n_levels; ++l) {
        const int n = sizes[l], nc = sizes[l + 1];
        if (n < 1 || nc < 1) return fail(SMG_ERR_INVALID_ARG, "empty level");
        std::vector<int32_t> pc(p_cols[l], p_cols[l] + 3 * (size_t)n);
        std::vector<double> pw(p_w[l], p_w[l] + 3 * (size_t)n);
        for (size_t e = 0; e < pc.size(); ++e) {
            if (pc[e] >= nc || pw[e] < 0.0 || !std::isfinite(pw[e]))
                return fail(SMG_ERR_INVALID_ARG, "prolongation entry out of range");
            if (pc[e] < 0 || pw[e] == 0.0) { pc[e] = -1; pw[e] = 0.0; }
        }
        for (int i = 0; i < n; ++i)
            if (pc[3 * (size_t)i] < 0 && pc[3 * (size_t)i + 1] < 0 && pc[3 * (size_t)i + 2] < 0)
                return fail(SMG_ERR_INVALID_ARG, "prolongation row " + std::to_string(i) + " of level " +
                                                     std::to_string(l) + " has no positive weight");
        h->H.pcols.push_back(std::move(pc));
        h->H.pw.push_back(std::move(pw));
        h->H.stats.push_back({0, 0, 0, 0, 0, 0, 0, 0});
    }
    *out = h.release();
    return SMG_OK;
}

extern "C" smg_status smg_pre_assemble(const double *V, int32_t n, const int32_t *F, int32_t m,
                                       const int32_t *rowptr, const int32_t *cols, double *L_vals,
                                       double *M_diag) {
    if (!V || !F || !rowptr || !cols || !L_vals || !M_diag || n < 1 || m < 1)
        return fail(SMG_ERR_INVALID_ARG, "smg_pre_assemble: null or empty argument");
    for (int64_t i = 0; i < 3 * (int64_t)m; ++i)
        if (F[i] < 0 || F[i] >= n) return fail(SMG_ERR_INVALID_ARG, "smg_pre_assemble: face index out of range");
    if (rowptr[0] != 0) return fail(SMG_ERR_INVALID_ARG, "smg_pre_assemble: rowptr[0] != 0");
    for (int i = 0; i < n; ++i)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (cols[p] < 0 || cols[p] >= n || (p > rowptr[i] && cols[p] <= cols[p - 1]))
                return fail(SMG_ERR_INVALID_ARG, "smg_pre_assemble: columns out of range or not ascending");
    std::string err;
    if (!host_assemble(V, n, F, m, rowptr, cols, L_vals, M_diag, err))
        return fail(SMG_ERR_INVALID_ARG, "smg_pre_assemble: " + err);
    return SMG_OK;
}

extern "C" smg_status smg_hier_save(smg_hier h, const char *path) {
    if (!h || !path) return fail(SMG_ERR_INVALID_ARG, "smg_hier_save: null argument");
    std::string err;
    if (!hier_write(h->H, path, err)) return fail(SMG_ERR_INVALID_ARG, "smg_hier_save: " + err);
    return SMG_OK;
}

extern "C" smg_status smg_hier_load(const char *path, smg_hier *out) {
    if (!path || !out) return fail(SMG_ERR_INVALID_ARG, "smg_hier_load: null argument");
    *out = nullptr;
    auto h = std::make_unique<smg_hier_s>();
    std::string err;
    if (!hier_read(path, h->H, err)) return fail(SMG_ERR_INVALID_ARG, "smg_hier_load: " + err);
    *out = h.release();
    return SMG_OK;
}

extern "C" int32_t smg_hier_num_levels(smg_hier h) { return h ? h->H.nlev : 0; }
extern "C" int32_t smg_hier_level_size(smg_hier h, int32_t l) {
    return (h && l >= 0 && l < h->H.nlev) ? h->H.sizes[l] : -1;
}
extern "C" smg_status smg_hier_get_prolongation(smg_hier h, int32_t l, int32_t *cols, double *w) {
    if (!h || l < 0 || l + 1 >= h->H.nlev || !cols || !w) return fail(SMG_ERR_INVALID_ARG, "bad level");
    std::copy(h->H.pcols[l].begin(), h->H.pcols[l].end(), cols);
    std::copy(h->H.pw[l].begin(), h->H.pw[l].end(), w);
    return SMG_OK;
}
extern "C" smg_status smg_hier_stats(smg_hier h, int32_t l, double *s8) {
    if (!h || l < 0 || l + 1 >= h->H.nlev || !s8) return fail(SMG_ERR_INVALID_ARG, "bad level");
    std::copy(h->H.stats[l].begin(), h->H.stats[l].end(), s8);
    return SMG_OK;
}
extern "C" void smg_hier_free(smg_hier h) { delete h; }

// ------------------------------------------ Dirichlet conditions (App. B)
extern "C" smg_status smg_hier_dirichlet(smg_hier h, const uint8_t *known, smg_hier *out, int32_t *unknown_idx,
                                         int32_t *n_unknown) {
    if (!h || !known || !out || !unknown_idx || !n_unknown) return fail(SMG_ERR_INVALID_ARG, "null argument");
    const HierHost &H = h->H;
    const int n = H.sizes[0];
    int nu = 0;
    for (int i = 0; i < n; ++i) if (!known[i]) unknown_idx[nu++] = i;
    if (nu == 0) return fail(SMG_ERR_INVALID_ARG, "every value is known");
    auto r = std::make_unique<smg_hier_s>();
    HierHost &R = r->H;
    R = H;
    R.sizes[0] = nu;
    if (!H.X.empty() && H.X[0].size() == 3 * (size_t)n) {
        std::vector<double> X0;
        for (int q = 0; q < nu; ++q) X0.insert(X0.end(), H.X[0].begin() + 3 * unknown_idx[q], H.X[0].begin() + 3 * unknown_idx[q] + 3);
        R.X[0] = std::move(X0);
    }
    if (H.nlev > 1) {   // P_{u:}: the rows of P_0 of the unknowns
        std::vector<int32_t> pc;
        std::vector<double> pw;
        for (int q = 0; q < nu; ++q)
            for (int m = 0; m < 3; ++m) {
                pc.push_back(H.pcols[0][3 * (size_t)unknown_idx[q] + m]);
                pw.push_back(H.pw[0][3 * (size_t)unknown_idx[q] + m]);
            }
        R.pcols[0] = std::move(pc);
        R.pw[0] = std::move(pw);
        compact_zero_columns(R);
    }
    *n_unknown = nu;
    *out = r.release();
    return SMG_OK;
}

extern "C" smg_status smg_dirichlet_pattern(int32_t n, const int32_t *rowptr, const int32_t *cols,
                                            const uint8_t *known, int32_t *u_rowptr, int32_t *u_cols,
                                            int32_t *n_unknown, int32_t *nnz_unknown) {
    if (n < 1 || !rowptr || !cols || !known || !u_rowptr || !u_cols || !n_unknown || !nnz_unknown)
        return fail(SMG_ERR_INVALID_ARG, "bad arguments");
    std::vector<int32_t> umap(n, -1);
    int nu = 0;
    for (int i = 0; i < n; ++i) if (!known[i]) umap[i] = nu++;
    int64_t z = 0;
    u_rowptr[0] = 0;
    int r = 0;
    for (int i = 0; i < n; ++i) {
        if (known[i]) continue;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (cols[p] < 0 || cols[p] >= n) return fail(SMG_ERR_INVALID_ARG, "column out of range");
            if (umap[cols[p]] >= 0) u_cols[z++] = umap[cols[p]];
        }
        u_rowptr[++r] = (int32_t)z;
    }
    *n_unknown = nu;
    *nnz_unknown = (int32_t)z;
    return SMG_OK;
}

extern "C" smg_status smg_dirichlet_reduce(int32_t n_unknown, const int32_t *d_unknown_idx, const int32_t *d_rowptr,
                                           const int32_t *d_cols, const double *d_vals, const uint8_t *d_known,
                                           const double *d_x, const double *d_b, int32_t k,
                                           const int32_t *d_u_rowptr, double *d_u_vals, double *d_rhs,
                                           smg_stream stream) {
    if (n_unknown < 1 || !d_unknown_idx || !d_rowptr || !d_cols || !d_vals || !d_known || !d_x || !d_b ||
        !d_u_rowptr || !d_u_vals || !d_rhs || k < 1 || k > 4)
        return fail(SMG_ERR_INVALID_ARG, "bad arguments");
    HIPCHK(launch_dirichlet_reduce(n_unknown, d_unknown_idx, d_rowptr, d_cols, d_vals, d_known, d_x, d_b, k,
                                   d_u_rowptr, d_u_vals, d_rhs, (hipStream_t)stream));
    return SMG_OK;
}

extern "C" int32_t smg_color_pattern(int32_t n, const int32_t *rowptr, const int32_t *cols,
                                     int32_t *color) {
    if (n < 0 || !rowptr || !cols || !color) return fail(SMG_ERR_INVALID_ARG, "smg_color_pattern: bad arguments");
    for (int i = 0; i < n; ++i)
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (cols[p] < 0 || cols[p] >= n) return fail(SMG_ERR_INVALID_ARG, "column out of range");
    std::vector<int32_t> c;
    const int nc = greedy_coloring(n, rowptr, cols, c);
    std::copy(c.begin(), c.end(), color);
    return nc;
}

extern "C" smg_status smg_mesh_pattern(int32_t n, const int32_t *F, int32_t m, int32_t *rowptr,
                                       int32_t *cols, int32_t *nnz) {
    if (n < 1 || !F || m < 1 || !rowptr || !nnz) return fail(SMG_ERR_INVALID_ARG, "smg_mesh_pattern: bad arguments");
    std::vector<std::vector<int32_t>> adj(n);
    for (int f = 0; f < m; ++f)
        for (int c = 0; c < 3; ++c) {
            const int a = F[3 * f + c], b = F[3 * f + (c + 1) % 3];
            if (a < 0 || a >= n || b < 0 || b >= n) return fail(SMG_ERR_INVALID_ARG, "face index out of range");
            adj[a].push_back(b);
            adj[b].push_back(a);
        }
    int64_t total = 0;
    rowptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        adj[i].push_back(i);
        std::sort(adj[i].begin(), adj[i].end());
        adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
        total += (int64_t)adj[i].size();
        if (total > INT32_MAX) return fail(SMG_ERR_INVALID_ARG, "pattern too large");
        rowptr[i + 1] = (int32_t)total;
    }
    if (cols) {
        if (*nnz < total) return fail(SMG_ERR_INVALID_ARG, "cols capacity too small");
        for (int i = 0; i < n; ++i) std::copy(adj[i].begin(), adj[i].end(), cols + rowptr[i]);
    }
    *nnz = (int32_t)total;
    return SMG_OK;
}

// ---------------------------------------------------------- device memory
namespace smg {

template <typename T>
static smg_status dalloc(T **p, size_t count, DevMem &owned) {
    if (count == 0) count = 1;
    *p = (T *)owned.take(count * sizeof(T));
    if (!*p) return fail(SMG_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    return SMG_OK;
}
template <typename T>
static smg_status dupload(T **p, const std::vector<T> &h, DevMem &owned) {
    smg_status st = dalloc(p, h.size(), owned);
    if (st) return st;
    if (!h.empty()) {
        hipError_t e = hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(SMG_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    return SMG_OK;
}

}  // namespace smg

#define CHK(call)                           \
    do {                                    \
        smg_status s_ = (call);             \
        if (s_ != SMG_OK) return s_;        \
    } while (0)

extern "C" smg_status smg_ctx_create(int32_t device, smg_alloc_fn alloc, smg_free_fn free_fn, void *user,
                                     smg_ctx *out) {
    if (!out) return fail(SMG_ERR_INVALID_ARG, "smg_ctx_create: null output");
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(SMG_ERR_INVALID_ARG, "smg_ctx_create: give both allocator functions or neither");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(SMG_ERR_INVALID_ARG, "smg_ctx_create: bad device");
    smg_ctx c = new smg_ctx_s;
    c->device = device;
    c->alloc = alloc;
    c->free = free_fn;
    c->user = user;
    *out = c;
    return SMG_OK;
}

extern "C" void smg_ctx_destroy(smg_ctx ctx) { delete ctx; }

static smg_status solver_create(const smg_ctx_s &ctx, smg_hier h, const int32_t *a0_rowptr,
                                const int32_t *a0_cols, const smg_opts *opts, smg_solver *out);

extern "C" smg_status smg_solver_create(int32_t device, smg_hier h, const int32_t *a0_rowptr,
                                        const int32_t *a0_cols, const smg_opts *opts, smg_solver *out) {
    smg_ctx_s ctx;
    ctx.device = device;
    return solver_create(ctx, h, a0_rowptr, a0_cols, opts, out);
}

extern "C" smg_status smg_solver_create_ctx(smg_ctx ctx, smg_hier h, const int32_t *a0_rowptr,
                                            const int32_t *a0_cols, const smg_opts *opts, smg_solver *out) {
    if (!ctx) return fail(SMG_ERR_INVALID_ARG, "smg_solver_create_ctx: null context");
    return solver_create(*ctx, h, a0_rowptr, a0_cols, opts, out);
}

static smg_status solver_create(const smg_ctx_s &ctx, smg_hier h, const int32_t *a0_rowptr,
                                const int32_t *a0_cols, const smg_opts *opts, smg_solver *out) {
    const int device = ctx.device;
    if (!h || !a0_rowptr || !a0_cols || !out) return fail(SMG_ERR_INVALID_ARG, "smg_solver_create: null argument");
    const int n0 = h->H.sizes[0];
    Csr A0;
    A0.n = A0.m = n0;
    A0.ptr.assign(a0_rowptr, a0_rowptr + n0 + 1);
    if (A0.ptr[0] != 0) return fail(SMG_ERR_INVALID_ARG, "rowptr[0] != 0");
    for (int i = 0; i < n0; ++i) if (A0.ptr[i + 1] < A0.ptr[i]) return fail(SMG_ERR_INVALID_ARG, "rowptr not monotone");
    A0.idx.assign(a0_cols, a0_cols + A0.ptr[n0]);
    for (int i = 0; i < n0; ++i)
        for (int p = A0.ptr[i]; p < A0.ptr[i + 1]; ++p) {
            if (A0.idx[p] < 0 || A0.idx[p] >= n0) return fail(SMG_ERR_INVALID_ARG, "column out of range");
            if (p > A0.ptr[i] && A0.idx[p] <= A0.idx[p - 1]) return fail(SMG_ERR_INVALID_ARG, "columns not strictly ascending");
        }
    // the coarsest level is factored densely (n_H^2 doubles, four copies,
    // 32-bit element indices in the factor kernels)
    const int n_coarse = h->H.sizes[h->H.nlev - 1];
    if (n_coarse > kCoarsestMax)
        return fail(SMG_ERR_INVALID_ARG, "smg_solver_create: coarsest level has " + std::to_string(n_coarse) +
                                             " rows; the dense factorization takes at most " +
                                             std::to_string(kCoarsestMax));
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(SMG_ERR_INVALID_ARG, "bad device");
    HIPCHK(hipSetDevice(device));
    auto S = std::make_unique<smg_solver_s>();
    S->device = device;
    S->owned.ctx = ctx;
    S->mu_pre = opts && opts->mu_pre >= 0 ? opts->mu_pre : 2;
    S->mu_post = opts && opts->mu_post >= 0 ? opts->mu_post : 2;
    if (!opts) S->mu_pre = S->mu_post = 2;
    const int tail_rows = (opts && opts->tail_rows != 0) ? opts->tail_rows : kTailRowsDefault;
    if (opts && (opts->team_level < 0 || opts->team_size < 0 || opts->team_size > 16))
        return fail(SMG_ERR_INVALID_ARG, "team_level must be >= 0 and team_size 0..16");
    S->team_level = opts ? opts->team_level : 0;
    if (S->team_level >= h->H.nlev - 1) S->team_level = 0;   // needs a smoothed level
    S->team_size = (opts && opts->team_size > 0) ? opts->team_size : 16;
    std::vector<int> lpr(16, 0);
    if (opts) for (int l = 0; l < 16; ++l) lpr[l] = opts->lanes_per_row[l];
    std::vector<LevelHost> levels;
    std::string err;
    if (build_levels(h->H, A0, lpr, tail_rows > 0 ? tail_rows : 0, levels, err) != 0)
        return fail(SMG_ERR_INVALID_ARG, "hierarchy setup: " + err);
    S->nlev = h->H.nlev;
    S->lev.resize(S->nlev);
    int64_t tmax = 1;
    int nmax = 1;
    std::vector<int32_t> tpass_h, twave_h;
    int npass_before = 0, nwave_before = 0;
    for (int l = 0; l < S->nlev; ++l) {
        LevelHost &L = levels[l];
        DevLevel &D = S->lev[l];
        D.n = L.n;
        D.coarsest = L.coarsest;
        D.ncolors = L.ncolors;
        D.nnz_nat = (int64_t)L.pat.idx.size();
        D.pat_ptr = L.pat.ptr;
        D.pat_idx = L.pat.idx;
        D.store_h = L.store;
        D.color_h = L.color;
        nmax = std::max(nmax, L.n);
        CHK(dupload(&D.perm, L.perm, S->owned));
        CHK(dupload(&D.store, L.store, S->owned));
        if (L.coarsest) {
            CHK(dalloc(&D.dense, (size_t)L.n * L.n, S->owned));
            CHK(dalloc(&D.dense_a, (size_t)L.n * L.n, S->owned));
            CHK(dalloc(&D.dense_w, (size_t)L.n * L.n, S->owned));
            CHK(dalloc(&D.dense_inv, (size_t)L.n * L.n, S->owned));
        } else {
            const SellLayout &Sl = L.sell;
            D.nslices = Sl.nslices;
            D.lpr = Sl.lpr;
            CHK(dupload(&D.color_row, Sl.color_row, S->owned));
            for (int c = 0; c < L.ncolors; ++c) {
                int64_t z = 0;
                for (int r = Sl.color_row[c]; r < Sl.color_row[c + 1]; ++r) z += Sl.rowlen[r];
                D.color_rows.push_back(Sl.color_row[c + 1] - Sl.color_row[c]);
                D.color_nnz.push_back(z);
                D.offdiag_nnz += z;
            }
            D.color_slice = Sl.color_slice;
            D.color_row_h = Sl.color_row;
            D.color_w = Sl.color_w;
            for (int c = 0; c < L.ncolors; ++c) D.color_off.push_back(Sl.slice_off[Sl.color_slice[c]]);
            D.slots = Sl.slots();
            std::vector<int32_t> row0 = Sl.slice_row0;
            row0.push_back(L.n);
            CHK(dupload(&D.slice_row0, row0, S->owned));
            CHK(dupload(&D.slice_off, Sl.slice_off, S->owned));
            CHK(dupload(&D.cols, Sl.cols, S->owned));
            CHK(dupload(&D.rowlen, Sl.rowlen, S->owned));
            CHK(dupload(&D.row_slice, Sl.row_slice, S->owned));
            {   // first slot of every row, for the one-workgroup and team kernels
                std::vector<int32_t> rb((size_t)L.n);
                for (int r = 0; r < L.n; ++r) {
                    const int sl = Sl.row_slice[r];
                    rb[r] = Sl.slice_off[sl] + (r - Sl.slice_row0[sl]) * Sl.lpr;
                }
                CHK(dupload(&D.row_base, rb, S->owned));
            }
            CHK(dalloc(&D.vals, (size_t)D.slots, S->owned));
            CHK(dalloc(&D.diag, (size_t)L.n, S->owned));
            CHK(dalloc(&D.vals32, (size_t)D.slots, S->owned));
            CHK(dalloc(&D.diag32, (size_t)L.n, S->owned));
            // transfer to the next level
            CHK(dupload(&D.pc, L.pc, S->owned));
            CHK(dupload(&D.pw, L.pw, S->owned));
            std::vector<float> pw32(L.pw.begin(), L.pw.end()), rw32(L.rw.begin(), L.rw.end());
            CHK(dupload(&D.pw32, pw32, S->owned));
            CHK(dupload(&D.rptr, L.rptr, S->owned));
            CHK(dupload(&D.ridx, L.ridx, S->owned));
            CHK(dupload(&D.rw, L.rw, S->owned));
            CHK(dupload(&D.rw32, rw32, S->owned));
            D.rs_lanes = L.rs_lanes;
            CHK(dupload(&D.rs_off, L.rs_off, S->owned));
            CHK(dupload(&D.rs_idx, L.rs_idx, S->owned));
            CHK(dupload(&D.rs_w, L.rs_w, S->owned));
            if (L.n >= kRegionOrderRows) {
                const std::vector<int32_t> ord = region_order(Sl.color_slice, Sl.nslices);
                if (!ord.empty()) CHK(dupload(&D.slice_order, ord, S->owned));
                const LevelHost &Lc = levels[l + 1];
                if (!Lc.coarsest) {
                    // restriction slices (rps coarse rows each) by the coarse color of their first row
                    const int rps = 64 / L.rs_lanes, nrs = (Lc.n + rps - 1) / rps;
                    std::vector<int32_t> bounds;
                    for (int c = 0; c <= Lc.ncolors; ++c)
                        bounds.push_back(std::min(nrs, (Lc.sell.color_row[c] + rps - 1) / rps));
                    const std::vector<int32_t> rord = region_order(bounds, nrs);
                    if (!rord.empty()) CHK(dupload(&D.rs_order, rord, S->owned));
                }
            }
            std::vector<float> rsw32(L.rs_w.begin(), L.rs_w.end());
            CHK(dupload(&D.rs_w32, rsw32, S->owned));
            CHK(dupload(&D.tptr, L.tptr, S->owned));
            CHK(dupload(&D.plan1ptr, L.plan1ptr, S->owned));
            CHK(dupload(&D.plan1, L.plan1, S->owned));
            CHK(dupload(&D.plan2ptr, L.plan2ptr, S->owned));
            CHK(dupload(&D.plan2, L.plan2, S->owned));
            CHK(dupload(&D.optr, L.optr, S->owned));
            CHK(dupload(&D.opos, L.opos, S->owned));
            D.tmax = L.tmax;
            D.cmax = L.cmax;
            tmax = std::max<int64_t>(tmax, L.tptr.back());
            if (tail_rows > 0 && L.n <= tail_rows) {   // records of the LDS tail
                TailLayout T;
                build_tail_layout(L, levels[l + 1].n, kTailThreads, lpr[l], T);
                if (!check_tail_layout(T, L.n, kTailThreads, err)) return fail(SMG_ERR_INVALID_ARG, err);
                D.tl = true;
                D.tl_lg = 0;
                while ((1 << D.tl_lg) < T.grp) ++D.tl_lg;
                D.tl_npass = (int)T.pass.size() / 4;
                D.tl_nwave = (int)T.wave.size() / 2;
                D.tl_nrec = (int64_t)T.src.size();
                D.tl_rk = T.rk;
                for (size_t p = 0; p < T.pass.size(); p += 4) {   // first wavefront: global index
                    tpass_h.insert(tpass_h.end(), T.pass.begin() + p, T.pass.begin() + p + 3);
                    tpass_h.push_back(T.pass[p + 3] + nwave_before);
                }
                twave_h.insert(twave_h.end(), T.wave.begin(), T.wave.end());
                CHK(dupload(&D.tl_src, T.src, S->owned));
                CHK(dupload(&D.tl_cols, T.cols, S->owned));
                CHK(dalloc(&D.tl_rec, (size_t)std::max<int64_t>(1, D.tl_nrec), S->owned));
                CHK(dalloc(&D.tl_rec32, (size_t)std::max<int64_t>(1, D.tl_nrec), S->owned));
                CHK(dupload(&D.tl_ridx, T.ridx, S->owned));
                CHK(dupload(&D.tl_rw, T.rw, S->owned));
                std::vector<float> trw32(T.rw.begin(), T.rw.end());
                CHK(dupload(&D.tl_rw32, trw32, S->owned));
            }
        }
        D.tl_pass0 = npass_before;
        npass_before += D.tl_npass;
        D.tl_wave0 = nwave_before;
        nwave_before += D.tl_nwave;
        const size_t nk = (size_t)L.n * 4;
        CHK(dalloc(&D.x, nk, S->owned));
        CHK(dalloc(&D.b, nk, S->owned));
        CHK(dalloc(&D.r, nk, S->owned));
        CHK(dalloc(&D.x32, nk, S->owned));
        CHK(dalloc(&D.b32, nk, S->owned));
        CHK(dalloc(&D.r32, nk, S->owned));
        // release host-only setup data of this level
        L = LevelHost();
    }
    CHK(dalloc(&S->tbuf, (size_t)tmax, S->owned));
    // LDS tail: per precision and k, the finest level from which every level
    // has records and the tail's LDS footprint fits one workgroup
    {
        int dev_lds = 0;
        HIPCHK(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
        const int last = S->nlev - 1;
        std::vector<int64_t> nsum(S->nlev + 1, 0);
        for (int l = 0; l < S->nlev; ++l) nsum[l + 1] = nsum[l] + S->lev[l].n;
        size_t need[2] = {0, 0};
        for (int pr = 0; pr < 2; ++pr)
            for (int k = 1; k <= 4; ++k) {
                S->tail_first[pr][k] = last;
                S->tail_lds[pr][k].assign(S->nlev, 0);
                for (int l = last - 1; l >= 0 && S->lev[l].tl; --l) {
                    const size_t bytes = tail_lds_bytes(npass_before - S->lev[l].tl_pass0,
                                                        nwave_before - S->lev[l].tl_wave0, nsum[last + 1] - nsum[l],
                                                        S->lev[last].n, kTailPerColumn ? 1 : k, pr == 0 ? 8 : 4);
                    if (bytes > (size_t)dev_lds) break;
                    S->tail_first[pr][k] = l;
                    S->tail_lds[pr][k][l] = bytes;
                    need[pr] = std::max(need[pr], bytes);
                }
            }
        if (need[0]) HIPCHK(tail_lds_allow<double>(need[0]));
        if (need[1]) HIPCHK(tail_lds_allow<float>(need[1]));
        S->lev[last].tl_pass0 = npass_before;
        S->lev[last].tl_wave0 = nwave_before;
        if (tpass_h.empty()) tpass_h.assign(4, 0);
        if (twave_h.empty()) twave_h.assign(2, 0);
        CHK(dupload(&S->tpass, tpass_h, S->owned));
        CHK(dupload(&S->twave, twave_h, S->owned));
        std::vector<LdsLevel<double>> t64(S->nlev);
        std::vector<LdsLevel<float>> t32(S->nlev);
        for (int l = 0; l < S->nlev; ++l) {
            const DevLevel &D = S->lev[l];
            const int nc = l + 1 < S->nlev ? S->lev[l + 1].n : 0;
            t64[l] = {D.n, D.tl_lg, D.tl_pass0, D.tl_npass, D.tl_wave0, (int)nsum[l], D.tl_rec, D.diag,
                      D.b, D.r, D.x, D.pc, D.pw, D.tl_rk, nc, D.tl_ridx, D.tl_rw};
            t32[l] = {D.n, D.tl_lg, D.tl_pass0, D.tl_npass, D.tl_wave0, (int)nsum[l], D.tl_rec32, D.diag32,
                      D.b32, D.r32, D.x32, D.pc, D.pw32, D.tl_rk, nc, D.tl_ridx, D.tl_rw32};
        }
        CHK(dupload(&S->lds64, t64, S->owned));
        CHK(dupload(&S->lds32, t32, S->owned));
    }
    int64_t maxblk = (nmax + 255) / 256 + 1;
    for (const DevLevel &D : S->lev) maxblk = std::max<int64_t>(maxblk, (D.nslices + 3) / 4 + 1);
    S->npartial = 2 * 4 * maxblk;
    CHK(dalloc(&S->partial, (size_t)S->npartial, S->owned));
    CHK(dalloc(&S->norms, 16, S->owned));
    CHK(dalloc(&S->flag, 4, S->owned));
    HIPCHK(hipMemset(S->flag, 0, 4 * sizeof(int)));
    // one-XCD team: the levels as the team code reads them, and its counter
    {
        std::vector<TailLevel<double>> h64(S->nlev);
        std::vector<TailLevel<float>> h32(S->nlev);
        for (int l = 0; l < S->nlev; ++l) {
            const DevLevel &D = S->lev[l];
            const int grp = l == 0 ? 1 : 8;
            h64[l] = {D.n, D.ncolors, D.lpr, grp, D.color_row, D.slice_row0, D.slice_off, D.row_slice, D.rowlen,
                      D.cols, D.vals, D.diag, D.x, D.b, D.r, D.pc, D.pw, D.rptr, D.ridx, D.rw, D.row_base};
            h32[l] = {D.n, D.ncolors, D.lpr, grp, D.color_row, D.slice_row0, D.slice_off, D.row_slice, D.rowlen,
                      D.cols, D.vals32, D.diag32, D.x32, D.b32, D.r32, D.pc, D.pw32, D.rptr, D.ridx, D.rw32, D.row_base};
        }
        CHK(dupload(&S->team64, h64, S->owned));
        CHK(dupload(&S->team32, h32, S->owned));
        CHK(dalloc(&S->team_ctr, 64, S->owned));
    }
    // work vectors of the later entry points, so that none of them allocates:
    // damped Jacobi (a second iterate per smoothed level, power-step scratch,
    // per-level factors) and preconditioned CG (x, p, A p, column scalars)
    {
        int64_t nmax = 1;
        for (smg::DevLevel &D : S->lev)
            if (!D.coarsest) {
                nmax = std::max<int64_t>(nmax, D.n);
                CHK(dalloc(&D.xj, (size_t)D.n * 4, S->owned));
                CHK(dalloc(&D.xj32, (size_t)D.n * 4, S->owned));
            }
        CHK(dalloc(&S->jac_v, (size_t)nmax, S->owned));
        CHK(dalloc(&S->jac_u, (size_t)nmax, S->owned));
        CHK(dalloc(&S->jac_sums, 4, S->owned));
        CHK(dalloc(&S->d_omega, (size_t)S->nlev, S->owned));
        const size_t nv = (size_t)S->lev[0].n * 4;
        CHK(dalloc(&S->cg_x, nv, S->owned));
        CHK(dalloc(&S->cg_p, nv, S->owned));
        CHK(dalloc(&S->cg_ap, nv, S->owned));
        CHK(dalloc(&S->cg_s, 32, S->owned));
    }
    HIPCHK(hipHostMalloc((void **)&S->h_norms, 16 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&S->d_hnorms, S->h_norms, 0));
    HIPCHK(hipHostMalloc((void **)&S->h_flag, 4 * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipStreamCreateWithFlags(&S->gstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&S->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&S->ev_out, hipEventDisableTiming));
    HIPCHK(hipEventCreate(&S->ev_prep0));
    HIPCHK(hipEventCreate(&S->ev_prep1));
    *out = S.release();
    return SMG_OK;
}

smg_solver_s::~smg_solver_s() {
    (void)hipSetDevice(device);
    for (auto &g : graphs) if (g.exec) (void)hipGraphExecDestroy(g.exec);
    owned.release_all();
    if (h_norms) (void)hipHostFree(h_norms);
    if (h_flag) (void)hipHostFree(h_flag);
    for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : ph_pool) (void)hipEventDestroy(e);
    if (ev_prep0) (void)hipEventDestroy(ev_prep0);
    if (ev_prep1) (void)hipEventDestroy(ev_prep1);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
}

extern "C" void smg_solver_destroy(smg_solver s) { delete s; }

extern "C" int32_t smg_num_levels(smg_solver s) { return s ? s->nlev : 0; }
extern "C" int32_t smg_level_size(smg_solver s, int32_t l) {
    return (s && l >= 0 && l < s->nlev) ? s->lev[l].n : -1;
}
extern "C" int64_t smg_level_nnz(smg_solver s, int32_t l) {
    return (s && l >= 0 && l < s->nlev) ? s->lev[l].nnz_nat : -1;
}
extern "C" int32_t smg_level_colors(smg_solver s, int32_t l, int32_t *color) {
    if (!s || l < 0 || l >= s->nlev) return -1;
    const DevLevel &D = s->lev[l];
    if (color && !D.coarsest) std::copy(D.color_h.begin(), D.color_h.end(), color);
    return D.coarsest ? 0 : D.ncolors;
}

// ---------------------------------------------------------- mesh assembly
extern "C" smg_status smg_solver_attach_mesh(smg_solver s, const int32_t *F, int32_t m) {
    if (!s || !F || m < 1) return fail(SMG_ERR_INVALID_ARG, "smg_solver_attach_mesh: bad arguments");
    HIPCHK(hipSetDevice(s->device));
    const DevLevel &D = s->lev[0];
    const int n = D.n;
    auto find = [&](int i, int j) -> int {
        auto b = D.pat_idx.begin() + D.pat_ptr[i], e = D.pat_idx.begin() + D.pat_ptr[i + 1];
        auto it = std::lower_bound(b, e, j);
        return (it != e && *it == j) ? (int)(it - D.pat_idx.begin()) : -1;
    };
    std::vector<int32_t> vf_ptr(n + 1, 0), vf_face, slot_a, slot_b, diag_pos(n), eoe(D.pat_idx.size(), -1);
    for (int f = 0; f < m; ++f)
        for (int c = 0; c < 3; ++c) {
            const int v = F[3 * f + c];
            if (v < 0 || v >= n) return fail(SMG_ERR_INVALID_ARG, "face index out of range");
            vf_ptr[v + 1]++;
        }
    for (int v = 0; v < n; ++v) vf_ptr[v + 1] += vf_ptr[v];
    vf_face.resize(vf_ptr[n]);
    slot_a.resize(vf_ptr[n]);
    slot_b.resize(vf_ptr[n]);
    std::vector<int32_t> fill(vf_ptr.begin(), vf_ptr.end() - 1);
    for (int f = 0; f < m; ++f)
        for (int c = 0; c < 3; ++c) {
            const int v = F[3 * f + c], a = F[3 * f + (c + 1) % 3], b = F[3 * f + (c + 2) % 3];
            const int q = fill[v]++;
            vf_face[q] = f;
            slot_a[q] = find(v, a);
            slot_b[q] = find(v, b);
            if (slot_a[q] < 0 || slot_b[q] < 0) return fail(SMG_ERR_INVALID_ARG, "mesh edge missing from the level-0 pattern");
        }
    int32_t eid = 0;
    for (int i = 0; i < n; ++i) {
        diag_pos[i] = find(i, i);
        for (int p = D.pat_ptr[i]; p < D.pat_ptr[i + 1]; ++p)
            if (D.pat_idx[p] > i) eoe[p] = eid++;
    }
    for (int i = 0; i < n; ++i)
        for (int p = D.pat_ptr[i]; p < D.pat_ptr[i + 1]; ++p)
            if (D.pat_idx[p] < i) eoe[p] = eoe[find(D.pat_idx[p], i)];
    MeshDev &M = s->mesh;
    M.n = n;
    M.m = m;
    M.nedges = eid;
    std::vector<int32_t> Fv(F, F + 3 * (size_t)m);
    CHK(dupload(&M.faces, Fv, s->owned));
    CHK(dupload(&M.vf_ptr, vf_ptr, s->owned));
    CHK(dupload(&M.vf_face, vf_face, s->owned));
    CHK(dupload(&M.slot_a, slot_a, s->owned));
    CHK(dupload(&M.slot_b, slot_b, s->owned));
    CHK(dupload(&M.eoe, eoe, s->owned));
    CHK(dupload(&M.diag_pos, diag_pos, s->owned));
    CHK(dupload(&M.rowptr, D.pat_ptr, s->owned));
    CHK(dupload(&M.cols, D.pat_idx, s->owned));
    M.attached = true;
    return SMG_OK;
}

extern "C" smg_status smg_assemble(smg_solver s, const double *d_V, double t,
                                   const double *d_mass_scale, const float *d_edge_w,
                                   double *d_a0_vals, double *d_l_vals, double *d_mass,
                                   smg_stream stream) {
    if (!s || !d_V || !d_a0_vals) return fail(SMG_ERR_INVALID_ARG, "smg_assemble: null argument");
    if (!s->mesh.attached) return fail(SMG_ERR_STATE, "smg_assemble: no mesh attached");
    HIPCHK(hipSetDevice(s->device));
    const MeshDev &M = s->mesh;
    MeshView mv{M.n, M.vf_ptr, M.vf_face, M.faces, M.slot_a, M.slot_b, M.eoe, M.diag_pos, M.rowptr};
    HIPCHK(launch_assemble(mv, d_V, t, d_mass_scale, d_edge_w, d_a0_vals, d_l_vals, d_mass,
                           (hipStream_t)stream));
    return SMG_OK;
}

// -------------------------------------------------------- hierarchy values
extern "C" smg_status smg_set_values(smg_solver s, const double *d_a0_vals, smg_stream stream) {
    if (!s || !d_a0_vals) return fail(SMG_ERR_INVALID_ARG, "smg_set_values: null argument");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipEventRecord(s->ev_prep0, st));
    CHK(refresh_values(s, d_a0_vals, st));
    HIPCHK(hipEventRecord(s->ev_prep1, st));
    HIPCHK(hipMemcpyAsync(s->h_flag, s->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, s->ev_prep0, s->ev_prep1));
        s->ms_prepare = ms;
    }
    if (s->h_flag[0]) { s->values_set = false; return fail(SMG_ERR_NONFINITE, "non-finite matrix value"); }
    if (s->h_flag[1]) { s->values_set = false; return fail(SMG_ERR_NOT_SPD, "coarsest Cholesky: non-positive pivot"); }
    s->values_set = true;
    return SMG_OK;
}

// ------------------------------------------- split Galerkin (App. E)
// Galerkin products are linear in A: P^T (a Q + b M) P = a P^T Q P + b P^T M P.
// smg_split_prepare keeps every level of Q and of M; smg_split_combine forms
// the levels of a Q + b M with one axpby per level.
static smg_status split_keep(smg_solver_s *s, int which, hipStream_t st) {
    for (DevLevel &D : s->lev) {
        double *v = which ? D.sm_vals : D.sq_vals, *d = which ? D.sm_diag : D.sq_diag;
        if (D.coarsest) {
            HIPCHK(hipMemcpyAsync(v, D.dense_a, (size_t)D.n * D.n * sizeof(double), hipMemcpyDeviceToDevice, st));
        } else {
            HIPCHK(hipMemcpyAsync(v, D.vals, (size_t)D.slots * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(d, D.diag, (size_t)D.n * sizeof(double), hipMemcpyDeviceToDevice, st));
        }
    }
    return SMG_OK;
}

extern "C" smg_status smg_split_prepare(smg_solver s, const double *d_q_vals, const double *d_m_vals,
                                        smg_stream stream) {
    if (!s || !d_q_vals || !d_m_vals) return fail(SMG_ERR_INVALID_ARG, "smg_split_prepare: null argument");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    if (!s->split_ready_alloc) {
        for (DevLevel &D : s->lev) {
            const size_t nv = D.coarsest ? (size_t)D.n * D.n : (size_t)D.slots;
            CHK(dalloc(&D.sq_vals, nv, s->owned));
            CHK(dalloc(&D.sm_vals, nv, s->owned));
            if (!D.coarsest) {
                CHK(dalloc(&D.sq_diag, (size_t)D.n, s->owned));
                CHK(dalloc(&D.sm_diag, (size_t)D.n, s->owned));
            }
        }
        s->split_ready_alloc = true;
    }
    s->values_set = false;
    s->split_ready = false;
    int bad = 0;
    for (int which = 0; which < 2; ++which) {
        CHK(galerkin_values(s, which ? d_m_vals : d_q_vals, st));
        CHK(split_keep(s, which, st));
        HIPCHK(hipMemcpyAsync(s->h_flag, s->flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bad |= s->h_flag[0];
    }
    if (bad) return fail(SMG_ERR_NONFINITE, "non-finite matrix value");
    s->split_ready = true;
    return SMG_OK;
}

extern "C" smg_status smg_split_combine(smg_solver s, double a, double b, smg_stream stream) {
    if (!s) return fail(SMG_ERR_INVALID_ARG, "null solver");
    if (!s->split_ready) return fail(SMG_ERR_STATE, "smg_split_prepare has not run");
    if (!std::isfinite(a) || !std::isfinite(b)) return fail(SMG_ERR_INVALID_ARG, "non-finite coefficient");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipEventRecord(s->ev_prep0, st));
    HIPCHK(launch_fill<int>(s->flag, 0, 2, st));
    for (DevLevel &D : s->lev) {
        if (D.coarsest) {
            HIPCHK(launch_axpby((int64_t)D.n * D.n, a, D.sq_vals, b, D.sm_vals, D.dense_a, st));
        } else {
            HIPCHK(launch_axpby(D.slots, a, D.sq_vals, b, D.sm_vals, D.vals, st));
            HIPCHK(launch_axpby(D.n, a, D.sq_diag, b, D.sm_diag, D.diag, st));
        }
    }
    CHK(finish_values(s, st));
    HIPCHK(hipEventRecord(s->ev_prep1, st));
    HIPCHK(hipMemcpyAsync(s->h_flag, s->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, s->ev_prep0, s->ev_prep1));
        s->ms_prepare = ms;
    }
    if (s->h_flag[1]) { s->values_set = false; return fail(SMG_ERR_NOT_SPD, "coarsest Cholesky: non-positive pivot"); }
    s->values_set = true;
    return SMG_OK;
}

namespace smg {

smg_status refresh_values(smg_solver_s *s, const double *d_a0_vals, hipStream_t st) {
    CHK(galerkin_values(s, d_a0_vals, st));
    return finish_values(s, st);
}

// A_0 values into level 0 and every Galerkin product A_{l+1} = P_l^T A_l P_l
// (FP64 values and diagonals, dense A_H on the coarsest level)
smg_status galerkin_values(smg_solver_s *s, const double *d_a0_vals, hipStream_t st) {
    HIPCHK(launch_fill<int>(s->flag, 0, 2, st));
    for (int l = 0; l < s->nlev; ++l) {
        DevLevel &D = s->lev[l];
        if (D.coarsest) HIPCHK(launch_fill<double>(D.dense_a, 0.0, (int64_t)D.n * D.n, st));
        else {
            HIPCHK(launch_fill<double>(D.vals, 0.0, D.slots, st));
            HIPCHK(launch_fill<double>(D.diag, 0.0, D.n, st));
        }
    }
    DevLevel &L0 = s->lev[0];
    HIPCHK(launch_scatter_values(d_a0_vals, L0.store, L0.nnz_nat, L0.coarsest ? L0.dense_a : L0.vals,
                                 L0.coarsest ? nullptr : L0.diag, s->flag, st));
    for (int l = 0; l + 1 < s->nlev; ++l) {
        DevLevel &D = s->lev[l];
        DevLevel &C = s->lev[l + 1];
        HIPCHK(launch_galerkin_t(D.n, D.tmax, D.tptr, D.plan1ptr, D.plan1, D.row_slice, D.slice_row0,
                                 D.slice_off, D.lpr, D.rowlen, D.cols, D.vals, D.diag, D.pw, s->tbuf, st));
        HIPCHK(launch_galerkin_c(C.n, D.cmax, D.plan2ptr, D.plan2, D.rptr, D.ridx, D.rw, D.tptr, s->tbuf,
                                 D.optr, D.opos, C.coarsest ? C.dense_a : C.vals, C.coarsest ? nullptr : C.diag, st));
    }
    return SMG_OK;
}

// everything derived from the FP64 level values: FP32 copies, LDS-tail
// records, the coarsest factor and inverse, Jacobi factors
smg_status finish_values(smg_solver_s *s, hipStream_t st) {
    for (int l = 0; l < s->nlev; ++l) {
        DevLevel &D = s->lev[l];
        if (D.coarsest) continue;
        HIPCHK(launch_to_f32(D.vals, D.vals32, D.slots, st));
        HIPCHK(launch_to_f32(D.diag, D.diag32, D.n, st));
    }
    for (int l = 0; l < s->nlev; ++l) {
        DevLevel &D = s->lev[l];
        if (D.tl) HIPCHK(launch_gather_records(D.tl_src, D.tl_cols, D.tl_nrec, D.vals, D.vals32, D.tl_rec, D.tl_rec32, st));
    }
    DevLevel &Lc = s->lev[s->nlev - 1];
    HIPCHK(hipMemcpyAsync(Lc.dense, Lc.dense_a, (size_t)Lc.n * Lc.n * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_cholesky(Lc.dense, Lc.n, s->flag + 1, st));
    HIPCHK(launch_coarse_inverse(Lc.dense, Lc.n, Lc.dense_w, Lc.dense_inv, st));
    if (s->smoother == SMG_SMOOTH_JACOBI) CHK(jacobi_factors(s, st));
    return SMG_OK;
}

// Jacobi factor of every smoothed level into d_omega: the set factor, or
// 2 / (1 + lambda_l) from the power-step estimate of lambda_max(D^{-1} A_l).
smg_status jacobi_factors(smg_solver_s *s, hipStream_t st) {
    for (int l = 0; l < s->nlev; ++l) {
        DevLevel &D = s->lev[l];
        if (D.coarsest) continue;
        if (s->omega > 0.0) HIPCHK(launch_fill<double>(s->d_omega + l, s->omega, 1, st));
        else HIPCHK(launch_jacobi_factor(SellView<double>{D.n, D.lpr, D.slice_row0, D.slice_off, D.cols, D.vals, D.diag},
                                         D.n, D.nslices, D.perm, s->jac_v, s->jac_u,
                                         s->partial, s->jac_sums, s->d_omega + l, st));
    }
    return SMG_OK;
}

}  // namespace smg

extern "C" smg_status smg_get_level_matrix(smg_solver s, int32_t l, int32_t *rowptr, int32_t *cols,
                                           double *vals) {
    if (!s || l < 0 || l >= s->nlev || !rowptr || !cols || !vals) return fail(SMG_ERR_INVALID_ARG, "bad arguments");
    if (!s->values_set) return fail(SMG_ERR_STATE, "values not set");
    HIPCHK(hipSetDevice(s->device));
    const DevLevel &D = s->lev[l];
    std::copy(D.pat_ptr.begin(), D.pat_ptr.end(), rowptr);
    std::copy(D.pat_idx.begin(), D.pat_idx.end(), cols);
    if (D.coarsest) {
        std::vector<double> dense((size_t)D.n * D.n);
        HIPCHK(hipMemcpy(dense.data(), D.dense_a, dense.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t p = 0; p < D.store_h.size(); ++p) vals[p] = dense[D.store_h[p]];
    } else {
        std::vector<double> sv((size_t)D.slots), dg(D.n);
        HIPCHK(hipMemcpy(sv.data(), D.vals, sv.size() * sizeof(double), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(dg.data(), D.diag, dg.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t p = 0; p < D.store_h.size(); ++p) {
            const int32_t sp = D.store_h[p];
            vals[p] = sp >= 0 ? sv[sp] : dg[-1 - sp];
        }
    }
    return SMG_OK;
}

extern "C" smg_status smg_get_coarse_factor(smg_solver s, double *G) {
    if (!s || !G) return fail(SMG_ERR_INVALID_ARG, "bad arguments");
    if (!s->values_set) return fail(SMG_ERR_STATE, "values not set");
    HIPCHK(hipSetDevice(s->device));
    const DevLevel &D = s->lev[s->nlev - 1];
    HIPCHK(hipMemcpy(G, D.dense, (size_t)D.n * D.n * sizeof(double), hipMemcpyDeviceToHost));
    return SMG_OK;
}

// ----------------------------------------------------------- V-cycle core
namespace smg {

template <typename T>
static SellView<T> sell_view(const DevLevel &D);
template <>
SellView<double> sell_view<double>(const DevLevel &D) {
    return {D.n, D.lpr, D.slice_row0, D.slice_off, D.cols, D.vals, D.diag, D.slice_order};
}
template <>
SellView<float> sell_view<float>(const DevLevel &D) {
    return {D.n, D.lpr, D.slice_row0, D.slice_off, D.cols, D.vals32, D.diag32, D.slice_order};
}
template <typename T> static const TailLevel<T> *team_desc(const smg_solver_s *s);
template <> const TailLevel<double> *team_desc<double>(const smg_solver_s *s) { return s->team64; }
template <> const TailLevel<float> *team_desc<float>(const smg_solver_s *s) { return s->team32; }
template <typename T> static const LdsLevel<T> *tail_desc(const smg_solver_s *s);
template <> const LdsLevel<double> *tail_desc<double>(const smg_solver_s *s) { return s->lds64; }
template <> const LdsLevel<float> *tail_desc<float>(const smg_solver_s *s) { return s->lds32; }
static TransferView transfer_view(const DevLevel &D, const DevLevel &C) {
    return {D.n, C.n, D.rs_lanes, D.pc, D.rs_off, D.rs_idx, D.rs_order};
}
template <typename T> static T *xbuf(DevLevel &D);
template <> double *xbuf<double>(DevLevel &D) { return D.x; }
template <> float *xbuf<float>(DevLevel &D) { return D.x32; }
template <typename T> static T *bbuf(DevLevel &D);
template <> double *bbuf<double>(DevLevel &D) { return D.b; }
template <> float *bbuf<float>(DevLevel &D) { return D.b32; }
template <typename T> static T *rbuf(DevLevel &D);
template <> double *rbuf<double>(DevLevel &D) { return D.r; }
template <> float *rbuf<float>(DevLevel &D) { return D.r32; }
template <typename T> static const T *pwbuf(const DevLevel &D);
template <> const double *pwbuf<double>(const DevLevel &D) { return D.pw; }
template <> const float *pwbuf<float>(const DevLevel &D) { return D.pw32; }
template <typename T> static const T *rwbuf(const DevLevel &D);
template <> const double *rwbuf<double>(const DevLevel &D) { return D.rs_w; }
template <> const float *rwbuf<float>(const DevLevel &D) { return D.rs_w32; }

template <typename T> T *xjbuf(DevLevel &D);
template <> double *xjbuf<double>(DevLevel &D) { return D.xj; }
template <> float *xjbuf<float>(DevLevel &D) { return D.xj32; }

// damped Jacobi sweeps: x -> xj -> x ...; an odd count copies the result back.
// x_zero: the iterate is zero on entry (a coarse level's pre-relaxation), so
// the first sweep needs no matrix.
// Algorithmic bytes of a relaxation sweep or residual over rows holding z
// matrix entries (diagonal included) and n rows: what a CSR sweep must move,
// z (s + 4) for values and column indices, 4 (n + 1) for row pointers, and
// 3 k n s for b, x read and x (or r) written, with s bytes per value and
// neighbour values of x counted once.  A color of a sweep gets its own rows'
// share and the first color the one extra row pointer.
static double sweep_bytes(int64_t z, int64_t n, int k, double sb, bool first) {
    return (double)z * (sb + 4) + 4.0 * (double)(n + (first ? 1 : 0)) + 3.0 * k * (double)n * sb;
}

template <typename T>
smg_status jacobi_level(smg_solver_s *s, int l, int k, int sweeps, hipStream_t st, bool x_zero) {
    phase_mark(s, st, SMG_PHASE_RELAX);
    DevLevel &D = s->lev[l];
    const SellView<T> A = sell_view<T>(D);
    const double sb = sizeof(T);
    T *x = xbuf<T>(D), *y = xjbuf<T>(D);
    for (int sw = 0; sw < sweeps; ++sw) {
        if (sw == 0 && x_zero) {
            HIPCHK(launch_jacobi_first<T>(D.n, k, A.diag, bbuf<T>(D), y, s->d_omega + l, st));
            continue;
        }
        const int pi = prof_begin(s, SMG_PROF_GS, l, sweep_bytes(D.offdiag_nnz + D.n, D.n, k, sb, true), st);
        HIPCHK(launch_jacobi<T>(A, D.nslices, bbuf<T>(D), sw % 2 ? y : x, sw % 2 ? x : y, s->d_omega + l, k, st,
                                prof_ev(s, pi, 0), prof_ev(s, pi, 1)));
    }
    if (sweeps % 2) HIPCHK(hipMemcpyAsync(x, y, (size_t)D.n * k * sizeof(T), hipMemcpyDeviceToDevice, st));
    return SMG_OK;
}

template <typename T>
smg_status smooth_level(smg_solver_s *s, int l, int k, int sweeps, hipStream_t st, bool descending = false,
                        bool x_zero = false) {
    if (s->smoother == SMG_SMOOTH_JACOBI) return jacobi_level<T>(s, l, k, sweeps, st, x_zero);
    phase_mark(s, st, SMG_PHASE_RELAX);
    DevLevel &D = s->lev[l];
    const SellView<T> A = sell_view<T>(D);
    const double sb = sizeof(T);
    // group timing: one event pair around all of this call's launches
    const int pg = s->prof_group ? prof_begin(s, SMG_PROF_GS, l, sweeps * sweep_bytes(D.offdiag_nnz + D.n, D.n, k, sb, true),
                                              st, (int64_t)sweeps * D.ncolors)
                                 : -1;
    if (pg >= 0) HIPCHK(hipEventRecord(prof_ev(s, pg, 0), st));
    for (int sw = 0; sw < sweeps; ++sw)
        for (int cc = 0; cc < D.ncolors; ++cc) {
            const int c = descending ? D.ncolors - 1 - cc : cc;
            const int pi = s->prof_group ? -1
                                         : prof_begin(s, SMG_PROF_GS, l,
                                                      sweep_bytes(D.color_nnz[c] + D.color_rows[c], D.color_rows[c],
                                                                  k, sb, cc == 0),
                                                      st);
            const ColorSpan span{D.color_slice[c], D.color_slice[c + 1], D.color_row_h[c], D.color_row_h[c + 1],
                                 D.color_off[c], D.color_w[c]};
            HIPCHK(launch_gs_color<T>(A, span, bbuf<T>(D), xbuf<T>(D), k, st,
                                      prof_ev(s, pi, 0), prof_ev(s, pi, 1)));
        }
    if (pg >= 0) HIPCHK(hipEventRecord(prof_ev(s, pg, 1), st));
    return SMG_OK;
}

template <typename T>
smg_status residual_level(smg_solver_s *s, int l, int k, bool norms, hipStream_t st) {
    phase_mark(s, st, norms ? SMG_PHASE_NORM : SMG_PHASE_TRANSFER);
    DevLevel &D = s->lev[l];
    int nblk = 0;
    const double sb = sizeof(T);
    const int pi = prof_begin(s, SMG_PROF_RESIDUAL, l, sweep_bytes(D.offdiag_nnz + D.n, D.n, k, sb, true), st);
    HIPCHK(launch_residual<T>(sell_view<T>(D), D.nslices, bbuf<T>(D), xbuf<T>(D), rbuf<T>(D), k,
                              norms ? s->partial : nullptr, &nblk, st, prof_ev(s, pi, 0), prof_ev(s, pi, 1)));
    if (norms) HIPCHK(launch_reduce_partial(s->partial, nblk, k, s->norms, st, s->d_hnorms, s->norm_seq));
    return SMG_OK;
}

// Alg. "V-cycle" from level l with b_l, x_l in the level buffers (x_l in/out).
// `part` splits off level l's pre-relaxation (empty when level l is the
// coarsest or runs in the LDS tail); `sym` runs the post-relaxation's colors
// in descending order (the cycle is then symmetric, for CG).
template <typename T>
smg_status vcycle_from(smg_solver_s *s, int l, int k, hipStream_t st, int part, bool sym) {
    DevLevel &D = s->lev[l];
    if (D.coarsest) {
        phase_mark(s, st, SMG_PHASE_OTHER);
        if (part != kCyclePre)
            HIPCHK((launch_coarse_solve<T, T>(D.dense_inv, D.n, bbuf<T>(D), xbuf<T>(D), k, st)));
        return SMG_OK;
    }
    const int pr = sizeof(T) == 8 ? 0 : 1;
    if (s->smoother == SMG_SMOOTH_GS && s->team_level > 0 && l == s->team_level && !sym) {
        phase_mark(s, st, SMG_PHASE_RELAX);
        if (part != kCyclePre)
            HIPCHK(launch_team_vcycle<T>(team_desc<T>(s), l, s->nlev, s->mu_pre, s->mu_post,
                                         s->lev[s->nlev - 1].dense_inv, s->team_ctr, s->flag + 2, s->team_size, k,
                                         st));
        return SMG_OK;
    }
    if (s->smoother == SMG_SMOOTH_GS && l >= s->tail_first[pr][k]) {   // this level and all coarser ones in one launch
        phase_mark(s, st, SMG_PHASE_RELAX);
        if (part != kCyclePre)
            HIPCHK(launch_tail_lds<T>(tail_desc<T>(s), s->tpass, s->twave, l, s->nlev, s->mu_pre, s->mu_post,
                                      s->lev[s->nlev - 1].dense_inv, k, s->tail_lds[pr][k][l], st, sym,
                                      kTailPerColumn));
        return SMG_OK;
    }
    DevLevel &C = s->lev[l + 1];
    const TransferView P = transfer_view(D, C);
    // pre-relaxation; below level 0 the iterate starts at zero (cleared by the restriction)
    if (part != kCycleAfterPre) CHK(smooth_level<T>(s, l, k, s->mu_pre, st, false, l > 0));
    if (part == kCyclePre) return SMG_OK;
    CHK(residual_level<T>(s, l, k, false, st));                    // r = b - A x'
    // P^T r; the coarse iterate starts from zero
    phase_mark(s, st, SMG_PHASE_TRANSFER);
    HIPCHK(launch_restrict<T>(P, rwbuf<T>(D), rbuf<T>(D), bbuf<T>(C), k, st, C.coarsest ? nullptr : xbuf<T>(C)));
    CHK(vcycle_from<T>(s, l + 1, k, st, kCycleWhole, sym));        // coarse correction
    phase_mark(s, st, SMG_PHASE_TRANSFER);
    HIPCHK(launch_prolong_add<T>(P, pwbuf<T>(D), xbuf<T>(C), xbuf<T>(D), k, st));  // x' + P c
    CHK(smooth_level<T>(s, l, k, s->mu_post, st, sym));            // post-relaxation
    return SMG_OK;
}

template smg_status vcycle_from<double>(smg_solver_s *, int, int, hipStream_t, int, bool);
template smg_status vcycle_from<float>(smg_solver_s *, int, int, hipStream_t, int, bool);
template smg_status residual_level<double>(smg_solver_s *, int, int, bool, hipStream_t);
template smg_status residual_level<float>(smg_solver_s *, int, int, bool, hipStream_t);

}  // namespace smg

// ----------------------------------------------------- per-step entry points
static smg_status check_level(smg_solver s, int l, int k) {
    if (!s) return fail(SMG_ERR_INVALID_ARG, "null solver");
    if (l < 0 || l >= s->nlev) return fail(SMG_ERR_INVALID_ARG, "level out of range");
    if (k < 1 || k > 4) return fail(SMG_ERR_INVALID_ARG, "k must be 1..4");
    if (!s->values_set) return fail(SMG_ERR_STATE, "values not set");
    return SMG_OK;
}

static smg_status check_precision(int precision) {
    if (precision != SMG_FP64 && precision != SMG_FP32_IR) return fail(SMG_ERR_INVALID_ARG, "bad precision");
    return SMG_OK;
}

namespace smg {

// The per-step entry points in one value type: caller vectors (FP64, natural
// order) are gathered into the level's permuted buffers of type T (rounded to
// FP32 for T = float), the step runs on them, and the result is scattered back.
template <typename T>
static smg_status step_residual(smg_solver_s *s, int l, const double *d_b, const double *d_x, double *d_r, int k,
                                hipStream_t st) {
    DevLevel &D = s->lev[l];
    HIPCHK(launch_gather_rows(D.perm, d_b, bbuf<T>(D), D.n, k, st));
    HIPCHK(launch_gather_rows(D.perm, d_x, xbuf<T>(D), D.n, k, st));
    CHK(residual_level<T>(s, l, k, false, st));
    HIPCHK(launch_scatter_rows(D.perm, (const T *)rbuf<T>(D), d_r, D.n, k, st));
    return SMG_OK;
}
template <typename T>
static smg_status step_smooth(smg_solver_s *s, int l, const double *d_b, double *d_x, int k, int sweeps,
                              hipStream_t st) {
    DevLevel &D = s->lev[l];
    HIPCHK(launch_gather_rows(D.perm, d_b, bbuf<T>(D), D.n, k, st));
    HIPCHK(launch_gather_rows(D.perm, (const double *)d_x, xbuf<T>(D), D.n, k, st));
    CHK(smooth_level<T>(s, l, k, sweeps, st));
    HIPCHK(launch_scatter_rows(D.perm, (const T *)xbuf<T>(D), d_x, D.n, k, st));
    return SMG_OK;
}
template <typename T>
static smg_status step_restrict(smg_solver_s *s, int l, const double *d_r, double *d_rc, int k, hipStream_t st) {
    DevLevel &D = s->lev[l], &C = s->lev[l + 1];
    HIPCHK(launch_gather_rows(D.perm, d_r, rbuf<T>(D), D.n, k, st));
    HIPCHK(launch_restrict<T>(transfer_view(D, C), rwbuf<T>(D), rbuf<T>(D), bbuf<T>(C), k, st));
    HIPCHK(launch_scatter_rows(C.perm, (const T *)bbuf<T>(C), d_rc, C.n, k, st));
    return SMG_OK;
}
template <typename T>
static smg_status step_prolong_add(smg_solver_s *s, int l, const double *d_e, double *d_x, int k, hipStream_t st) {
    DevLevel &D = s->lev[l], &C = s->lev[l + 1];
    HIPCHK(launch_gather_rows(C.perm, d_e, xbuf<T>(C), C.n, k, st));
    HIPCHK(launch_gather_rows(D.perm, (const double *)d_x, xbuf<T>(D), D.n, k, st));
    HIPCHK(launch_prolong_add<T>(transfer_view(D, C), pwbuf<T>(D), xbuf<T>(C), xbuf<T>(D), k, st));
    HIPCHK(launch_scatter_rows(D.perm, (const T *)xbuf<T>(D), d_x, D.n, k, st));
    return SMG_OK;
}

}  // namespace smg

extern "C" smg_status smg_residual(smg_solver s, int32_t l, int32_t precision, const double *d_b,
                                   const double *d_x, double *d_r, int32_t k, smg_stream stream) {
    CHK(check_level(s, l, k));
    CHK(check_precision(precision));
    if (!d_b || !d_x || !d_r) return fail(SMG_ERR_INVALID_ARG, "null vector");
    if (s->lev[l].coarsest) return fail(SMG_ERR_INVALID_ARG, "residual on the coarsest level is not part of the cycle");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    return precision == SMG_FP64 ? step_residual<double>(s, l, d_b, d_x, d_r, k, st)
                                 : step_residual<float>(s, l, d_b, d_x, d_r, k, st);
}

extern "C" smg_status smg_smooth(smg_solver s, int32_t l, int32_t precision, const double *d_b, double *d_x,
                                 int32_t k, int32_t sweeps, smg_stream stream) {
    CHK(check_level(s, l, k));
    CHK(check_precision(precision));
    if (!d_b || !d_x || sweeps < 0) return fail(SMG_ERR_INVALID_ARG, "bad arguments");
    if (s->lev[l].coarsest) return fail(SMG_ERR_INVALID_ARG, "the coarsest level is not smoothed");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    return precision == SMG_FP64 ? step_smooth<double>(s, l, d_b, d_x, k, sweeps, st)
                                 : step_smooth<float>(s, l, d_b, d_x, k, sweeps, st);
}

extern "C" smg_status smg_restrict(smg_solver s, int32_t l, int32_t precision, const double *d_r, double *d_rc,
                                   int32_t k, smg_stream stream) {
    CHK(check_level(s, l, k));
    CHK(check_precision(precision));
    if (l + 1 >= s->nlev || !d_r || !d_rc) return fail(SMG_ERR_INVALID_ARG, "bad arguments");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    return precision == SMG_FP64 ? step_restrict<double>(s, l, d_r, d_rc, k, st)
                                 : step_restrict<float>(s, l, d_r, d_rc, k, st);
}

extern "C" smg_status smg_prolong_add(smg_solver s, int32_t l, int32_t precision, const double *d_e, double *d_x,
                                      int32_t k, smg_stream stream) {
    CHK(check_level(s, l, k));
    CHK(check_precision(precision));
    if (l + 1 >= s->nlev || !d_e || !d_x) return fail(SMG_ERR_INVALID_ARG, "bad arguments");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    return precision == SMG_FP64 ? step_prolong_add<double>(s, l, d_e, d_x, k, st)
                                 : step_prolong_add<float>(s, l, d_e, d_x, k, st);
}

static_assert(SMG_TAIL_RELAX == kTailStepRelax && SMG_TAIL_RESIDUAL == kTailStepResidual &&
                  SMG_TAIL_RESTRICT == kTailStepRestrict && SMG_TAIL_PROLONG == kTailStepProlong &&
                  SMG_TAIL_COARSE == kTailStepCoarse,
              "tail step codes of the ABI and the kernels");

namespace smg {

// One step of the one-workgroup tail (see smg_tail_step) in value type T.
template <typename T>
static smg_status tail_step(smg_solver_s *s, int l, int step, const double *d_in, const double *d_in2,
                            double *d_out, int k, int sweeps, bool desc, hipStream_t st) {
    DevLevel &D = s->lev[l];
    const int last = s->nlev - 1;
    const int nc = l < last ? s->lev[l + 1].n : 0;
    int np = 0, nw = 0;
    if (l < last) { np = D.tl_npass; nw = s->lev[l + 1].tl_wave0 - D.tl_wave0; }
    const size_t bytes = tail_step_lds_bytes(np, nw, D.n, step == kTailStepCoarse ? D.n : nc, sizeof(T));
    switch (step) {
    case kTailStepRelax:
        HIPCHK(launch_gather_rows(D.perm, d_in, bbuf<T>(D), D.n, k, st));
        HIPCHK(launch_gather_rows(D.perm, (const double *)d_out, xbuf<T>(D), D.n, k, st));
        break;
    case kTailStepResidual:
        HIPCHK(launch_gather_rows(D.perm, d_in, bbuf<T>(D), D.n, k, st));
        HIPCHK(launch_gather_rows(D.perm, d_in2, xbuf<T>(D), D.n, k, st));
        break;
    case kTailStepRestrict:
        HIPCHK(launch_gather_rows(D.perm, d_in, rbuf<T>(D), D.n, k, st));
        break;
    case kTailStepProlong:
        HIPCHK(launch_gather_rows(s->lev[l + 1].perm, d_in, xbuf<T>(s->lev[l + 1]), nc, k, st));
        HIPCHK(launch_gather_rows(D.perm, (const double *)d_out, xbuf<T>(D), D.n, k, st));
        break;
    default:
        HIPCHK(launch_gather_rows(D.perm, d_in, bbuf<T>(D), D.n, k, st));
    }
    HIPCHK(launch_tail_step<T>(tail_desc<T>(s), s->tpass, s->twave, l, s->nlev, step, sweeps, desc,
                               s->lev[last].dense_inv, k, bytes, st));
    switch (step) {
    case kTailStepResidual: HIPCHK(launch_scatter_rows(D.perm, (const T *)rbuf<T>(D), d_out, D.n, k, st)); break;
    case kTailStepRestrict:
        HIPCHK(launch_scatter_rows(s->lev[l + 1].perm, (const T *)bbuf<T>(s->lev[l + 1]), d_out, nc, k, st));
        break;
    default: HIPCHK(launch_scatter_rows(D.perm, (const T *)xbuf<T>(D), d_out, D.n, k, st));
    }
    return SMG_OK;
}

}  // namespace smg

extern "C" int32_t smg_tail_first_level(smg_solver s, int32_t precision, int32_t k) {
    if (!s || (precision != SMG_FP64 && precision != SMG_FP32_IR) || k < 1 || k > 4) return -1;
    if (s->smoother != SMG_SMOOTH_GS) return s->nlev - 1;   // Jacobi cycles use no tail
    return s->tail_first[precision == SMG_FP64 ? 0 : 1][k];
}

extern "C" smg_status smg_tail_step(smg_solver s, int32_t level, int32_t step, int32_t precision,
                                    const double *d_in, const double *d_in2, double *d_out, int32_t k,
                                    int32_t sweeps, smg_stream stream) {
    CHK(check_level(s, level, k));
    CHK(check_precision(precision));
    if (step < SMG_TAIL_RELAX || step > SMG_TAIL_COARSE) return fail(SMG_ERR_INVALID_ARG, "unknown tail step");
    const int last = s->nlev - 1;
    const int pr = precision == SMG_FP64 ? 0 : 1;
    if ((step == SMG_TAIL_COARSE) != (level == last))
        return fail(SMG_ERR_INVALID_ARG, "the coarsest solve is the only step on the coarsest level");
    if (level < last && level < s->tail_first[pr][k])
        return fail(SMG_ERR_INVALID_ARG, "level is not in the one-workgroup tail for this precision and k");
    if (!d_in || !d_out || (step == SMG_TAIL_RESIDUAL && !d_in2)) return fail(SMG_ERR_INVALID_ARG, "null vector");
    if (step == SMG_TAIL_RELAX && sweeps == 0) return SMG_OK;
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    const bool desc = sweeps < 0;
    const int sw = sweeps < 0 ? -sweeps : sweeps;
    return pr == 0 ? tail_step<double>(s, level, step, d_in, d_in2, d_out, k, sw, desc, st)
                   : tail_step<float>(s, level, step, d_in, d_in2, d_out, k, sw, desc, st);
}

extern "C" smg_status smg_coarse_solve(smg_solver s, int32_t precision, const double *d_b, double *d_x, int32_t k,
                                       smg_stream stream) {
    if (!s) return fail(SMG_ERR_INVALID_ARG, "null solver");
    CHK(check_level(s, s->nlev - 1, k));
    CHK(check_precision(precision));
    if (!d_b || !d_x) return fail(SMG_ERR_INVALID_ARG, "null vector");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    DevLevel &D = s->lev[s->nlev - 1];
    if (precision == SMG_FP64) {
        HIPCHK((launch_coarse_solve<double, double>(D.dense_inv, D.n, d_b, d_x, k, st)));
    } else {
        HIPCHK(launch_gather_rows(D.perm, d_b, D.b32, D.n, k, st));
        HIPCHK((launch_coarse_solve<float, float>(D.dense_inv, D.n, D.b32, D.x32, k, st)));
        HIPCHK(launch_scatter_rows(D.perm, (const float *)D.x32, d_x, D.n, k, st));
    }
    return SMG_OK;
}

extern "C" smg_status smg_vcycle(smg_solver s, int32_t precision, const double *d_b, double *d_x, int32_t k,
                                 smg_stream stream) {
    CHK(check_level(s, 0, k));
    CHK(check_precision(precision));
    if (!d_b || !d_x) return fail(SMG_ERR_INVALID_ARG, "null vector");
    if (s->lev[0].coarsest && precision != SMG_FP64)
        return fail(SMG_ERR_INVALID_ARG, "a one-level hierarchy has no refinement cycle (its cycle is the FP64 direct solve)");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    DevLevel &D = s->lev[0];
    HIPCHK(launch_gather_rows(D.perm, d_b, D.b, D.n, k, st));
    HIPCHK(launch_gather_rows(D.perm, (const double *)d_x, D.x, D.n, k, st));
    if (precision == SMG_FP64) {
        CHK(vcycle_from<double>(s, 0, k, st));
    } else {
        // one refinement step: r = b - A x and max |r| per column (FP64), then
        // the FP32 cycle on r / max|r| from zero and x += max|r| * d (FP64)
        CHK(residual_level<double>(s, 0, k, true, st));
        HIPCHK(launch_fill<float>(D.x32, 0.0f, (int64_t)D.n * k, st));
        HIPCHK(launch_ir_down(D.r, s->norms, D.b32, D.n, k, st));
        CHK(vcycle_from<float>(s, 0, k, st));
        HIPCHK(launch_ir_up(D.x32, s->norms, D.x, D.n, k, st));
    }
    HIPCHK(launch_scatter_rows(D.perm, (const double *)D.x, d_x, D.n, k, st));
    return SMG_OK;
}

// ------------------------------------------------------------------ solve
namespace smg {

// The one-XCD team raises flag[2] when a workgroup ran on another XCD or a
// barrier wait timed out; the result of that solve is then not to be used.
static smg_status check_team(smg_solver_s *s, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(s->h_flag + 2, s->flag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (s->h_flag[2]) {
        const int code = s->h_flag[2];
        HIPCHK(launch_fill<int>(s->flag + 2, 0, 1, st));
        HIPCHK(hipStreamSynchronize(st));
        return fail(SMG_ERR_HIP, "team V-cycle: a barrier wait timed out (code " + std::to_string(code) + ")");
    }
    return SMG_OK;
}

// Wait for the column norms (sum of squares, max) of the last reduction: the
// reduction kernel writes them to h_norms itself (no copy back), so this only
// waits, polling, for the stream to drain.
static smg_status fetch_norms(smg_solver_s *s, int k, hipStream_t st) {
    (void)k;
    for (;;) {
        const hipError_t e = hipStreamQuery(st);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) return fail(SMG_ERR_HIP, std::string("hipStreamQuery: ") + hipGetErrorString(e));
    }
    return SMG_OK;
}

// Wait until the norm reduction tagged `seq` has written its k column norms to
// h_norms; work enqueued after it keeps the device busy meanwhile.  The wait
// ends with the stream at the latest: a drained stream without the tag is an
// error.
static smg_status wait_norms(smg_solver_s *s, int k, double seq, hipStream_t st) {
    volatile double *tag = s->h_norms + 2 * k;
    for (unsigned it = 1;; ++it) {
        if (*tag == seq) break;
        if ((it & 1023) == 0) {
            const hipError_t e = hipStreamQuery(st);
            if (e == hipSuccess) {
                if (*tag == seq) break;
                return fail(SMG_ERR_HIP, "residual norms were not reported");
            }
            if (e != hipErrorNotReady) return fail(SMG_ERR_HIP, std::string("hipStreamQuery: ") + hipGetErrorString(e));
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return SMG_OK;
}

// One refinement or plain cycle, enqueued; ends with the FP64 level-0
// residual and its column norms in s->norms (and in h_norms, tagged with
// s->norm_seq).  A refinement cycle can be enqueued in two parts: kCyclePre
// (the correction's right-hand side and the level-0 pre-relaxation) writes
// FP32 buffers only, so x still holds the previous iterate until the
// kCycleAfterPre part has run.
smg_status cycle_enqueue(smg_solver_s *s, int k, int precision, hipStream_t st, int part) {
    DevLevel &D = s->lev[0];
    if (precision == SMG_FP64) {
        if (part != kCycleWhole) return fail(SMG_ERR_INVALID_ARG, "FP64 cycles are enqueued whole");
        CHK(vcycle_from<double>(s, 0, k, st));
    } else {
        // x32 is zero here: cleared at the start of the solve and by every ir_up
        if (part != kCycleAfterPre) {
            phase_mark(s, st, SMG_PHASE_OTHER);
            HIPCHK(launch_ir_down(D.r, s->norms, D.b32, D.n, k, st));
        }
        CHK(vcycle_from<float>(s, 0, k, st, part));
        if (part == kCyclePre) return SMG_OK;
        phase_mark(s, st, SMG_PHASE_OTHER);
        HIPCHK(launch_ir_up(D.x32, s->norms, D.x, D.n, k, st));
    }
    if (D.coarsest) {
        // single-level hierarchy: the residual is not smoothed-level work
        return SMG_OK;
    }
    CHK(residual_level<double>(s, 0, k, true, st));
    return SMG_OK;
}

}  // namespace smg

extern "C" smg_status smg_solve(smg_solver s, const double *d_b, double *d_x, int32_t k,
                                const smg_solve_params *p, smg_solve_info *info,
                                smg_stream stream) {
    CHK(check_level(s, 0, k));
    if (!d_b || !d_x || !p) return fail(SMG_ERR_INVALID_ARG, "null argument");
    if (p->precision != SMG_FP64 && p->precision != SMG_FP32_IR) return fail(SMG_ERR_INVALID_ARG, "bad precision");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t caller = (hipStream_t)stream;
    DevLevel &D = s->lev[0];
    if (D.coarsest) return smg_solve_single_level(s, d_b, d_x, k, p, info, caller);
    const auto t0 = std::chrono::steady_clock::now();
    // graph capture needs a capturable stream: the cycles then run on the
    // solver's own stream, ordered after and before the caller's work
    hipStream_t st = caller;
    const bool graphs = p->use_graph && s->prof_kind < 0 && !p->timed;
    if (graphs) {
        st = s->gstream;
        HIPCHK(hipEventRecord(s->ev_in, caller));
        HIPCHK(hipStreamWaitEvent(st, s->ev_in, 0));
    }
    s->ph_on = p->timed != 0;
    s->ph_cur = -1;
    s->ph_tag.clear();
    // an early return leaves no phase timing switched on
    struct PhaseOff {
        smg_solver_s *s;
        ~PhaseOff() { s->ph_on = false; s->ph_cur = -1; s->ph_tag.clear(); }
    } phase_off{s};
    phase_mark(s, st, SMG_PHASE_OTHER);
    HIPCHK(launch_fill<int>(s->flag, 0, 1, st));
    HIPCHK(launch_check_finite(d_b, (int64_t)D.n * k, s->flag, st));
    HIPCHK(launch_gather_rows(D.perm, d_b, D.b, D.n, k, st));
    HIPCHK(launch_fill<double>(D.x, 0.0, (int64_t)D.n * k, st));
    HIPCHK(launch_fill<float>(D.x32, 0.0f, (int64_t)D.n * k, st));
    // r = b for x0 = 0 (FP32_IR needs r and its max-norm in s->norms)
    int nblk = 0;
    HIPCHK(hipMemcpyAsync(D.r, D.b, (size_t)D.n * k * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_colnorm_partial(D.b, D.n, k, s->partial, &nblk, st));
    HIPCHK(launch_reduce_partial(s->partial, nblk, k, s->norms, st, s->d_hnorms));
    HIPCHK(hipMemcpyAsync(s->h_flag, s->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    CHK(fetch_norms(s, k, st));
    if (s->h_flag[0]) return fail(SMG_ERR_NONFINITE, "non-finite right-hand side");
    double bn[4], rho[4];
    for (int q = 0; q < k; ++q) {
        bn[q] = std::sqrt(s->h_norms[q]);
        rho[q] = bn[q] > 0.0 ? 1.0 : 0.0;
    }
    int cycles = 0;
    smg_status status = SMG_OK;
    hipGraphExec_t gexec = nullptr;
    if (graphs) CHK(get_cycle_graph(s, k, p->precision, st, &gexec));
    // Refinement cycles run one part ahead: the next cycle's first part (FP32
    // buffers only) is enqueued before the host waits for this cycle's
    // residual norms, so the device does not idle on the convergence test;
    // when the test ends the solve, that part's result is left unused.
    const bool ahead = !gexec && p->fixed_cycles <= 0 && p->precision == SMG_FP32_IR;
    bool pre_queued = false;
    for (;;) {
        double worst = 0.0;
        for (int q = 0; q < k; ++q) worst = std::max(worst, rho[q]);
        if (p->fixed_cycles > 0) {
            if (cycles >= p->fixed_cycles) break;
        } else if (worst <= p->rtol) {
            break;
        } else if (cycles >= p->max_cycles) {
            status = SMG_ERR_NO_CONVERGENCE;
            break;
        }
        if (gexec) {
            HIPCHK(hipGraphLaunch(gexec, st));
        } else if (ahead) {
            if (!pre_queued) CHK(cycle_enqueue(s, k, p->precision, st, kCyclePre));
            s->norm_seq += 1.0;
            s->h_norms[2 * k] = -1.0;
            CHK(cycle_enqueue(s, k, p->precision, st, kCycleAfterPre));
        } else {
            CHK(cycle_enqueue(s, k, p->precision, st));
        }
        ++cycles;
        if (p->fixed_cycles > 0 && cycles < p->fixed_cycles) continue;
        if (ahead) {
            pre_queued = cycles < p->max_cycles;
            if (pre_queued) CHK(cycle_enqueue(s, k, p->precision, st, kCyclePre));
            CHK(wait_norms(s, k, s->norm_seq, st));
        } else {
            CHK(fetch_norms(s, k, st));
        }
        for (int q = 0; q < k; ++q) {
            const double rn = std::sqrt(s->h_norms[q]);
            rho[q] = bn[q] > 0.0 ? rn / bn[q] : rn;
            if (!std::isfinite(rho[q])) status = SMG_ERR_NONFINITE;
        }
        if (status == SMG_ERR_NONFINITE) break;
    }
    HIPCHK(launch_scatter_rows(D.perm, D.x, d_x, D.n, k, st));
    if (st != caller) {
        HIPCHK(hipEventRecord(s->ev_out, st));
        HIPCHK(hipStreamWaitEvent(caller, s->ev_out, 0));
    }
    double ph[5] = {0, 0, 0, 0, 0};
    CHK(phase_sum(s, st, ph));
    HIPCHK(hipStreamSynchronize(st));
    if (s->team_level > 0) CHK(check_team(s, st));
    if (info) {
        info->cycles = cycles;
        info->k = k;
        for (int q = 0; q < 4; ++q) info->rel_res[q] = q < k ? rho[q] : 0.0;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        ph[SMG_PHASE_PREPARE] = s->ms_prepare;
        for (int q = 0; q < 5; ++q) info->ms_phase[q] = ph[q];
    }
    if (s->prof_kind >= 0) CHK(prof_collect(s));
    if (status == SMG_ERR_NO_CONVERGENCE) return fail(status, "cycle cap reached");
    if (status == SMG_ERR_NONFINITE) return fail(status, "non-finite residual");
    return SMG_OK;
}

namespace smg {

// a one-level hierarchy: the V-cycle is the direct solve
smg_status smg_solve_single_level(smg_solver_s *s, const double *d_b, double *d_x, int k,
                                  const smg_solve_params *p, smg_solve_info *info, hipStream_t st) {
    (void)p;
    const DevLevel &D = s->lev[0];
    HIPCHK((launch_coarse_solve<double, double>(D.dense_inv, D.n, d_b, d_x, k, st)));
    HIPCHK(hipStreamSynchronize(st));
    if (info) {
        info->cycles = 1;
        info->k = k;
        for (int q = 0; q < 4; ++q) info->rel_res[q] = 0.0;
        info->ms = 0.0;
        for (int q = 0; q < 5; ++q) info->ms_phase[q] = q == SMG_PHASE_PREPARE ? s->ms_prepare : 0.0;
    }
    return SMG_OK;
}

// Capture one cycle (V-cycle + FP64 residual with norms) into a hipGraph.
// No memset nodes are recorded: buffers are cleared by fill kernels.
smg_status get_cycle_graph(smg_solver_s *s, int k, int precision, hipStream_t st,
                           hipGraphExec_t *out) {
    for (auto &g : s->graphs)
        if (g.k == k && g.precision == precision && g.stream == st) { *out = g.exec; return SMG_OK; }
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    smg_status rc = cycle_enqueue(s, k, precision, st);
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc != SMG_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess) return fail(SMG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(SMG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    s->graphs.push_back({k, precision, st, exec});
    *out = exec;
    return SMG_OK;
}

}  // namespace smg

extern "C" smg_status smg_set_smoother(smg_solver s, int32_t kind, double omega) {
    if (!s) return fail(SMG_ERR_INVALID_ARG, "null solver");
    if (kind != SMG_SMOOTH_GS && kind != SMG_SMOOTH_JACOBI) return fail(SMG_ERR_INVALID_ARG, "unknown smoother");
    if (kind == SMG_SMOOTH_JACOBI && !(omega < 2.0)) return fail(SMG_ERR_INVALID_ARG, "Jacobi damping must be below 2");
    HIPCHK(hipSetDevice(s->device));
    // captured cycles hold the previous smoother's launches
    HIPCHK(hipDeviceSynchronize());
    for (auto &g : s->graphs) if (g.exec) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
    s->smoother = kind;
    if (kind == SMG_SMOOTH_JACOBI) {
        s->omega = omega > 0.0 ? omega : 0.0;
        if (s->values_set) {
            CHK(smg::jacobi_factors(s, nullptr));
            HIPCHK(hipDeviceSynchronize());
        }
    }
    return SMG_OK;
}

extern "C" smg_status smg_get_jacobi_omega(smg_solver s, int32_t level, double *omega) {
    if (!s || !omega) return fail(SMG_ERR_INVALID_ARG, "null argument");
    if (level < 0 || level >= s->nlev || s->lev[level].coarsest) return fail(SMG_ERR_INVALID_ARG, "level out of range");
    if (s->smoother != SMG_SMOOTH_JACOBI || !s->values_set) return fail(SMG_ERR_STATE, "no Jacobi factors (smoother or values not set)");
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(omega, s->d_omega + level, sizeof(double), hipMemcpyDeviceToHost));
    return SMG_OK;
}

// ------------------------------------------- V-cycle-preconditioned CG
namespace smg {

// z = B r, B one symmetric V-cycle from zero.  FP64: r in D.b, z in D.x.
// FP32: r in D.r, scaled by max |r| per column into D.b32 (the scale is
// s->norms[k + q], left there by the update's reduction), z in D.x32.  The
// iterate is zero on entry (cleared by the last direction update).
static smg_status cg_precond(smg_solver_s *s, int k, int precision, hipStream_t st) {
    DevLevel &D = s->lev[0];
    if (precision == SMG_FP64) return vcycle_from<double>(s, 0, k, st, kCycleWhole, true);
    HIPCHK(launch_ir_down(D.r, s->norms, D.b32, D.n, k, st));
    return vcycle_from<float>(s, 0, k, st, kCycleWhole, true);
}

// r.z reduced into out[0..k); then p = z + (out / rz_old) p and z cleared
static smg_status cg_direction(smg_solver_s *s, int k, int precision, double *out, const double *rz_old,
                               hipStream_t st) {
    DevLevel &D = s->lev[0];
    const bool f32 = precision != SMG_FP64;
    const double *r = f32 ? D.r : D.b;
    int nblk = 0;
    HIPCHK(launch_cg_dot(D.n, r, D.x, f32 ? D.x32 : nullptr, s->norms, k, s->partial, &nblk, st));
    HIPCHK(launch_reduce_partial(s->partial, nblk, k, out, st));
    HIPCHK(launch_cg_direction(D.n, out, rz_old, D.x, f32 ? D.x32 : nullptr, s->norms, s->cg_p, k, st));
    return SMG_OK;
}

}  // namespace smg

extern "C" smg_status smg_pcg_solve(smg_solver s, const double *d_b, double *d_x, int32_t k,
                                    const smg_solve_params *p, smg_solve_info *info, smg_stream stream) {
    CHK(check_level(s, 0, k));
    if (!d_b || !d_x || !p) return fail(SMG_ERR_INVALID_ARG, "null argument");
    if (p->precision != SMG_FP64 && p->precision != SMG_FP32_IR) return fail(SMG_ERR_INVALID_ARG, "bad precision");
    if (p->use_graph) return fail(SMG_ERR_INVALID_ARG, "graph replay is not offered for CG");
    if (s->mu_pre != s->mu_post) return fail(SMG_ERR_INVALID_ARG, "a symmetric V-cycle needs mu_pre == mu_post");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    DevLevel &D = s->lev[0];
    if (D.coarsest) return smg_solve_single_level(s, d_b, d_x, k, p, info, st);
    const auto t0 = std::chrono::steady_clock::now();
    const int prec = p->precision;
    const bool f32 = prec != SMG_FP64;
    double *r = f32 ? D.r : D.b;
    const int64_t nk = (int64_t)D.n * k;
    HIPCHK(launch_fill<int>(s->flag, 0, 1, st));
    HIPCHK(launch_check_finite(d_b, nk, s->flag, st));
    HIPCHK(launch_gather_rows(D.perm, d_b, r, D.n, k, st));
    HIPCHK(launch_fill<double>(D.x, 0.0, nk, st));
    HIPCHK(launch_fill<float>(D.x32, 0.0f, nk, st));
    HIPCHK(launch_fill<double>(s->cg_x, 0.0, nk, st));
    int nblk = 0;
    HIPCHK(launch_colnorm_partial(r, D.n, k, s->partial, &nblk, st));
    HIPCHK(launch_reduce_partial(s->partial, nblk, k, s->norms, st, s->d_hnorms, s->norm_seq));
    HIPCHK(hipMemcpyAsync(s->h_flag, s->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    CHK(fetch_norms(s, k, st));
    if (s->h_flag[0]) return fail(SMG_ERR_NONFINITE, "non-finite right-hand side");
    double bn[4], rho[4];
    for (int q = 0; q < k; ++q) {
        bn[q] = std::sqrt(s->h_norms[q]);
        rho[q] = bn[q] > 0.0 ? 1.0 : 0.0;
    }
    // first direction: z = B b, p = z, r.z into slot 0
    CHK(cg_precond(s, k, prec, st));
    CHK(cg_direction(s, k, prec, s->cg_s, nullptr, st));
    int it = 0, cur = 0;
    smg_status status = SMG_OK;
    for (;;) {
        double worst = 0.0;
        for (int q = 0; q < k; ++q) worst = std::max(worst, rho[q]);
        if (p->fixed_cycles > 0) {
            if (it >= p->fixed_cycles) break;
        } else if (worst <= p->rtol) {
            break;
        } else if (it >= p->max_cycles) {
            status = SMG_ERR_NO_CONVERGENCE;
            break;
        }
        double *rz = s->cg_s + 8 * cur, *rz_next = s->cg_s + 8 * (1 - cur), *pap = s->cg_s + 16;
        HIPCHK(launch_cg_spmv(sell_view<double>(D), D.nslices, s->cg_p, s->cg_ap, k, s->partial, &nblk, st));
        HIPCHK(launch_reduce_partial(s->partial, nblk, k, pap, st));
        s->norm_seq += 1.0;
        s->h_norms[2 * k] = -1.0;
        HIPCHK(launch_cg_update(D.n, rz, pap, s->cg_p, s->cg_ap, s->cg_x, r, k, s->partial, &nblk, st));
        HIPCHK(launch_reduce_partial(s->partial, nblk, k, s->norms, st, s->d_hnorms, s->norm_seq));
        ++it;
        const bool more = p->fixed_cycles > 0 ? it < p->fixed_cycles : it < p->max_cycles;
        // the preconditioner leaves x alone: it runs while the host tests r
        if (more) CHK(cg_precond(s, k, prec, st));
        if (p->fixed_cycles <= 0 || !more) {
            CHK(wait_norms(s, k, s->norm_seq, st));
            for (int q = 0; q < k; ++q) {
                const double rn = std::sqrt(s->h_norms[q]);
                rho[q] = bn[q] > 0.0 ? rn / bn[q] : rn;
                if (!std::isfinite(rho[q])) status = SMG_ERR_NONFINITE;
            }
            if (status == SMG_ERR_NONFINITE) break;
        }
        if (!more) continue;   // the loop head ends the solve
        if (p->fixed_cycles <= 0) {
            double w2 = 0.0;
            for (int q = 0; q < k; ++q) w2 = std::max(w2, rho[q]);
            if (w2 <= p->rtol) break;   // the queued preconditioner's result is unused
        }
        CHK(cg_direction(s, k, prec, rz_next, rz, st));
        cur = 1 - cur;
    }
    HIPCHK(launch_scatter_rows(D.perm, s->cg_x, d_x, D.n, k, st));
    HIPCHK(hipStreamSynchronize(st));
    if (info) {
        info->cycles = it;
        info->k = k;
        for (int q = 0; q < 4; ++q) info->rel_res[q] = q < k ? rho[q] : 0.0;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int q = 0; q < 5; ++q) info->ms_phase[q] = q == SMG_PHASE_PREPARE ? s->ms_prepare : 0.0;
    }
    if (status == SMG_ERR_NO_CONVERGENCE) return fail(status, "iteration cap reached");
    if (status == SMG_ERR_NONFINITE) return fail(status, "non-finite residual");
    return SMG_OK;
}

// ------------------------------------------------- adjoint helper kernels
extern "C" smg_status smg_spmv_dot(smg_solver s, const double *d_l_vals, const double *d_lambda,
                                   const double *d_u, double *h_out, smg_stream stream) {
    if (!s || !d_l_vals || !d_lambda || !d_u || !h_out) return fail(SMG_ERR_INVALID_ARG, "null argument");
    if (!s->mesh.attached) return fail(SMG_ERR_STATE, "no mesh attached (level-0 pattern on device)");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    int nblk = 0;
    HIPCHK(launch_spmv_dot(s->mesh.rowptr, s->mesh.cols, d_l_vals, d_lambda, d_u, s->lev[0].n,
                           s->partial, &nblk, st));
    HIPCHK(launch_reduce_partial(s->partial, nblk, 1, s->norms, st, s->d_hnorms));
    CHK(fetch_norms(s, 1, st));
    *h_out = s->h_norms[0];
    return SMG_OK;
}

// ------------------------------- lambda^T L u with no allocation at all
// Scratch of smg_spmv_dot_noalloc: per-block partial sums of k_spmv_dot (two
// doubles per block) and the reduced pair, in a file-scope device array.
// Each device holds its own copy until the process ends; the host reaches it
// only through the address hipGetSymbolAddress returns on that device.
constexpr size_t kNoallocScratch = size_t(1) << 17;             // doubles (1 MiB)
static __device__ __align__(256) double scratch[kNoallocScratch];
constexpr int kNoallocMaxBlocks = (int)((kNoallocScratch - 2) / 2);
static std::mutex g_scratch_mu;
static double *g_scratch[64] = {};                               // per device, set once

static smg_status noalloc_scratch(int device, double **out) {
    if (device < 0 || device >= 64) return fail(SMG_ERR_INVALID_ARG, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SMG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[device] = (double *)p;
    }
    *out = g_scratch[device];
    return SMG_OK;
}

extern "C" smg_status smg_spmv_dot_noalloc(int32_t n, const int32_t *d_rowptr, const int32_t *d_cols,
                                           const double *d_vals, const double *d_lambda, const double *d_u,
                                           double *d_out, smg_stream stream) {
    if (!d_rowptr || !d_cols || !d_vals || !d_lambda || !d_u || !d_out || n < 1)
        return fail(SMG_ERR_INVALID_ARG, "smg_spmv_dot_noalloc: null argument or empty matrix");
    if ((n + 255) / 256 > kNoallocMaxBlocks)
        return fail(SMG_ERR_INVALID_ARG, "smg_spmv_dot_noalloc: " + std::to_string(n) + " rows; at most " +
                                             std::to_string((int64_t)kNoallocMaxBlocks * 256));
    int device = 0;
    HIPCHK(hipGetDevice(&device));
    double *scr = nullptr;
    CHK(noalloc_scratch(device, &scr));
    hipStream_t st = (hipStream_t)stream;
    int nblk = 0;
    double *partial = scr, *red = scr + kNoallocScratch - 2;
    HIPCHK(launch_spmv_dot(d_rowptr, d_cols, d_vals, d_lambda, d_u, n, partial, &nblk, st));
    HIPCHK(launch_reduce_partial(partial, nblk, 1, red, st));
    HIPCHK(launch_axpby(1, 1.0, red, 0.0, red, d_out, st));   // d_out = the sum
    return SMG_OK;
}

extern "C" smg_status smg_mass_grad(smg_solver s, const double *d_lambda, const double *d_m,
                                    const double *d_u, double *d_out, smg_stream stream) {
    if (!s || !d_lambda || !d_m || !d_u || !d_out) return fail(SMG_ERR_INVALID_ARG, "null argument");
    HIPCHK(hipSetDevice(s->device));
    HIPCHK(launch_mass_grad(d_lambda, d_m, d_u, d_out, s->lev[0].n, (hipStream_t)stream));
    return SMG_OK;
}

// --------------------------------------------------------------- profiling
namespace smg {

int prof_begin(smg_solver_s *s, int kind, int level, double bytes, hipStream_t st, int64_t launches) {
    if (s->prof_kind != kind || (s->prof_level >= 0 && s->prof_level != level)) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return -1;
    while (s->prof_pool.size() < 2 * (s->prof_used + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        s->prof_pool.push_back(e);
    }
    const int idx = (int)s->prof_used++;
    s->prof_bytes_pending.push_back(bytes);
    s->prof_launches_pending.push_back(launches);
    return idx;
}

void phase_mark(smg_solver_s *s, hipStream_t st, int phase) {
    if (!s->ph_on || phase == s->ph_cur) return;
    const size_t i = s->ph_tag.size();
    if (s->ph_pool.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { s->ph_on = false; return; }
        s->ph_pool.push_back(e);
    }
    if (hipEventRecord(s->ph_pool[i], st) != hipSuccess) { s->ph_on = false; return; }
    s->ph_tag.push_back(phase);
    s->ph_cur = phase;
}

smg_status phase_sum(smg_solver_s *s, hipStream_t st, double *ms) {
    const bool was_on = s->ph_on;
    phase_mark(s, st, -1);   // closes the last interval
    s->ph_on = false;
    s->ph_cur = -1;
    if (was_on) {
        HIPCHK(hipStreamSynchronize(st));
        for (size_t i = 0; i + 1 < s->ph_tag.size(); ++i) {
            float dt = 0.0f;
            HIPCHK(hipEventElapsedTime(&dt, s->ph_pool[i], s->ph_pool[i + 1]));
            if (ms && s->ph_tag[i] >= 0 && s->ph_tag[i] < 5) ms[s->ph_tag[i]] += dt;
        }
    }
    s->ph_tag.clear();
    return SMG_OK;
}

hipEvent_t prof_ev(smg_solver_s *s, int idx, int which) {
    return idx < 0 ? nullptr : s->prof_pool[2 * idx + which];
}

smg_status prof_collect(smg_solver_s *s) {
    for (size_t i = 0; i < s->prof_used; ++i) {
        HIPCHK(hipEventSynchronize(s->prof_pool[2 * i + 1]));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, s->prof_pool[2 * i], s->prof_pool[2 * i + 1]));
        s->prof_ms += ms;
        s->prof_bytes += s->prof_bytes_pending[i];
        s->prof_launches += s->prof_launches_pending[i];
    }
    s->prof_used = 0;
    s->prof_bytes_pending.clear();
    s->prof_launches_pending.clear();
    return SMG_OK;
}

}  // namespace smg

extern "C" smg_status smg_profile_enable(smg_solver s, int32_t kind, int32_t level) {
    if (!s) return fail(SMG_ERR_INVALID_ARG, "null solver");
    HIPCHK(hipSetDevice(s->device));
    CHK(prof_collect(s));
    s->prof_group = kind >= 0 && (kind & SMG_PROF_GROUP);
    s->prof_kind = kind >= 0 ? (kind & ~SMG_PROF_GROUP) : -1;
    s->prof_level = level;
    s->prof_ms = 0.0;
    s->prof_bytes = 0.0;
    s->prof_launches = 0;
    return SMG_OK;
}

extern "C" smg_status smg_launch_floor(smg_solver s, int32_t kind, int32_t level, int32_t launches,
                                       smg_stream stream, double *us, double *us_host) {
    if (!s || !us || kind < 0 || kind > 2 || launches < 1 || launches > 4000 || level < 0 ||
        level >= s->nlev || s->lev[level].coarsest)
        return fail(SMG_ERR_INVALID_ARG, "smg_launch_floor: bad arguments");
    HIPCHK(hipSetDevice(s->device));
    hipStream_t st = (hipStream_t)stream;
    const DevLevel &D = s->lev[level];
    // the grid of the level's widest color launch
    int slices = 1;
    for (int c = 0; c < D.ncolors; ++c) slices = std::max(slices, D.color_slice[c + 1] - D.color_slice[c]);
    const int n = (int)std::min<int64_t>(std::min<int64_t>((int64_t)slices * 64, D.n), D.slots);
    if (n < 1) return fail(SMG_ERR_INVALID_ARG, "smg_launch_floor: level has no slots");
    // inputs: the level's own buffers: the first slots of its sliced column
    // array as indices (neighbours of nearby rows, the gather's own locality;
    // padding slots hold valid rows), x32 as values, r32 as output
    static_assert(sizeof(*D.cols) == sizeof(int32_t), "int32 columns");
    // The launches are queued behind a bounded sleep kernel that outlasts
    // their enqueueing, so the device runs them back to back at its own pace
    // (enqueueing one takes the host about as long as the device runs one).
    hipEvent_t ed = nullptr;
    HIPCHK(hipEventCreate(&ed));
    smg_status rc = SMG_OK;
    double dev_ms = 0.0, host_ms = 0.0;
    int iters = 2 * launches + 64;   // ~3.4 us per iteration
    for (int rep = 0; rep < 4 && rc == SMG_OK; ++rep) {   // the first repetition warms up
        if (hipEventRecord(ed, st) != hipSuccess || launch_delay(iters, st) != hipSuccess ||
            hipEventRecord(s->ev_prep0, st) != hipSuccess) { rc = SMG_ERR_HIP; break; }
        const auto t0 = std::chrono::steady_clock::now();
        for (int i = 0; i < launches && rc == SMG_OK; ++i) {
            // kind 2: the two FP32 work vectors alternate, so each launch gathers
            // what the previous one wrote
            const bool swap = kind == 2 && (i & 1);
            if (launch_floor(kind == 0 ? 0 : 1, slices, D.cols, swap ? D.r32 : D.x32, swap ? D.x32 : D.r32, n, st) !=
                hipSuccess)
                rc = SMG_ERR_HIP;
        }
        const auto t1 = std::chrono::steady_clock::now();
        if (rc != SMG_OK || hipEventRecord(s->ev_prep1, st) != hipSuccess ||
            hipEventSynchronize(s->ev_prep1) != hipSuccess) { rc = SMG_ERR_HIP; break; }
        float dm = 0.0f, delay = 0.0f;
        if (hipEventElapsedTime(&dm, s->ev_prep0, s->ev_prep1) != hipSuccess ||
            hipEventElapsedTime(&delay, ed, s->ev_prep0) != hipSuccess) { rc = SMG_ERR_HIP; break; }
        dev_ms = dm;
        host_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        if (rep == 0) continue;
        if (host_ms < 0.9 * delay) break;   // every launch was queued before the device reached it
        iters *= 2;                         // the host was not ahead: a longer hold
    }
    (void)hipEventDestroy(ed);
    if (rc != SMG_OK) return fail(rc, "smg_launch_floor: timing failed");
    // leave the work vectors as a solve leaves them (zero)
    HIPCHK(launch_fill<float>(D.x32, 0.0f, (int64_t)D.n * 4, st));
    HIPCHK(launch_fill<float>(D.r32, 0.0f, (int64_t)D.n * 4, st));
    HIPCHK(hipStreamSynchronize(st));
    *us = 1e3 * dev_ms / launches;
    if (us_host) *us_host = 1e3 * host_ms / launches;
    return SMG_OK;
}

extern "C" smg_status smg_profile_read(smg_solver s, double *total_ms, int64_t *launches,
                                       double *bytes) {
    if (!s || !total_ms || !launches || !bytes) return fail(SMG_ERR_INVALID_ARG, "null argument");
    HIPCHK(hipSetDevice(s->device));
    CHK(prof_collect(s));
    *total_ms = s->prof_ms;
    *launches = s->prof_launches;
    *bytes = s->prof_bytes;
    return SMG_OK;
}
