// Batched solves: every mesh's whole solve in one persistent kernel (one
// workgroup per mesh), replayed from a captured hipGraph, with an autotuner
// over the launch shape.
#include "smg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <memory>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "runtime.h"

using namespace smg;

#define HIPCHK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(SMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kXcds = 8;   // accelerator complex dies: workgroup i runs on die i mod 8

struct smg_batch_s {
    std::vector<smg_solver> solvers;
    int device = 0, count = 0;
    int threads = 1024, lanes0 = 1, lanes_c = 8, team_max = 8;   // launch shape
    int cus = 0, total_blocks = 0;
    int device_teams = 0;                                  // 1: no XCD packing (device-scope barriers)
    int local = 0;                                         // the current layout packs teams per XCD
    std::vector<int32_t> team;                             // workgroups per mesh
    // 1: workgroups per mesh in proportion to level-0 entries x the last
    // solve's cycles (the estimated work), once cycle counts are known; 0: to
    // entries alone (set by the autotuner)
    int balance = 0;
    bool balanced = false;                                 // the current layout used cycle counts
    std::vector<int32_t> last_cycles;                      // per mesh, from the last solve (empty: none yet)
    int32_t *d_team_mesh = nullptr, *d_team_rank = nullptr;
    unsigned *d_ctr = nullptr;
    int *d_abort = nullptr;
    double *d_partial = nullptr;
    int *h_abort = nullptr;
    std::string cache_file;
    uint64_t key = 0;                                      // workload fingerprint for the cache
    std::vector<TailLevel<double>> h64;                    // per mesh, nlev entries each
    std::vector<TailLevel<float>> h32;
    std::vector<int> off;                                  // first descriptor of mesh i
    TailLevel<double> *d64 = nullptr;
    TailLevel<float> *d32 = nullptr;
    BatchMesh *d_mesh = nullptr;
    double *d_out = nullptr, *h_out = nullptr;
    std::vector<BatchMesh> hm;
    hipStream_t stream = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_threads = 0, graph_blocks = 0;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // last solve's inputs, for the autotuner
    std::vector<const double *> last_b;
    std::vector<double *> last_x;
    std::vector<int32_t> last_k;
    smg_solve_params last_p{};
    bool have_last = false;
    int team_capacity = 0;                                 // entries of d_team_mesh / d_team_rank
    DevMem mem;                                            // device buffers (the first solver's allocator)
    ~smg_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        mem.release_all();
        if (h_abort) (void)hipHostFree(h_abort);
        if (h_out) (void)hipHostFree(h_out);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

static void apply_shape(smg_batch_s *b) {
    for (int i = 0; i < b->count; ++i) {
        const int nlev = b->solvers[i]->nlev;
        for (int l = 0; l < nlev; ++l) {
            const int lanes = l == 0 ? b->lanes0 : b->lanes_c;
            b->h64[b->off[i] + l].grp = lanes;
            b->h32[b->off[i] + l].grp = lanes;
        }
    }
}

// Workgroups per mesh: proportional to the mesh's level-0 entries (times its
// last cycle count when balancing), between 1 and team_max, scaled down until
// every workgroup of the launch can be
// resident at once (the team barriers need co-residency).  Blocks of the
// largest teams come first.
static smg_status layout_teams(smg_batch_s *b) {
    const int per_cu = batch_blocks_per_cu(b->threads);
    if (per_cu < 1) return fail(SMG_ERR_HIP, "batched kernel cannot be resident");
    const int capacity = per_cu * b->cus;
    const bool use_cycles = b->balance && (int)b->last_cycles.size() == b->count;
    auto weight = [&](int i) {
        const double z = (double)b->solvers[i]->lev[0].nnz_nat;
        return use_cycles ? z * std::max(1, b->last_cycles[i]) : z;
    };
    double wmax = 1.0;
    for (int i = 0; i < b->count; ++i) wmax = std::max(wmax, weight(i));
    b->balanced = use_cycles;
    int tmax = b->team_max;
    for (;;) {
        int total = 0;
        b->team.assign(b->count, 1);
        for (int i = 0; i < b->count; ++i) {
            const double share = weight(i) / wmax;
            b->team[i] = std::max(1, std::min(tmax, (int)std::lround(share * tmax)));
            total += b->team[i];
        }
        if (total <= capacity || tmax == 1) { b->total_blocks = total; break; }
        --tmax;
    }
    if (b->total_blocks > capacity) return fail(SMG_ERR_INVALID_ARG, "batch too large to be resident at once");
    if (b->total_blocks > b->team_capacity) return fail(SMG_ERR_INVALID_ARG, "batch team table too small");
    std::vector<int32_t> order(b->count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        if (b->team[a] != b->team[c]) return b->team[a] > b->team[c];
        return b->solvers[a]->lev[0].nnz_nat > b->solvers[c]->lev[0].nnz_nat;
    });
    std::vector<int32_t> tm, tr;
    // Whole teams onto the XCDs: workgroups are dispatched to the 8 XCDs
    // round robin, so workgroups x, x + 8, ... share one XCD; each team goes
    // (largest first) to the least-loaded of these 8 classes that still has
    // room for it, and its barriers then stay in that XCD's L2.  Slots left
    // over are idle workgroups (mesh -1).
    b->local = 0;
    if (!b->device_teams && b->cus % kXcds == 0) {
        const int per_xcd = capacity / kXcds;
        std::vector<std::vector<int>> bins(kXcds);
        std::vector<int> load(kXcds, 0);
        bool fits = true;
        for (int i : order) {
            int best = -1;
            for (int x = 0; x < kXcds; ++x)
                if (load[x] + b->team[i] <= per_xcd && (best < 0 || load[x] < load[best])) best = x;
            if (best < 0) { fits = false; break; }
            bins[best].push_back(i);
            load[best] += b->team[i];
        }
        const int rows = *std::max_element(load.begin(), load.end());
        if (fits && kXcds * rows <= b->team_capacity) {
            tm.assign((size_t)kXcds * rows, -1);
            tr.assign((size_t)kXcds * rows, 0);
            for (int x = 0; x < kXcds; ++x) {
                int j = 0;
                for (int i : bins[x])
                    for (int r = 0; r < b->team[i]; ++r, ++j) {
                        tm[(size_t)kXcds * j + x] = i;
                        tr[(size_t)kXcds * j + x] = r;
                    }
            }
            b->local = 1;
            b->total_blocks = kXcds * rows;
        }
    }
    if (!b->local)
        for (int i : order)
            for (int r = 0; r < b->team[i]; ++r) { tm.push_back(i); tr.push_back(r); }
    HIPCHK(hipMemcpy(b->d_team_mesh, tm.data(), tm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_team_rank, tr.data(), tr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return SMG_OK;
}

static smg_status upload_descriptors(smg_batch_s *b) {
    smg_status st = layout_teams(b);
    if (st) return st;
    apply_shape(b);
    HIPCHK(hipMemcpy(b->d64, b->h64.data(), b->h64.size() * sizeof(TailLevel<double>), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d32, b->h32.data(), b->h32.size() * sizeof(TailLevel<float>), hipMemcpyHostToDevice));
    return SMG_OK;
}

static bool read_cache(smg_batch_s *b) {
    if (b->cache_file.empty()) return false;
    FILE *f = std::fopen(b->cache_file.c_str(), "r");
    if (!f) return false;
    bool found = false;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long key;
        int t, l0, lc, tmx, bal = 0;
        const int got = std::sscanf(line, "%llx %d %d %d %d %d", &key, &t, &l0, &lc, &tmx, &bal);
        if (got >= 5 && key == b->key) {
            b->threads = t; b->lanes0 = l0; b->lanes_c = lc; b->team_max = tmx; b->balance = bal;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void write_cache(smg_batch_s *b) {
    if (b->cache_file.empty()) return;
    FILE *f = std::fopen(b->cache_file.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%llx %d %d %d %d %d\n", (unsigned long long)b->key, b->threads, b->lanes0, b->lanes_c,
                 b->team_max, b->balance);
    std::fclose(f);
}

extern "C" smg_status smg_batch_create(const smg_solver *solvers, int32_t count,
                                       const smg_batch_opts *o, smg_batch *out) {
    if (!solvers || count < 1 || !out) return fail(SMG_ERR_INVALID_ARG, "smg_batch_create: bad arguments");
    auto b = std::make_unique<smg_batch_s>();
    b->solvers.assign(solvers, solvers + count);
    b->count = count;
    b->device = solvers[0]->device;
    uint64_t key = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
    for (int i = 0; i < count; ++i) {
        smg_solver s = solvers[i];
        if (!s) return fail(SMG_ERR_INVALID_ARG, "null solver in batch");
        if (s->device != b->device) return fail(SMG_ERR_INVALID_ARG, "batched solvers must share a device");
        if (s->nlev < 2) return fail(SMG_ERR_INVALID_ARG, "batched solvers need at least two levels");
        if (s->smoother != SMG_SMOOTH_GS) return fail(SMG_ERR_INVALID_ARG, "batched solvers relax with Gauss-Seidel");
        b->off.push_back((int)b->h64.size());
        for (int l = 0; l < s->nlev; ++l) {
            const DevLevel &D = s->lev[l];
            b->h64.push_back({D.n, D.ncolors, D.lpr, D.lpr, D.color_row, D.slice_row0, D.slice_off,
                              D.row_slice, D.rowlen, D.cols, D.vals, D.diag, D.x, D.b, D.r, D.pc, D.pw,
                              D.rptr, D.ridx, D.rw, D.row_base});
            b->h32.push_back({D.n, D.ncolors, D.lpr, D.lpr, D.color_row, D.slice_row0, D.slice_off,
                              D.row_slice, D.rowlen, D.cols, D.vals32, D.diag32, D.x32, D.b32, D.r32,
                              D.pc, D.pw32, D.rptr, D.ridx, D.rw32, D.row_base});
            mix((uint64_t)D.n);
            mix((uint64_t)D.nnz_nat);
        }
    }
    b->key = key;
    if (o && o->cache_file) b->cache_file = o->cache_file;
    read_cache(b.get());
    if (o && o->threads) b->threads = o->threads;
    if (o && o->lanes_level0) b->lanes0 = o->lanes_level0;
    if (o && o->lanes_coarse) b->lanes_c = o->lanes_coarse;
    if (o && o->team_max) b->team_max = o->team_max;
    b->device_teams = o ? (o->device_teams != 0) : 0;
    if (o && o->balance) b->balance = 1;
    if (b->team_max < 1 || b->team_max > 64) return fail(SMG_ERR_INVALID_ARG, "team_max must be 1..64");
    if (b->threads != 256 && b->threads != 512 && b->threads != 1024) return fail(SMG_ERR_INVALID_ARG, "threads must be 256, 512 or 1024");
    if (b->lanes0 != 1 && b->lanes0 != 2) return fail(SMG_ERR_INVALID_ARG, "lanes_level0 must be 1 or 2");
    if (b->lanes_c != 1 && b->lanes_c != 2 && b->lanes_c != 4 && b->lanes_c != 8) return fail(SMG_ERR_INVALID_ARG, "lanes_coarse must be 1, 2, 4 or 8");
    HIPCHK(hipSetDevice(b->device));
    {
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, b->device));
        b->cus = prop.multiProcessorCount;
    }
    // every device buffer now, from the first solver's allocator; the team
    // tables hold the most workgroups any launch shape can keep resident
    b->mem.ctx = solvers[0]->owned.ctx;
    for (int t : {256, 512, 1024}) b->team_capacity = std::max(b->team_capacity, batch_blocks_per_cu(t) * b->cus);
    b->team_capacity = std::max(b->team_capacity, 1);
    auto take = [&](auto **p, size_t bytes) {
        *p = (std::remove_reference_t<decltype(**p)> *)b->mem.take(std::max<size_t>(bytes, 1));
        return *p != nullptr;
    };
    if (!take(&b->d64, b->h64.size() * sizeof(TailLevel<double>)) ||
        !take(&b->d32, b->h32.size() * sizeof(TailLevel<float>)) || !take(&b->d_mesh, count * sizeof(BatchMesh)) ||
        !take(&b->d_out, count * 8 * sizeof(double)) || !take(&b->d_ctr, (size_t)count * kBatchCtrStride * sizeof(unsigned)) ||
        !take(&b->d_abort, count * sizeof(int)) || !take(&b->d_partial, (size_t)count * 8 * 64 * sizeof(double)) ||
        !take(&b->d_team_mesh, (size_t)b->team_capacity * sizeof(int32_t)) ||
        !take(&b->d_team_rank, (size_t)b->team_capacity * sizeof(int32_t)))
        return fail(SMG_ERR_OOM, "smg_batch_create: device allocation failed");
    HIPCHK(hipHostMalloc((void **)&b->h_abort, count * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&b->h_out, count * 8 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    smg_status st = upload_descriptors(b.get());
    if (st) return st;
    b->hm.resize(count);
    *out = b.release();
    return SMG_OK;
}

extern "C" void smg_batch_destroy(smg_batch b) {
    if (b) (void)hipSetDevice(b->device);
    delete b;
}

// enqueue one batched solve on b->stream (graph on the first call per shape)
static smg_status batch_enqueue(smg_batch_s *b) {
    if (b->exec && (b->graph_threads != b->threads || b->graph_blocks != b->total_blocks)) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (!b->exec) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_batch_solve(b->d_mesh, b->d_team_mesh, b->d_team_rank, b->total_blocks,
                                          b->threads, b->d_ctr, b->d_abort, b->d_partial, b->count,
                                          b->stream);
        hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(SMG_ERR_HIP, std::string("batch graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(SMG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        b->graph_threads = b->threads;
        b->graph_blocks = b->total_blocks;
    }
    HIPCHK(hipGraphLaunch(b->exec, b->stream));
    return SMG_OK;
}

extern "C" smg_status smg_batch_solve(smg_batch b, const double *const *d_b, double *const *d_x,
                                      const int32_t *k, const smg_solve_params *p,
                                      smg_solve_info *infos, smg_stream stream) {
    if (!b || !d_b || !d_x || !k || !p) return fail(SMG_ERR_INVALID_ARG, "smg_batch_solve: null argument");
    if (p->precision != SMG_FP64 && p->precision != SMG_FP32_IR) return fail(SMG_ERR_INVALID_ARG, "bad precision");
    HIPCHK(hipSetDevice(b->device));
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < b->count; ++i) {
        smg_solver s = b->solvers[i];
        if (!s->values_set) return fail(SMG_ERR_STATE, "batch member without values");
        if (k[i] < 1 || k[i] > 4 || !d_b[i] || !d_x[i]) return fail(SMG_ERR_INVALID_ARG, "bad right-hand side");
        BatchMesh &M = b->hm[i];
        M.k = k[i];
        M.nlev = s->nlev;
        M.mu_pre = s->mu_pre;
        M.mu_post = s->mu_post;
        M.max_cycles = p->max_cycles;
        M.precision = p->precision == SMG_FP64 ? 0 : 1;
        M.rtol = p->rtol;
        M.l0 = b->h64[b->off[i]];
        M.l0.grp = b->lanes0;
        M.lv32 = b->d32 + b->off[i];
        M.lv64 = b->d64 + b->off[i];
        M.Ainv = s->lev[s->nlev - 1].dense_inv;
        M.perm0 = s->lev[0].perm;
        M.b_user = d_b[i];
        M.x_user = d_x[i];
        M.out = b->d_out + 8 * i;
        M.team = b->team[i];
        M.local = b->local;
    }
    b->last_b.assign(d_b, d_b + b->count);
    b->last_x.assign(d_x, d_x + b->count);
    b->last_k.assign(k, k + b->count);
    b->last_p = *p;
    b->have_last = true;
    hipStream_t caller = (hipStream_t)stream;
    HIPCHK(hipEventRecord(b->ev_in, caller));
    HIPCHK(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    HIPCHK(hipMemcpyAsync(b->d_mesh, b->hm.data(), b->count * sizeof(BatchMesh), hipMemcpyHostToDevice, b->stream));
    smg_status st = batch_enqueue(b);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(b->h_out, b->d_out, b->count * 8 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(b->h_abort, b->d_abort, b->count * sizeof(int), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipEventRecord(b->ev_out, b->stream));
    HIPCHK(hipStreamWaitEvent(caller, b->ev_out, 0));
    HIPCHK(hipStreamSynchronize(b->stream));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    smg_status worst = SMG_OK;
    for (int i = 0; i < b->count; ++i)
        if (b->h_abort[i])
            return fail(SMG_ERR_HIP, b->h_abort[i] == 2
                                         ? "batched solve: a workgroup of an XCD-local team ran on another XCD"
                                         : "batched solve: a team barrier timed out (workgroups not co-resident?)");
    b->last_cycles.resize(b->count);
    for (int i = 0; i < b->count; ++i) {
        const double *o = b->h_out + 8 * i;
        b->last_cycles[i] = (int32_t)o[0];
        bool conv = true, finite = true;
        for (int q = 0; q < k[i]; ++q) {
            if (!std::isfinite(o[1 + q])) finite = false;
            else if (o[1 + q] > p->rtol) conv = false;
        }
        if (!finite) worst = SMG_ERR_NONFINITE;
        else if (!conv && worst == SMG_OK) worst = SMG_ERR_NO_CONVERGENCE;
        if (infos) {
            infos[i].cycles = (int32_t)o[0];
            infos[i].k = k[i];
            for (int q = 0; q < 4; ++q) infos[i].rel_res[q] = q < k[i] ? o[1 + q] : 0.0;
            infos[i].ms = ms;
            for (int q = 0; q < 5; ++q) infos[i].ms_phase[q] = q == SMG_PHASE_PREPARE ? b->solvers[i]->ms_prepare : 0.0;
        }
    }
    // a balanced shape (read from the cache) needs cycle counts: lay the teams
    // out again for the next solve now that they are known
    if (b->balance && !b->balanced) {
        const smg_status st2 = upload_descriptors(b);
        if (st2) return st2;
    }
    if (worst == SMG_ERR_NONFINITE) return fail(worst, "non-finite residual in a batch member");
    if (worst == SMG_ERR_NO_CONVERGENCE) return fail(worst, "a batch member hit the cycle cap");
    return SMG_OK;
}

extern "C" smg_status smg_batch_shape(smg_batch b, int32_t *shape5) {
    if (!b || !shape5) return fail(SMG_ERR_INVALID_ARG, "null argument");
    shape5[0] = b->threads;
    shape5[1] = b->lanes0;
    shape5[2] = b->lanes_c;
    shape5[3] = b->team_max;
    shape5[4] = b->balance;
    return SMG_OK;
}

extern "C" smg_status smg_batch_autotune(smg_batch b, int32_t budget_ms, smg_stream stream) {
    if (!b) return fail(SMG_ERR_INVALID_ARG, "null batch");
    if (!b->have_last) return fail(SMG_ERR_STATE, "autotune needs a previous smg_batch_solve");
    HIPCHK(hipSetDevice(b->device));
    struct Shape { int t, l0, lc, tm, bal; };
    std::vector<Shape> cands;
    // each shape with teams by entries and, once cycle counts are known, by work
    const bool cyc = (int)b->last_cycles.size() == b->count;
    // (most promising first: the search stops at the budget)
    for (int tm : {32, 16, 8, 64, 4, 2})
        for (int bal : {1, 0})
            for (int t : {1024, 512, 256})
                for (int lc : {4, 8})
                    for (int l0 : {1, 2})
                        if (bal == 0 || cyc) cands.push_back({t, l0, lc, tm, bal});
    const Shape orig{b->threads, b->lanes0, b->lanes_c, b->team_max, b->balance};
    Shape bestS = orig;
    double best = 1e300;
    const auto start = std::chrono::steady_clock::now();
    for (const Shape &c : cands) {
        const double spent = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - start).count();
        if (spent > budget_ms && best < 1e300) break;
        b->threads = c.t;
        b->lanes0 = c.l0;
        b->lanes_c = c.lc;
        b->team_max = c.tm;
        b->balance = c.bal;
        smg_status st = upload_descriptors(b);
        if (st) return st;
        double tmin = 1e300;
        bool ok = true;
        for (int rep = 0; rep < 2 && ok; ++rep) {
            const auto t0 = std::chrono::steady_clock::now();
            st = smg_batch_solve(b, b->last_b.data(), b->last_x.data(), b->last_k.data(), &b->last_p, nullptr, stream);
            // a shape whose solve does not converge is no candidate, however fast
            if (st == SMG_ERR_NO_CONVERGENCE || st == SMG_ERR_NONFINITE) ok = false;
            else if (st != SMG_OK) return st;
            tmin = std::min(tmin, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        if (ok && tmin < best) { best = tmin; bestS = c; }
    }
    b->threads = bestS.t;
    b->lanes0 = bestS.l0;
    b->lanes_c = bestS.lc;
    b->team_max = bestS.tm;
    b->balance = bestS.bal;
    smg_status st = upload_descriptors(b);
    if (st) return st;
    // the caller's x again from a solve in the chosen shape
    st = smg_batch_solve(b, b->last_b.data(), b->last_x.data(), b->last_k.data(), &b->last_p, nullptr, stream);
    if (st) return st;
    write_cache(b);
    return SMG_OK;
}
