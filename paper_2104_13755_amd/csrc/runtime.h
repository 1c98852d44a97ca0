// Device-side state of a solver (private to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "kernels.h"
#include "smg.h"

struct smg_ctx_s {
    int device = 0;
    smg_alloc_fn alloc = nullptr;
    smg_free_fn free = nullptr;
    void *user = nullptr;
};

namespace smg {

// Device buffers owned by a solver or a batch: taken from the context's
// allocator (hipMalloc when it has none) and all returned on destruction.
struct DevMem {
    smg_ctx_s ctx;
    std::vector<std::pair<void *, size_t>> blocks;
    void *take(size_t bytes) {
        void *p = nullptr;
        if (ctx.alloc) {
            p = ctx.alloc(bytes, ctx.user);
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            p = nullptr;
        }
        if (p) blocks.push_back({p, bytes});
        return p;
    }
    void release_all() {
        for (auto &b : blocks) {
            if (ctx.free) ctx.free(b.first, b.second, ctx.user);
            else (void)hipFree(b.first);
        }
        blocks.clear();
    }
};

struct DevLevel {
    int n = 0, ncolors = 0, nslices = 0, lpr = 1;
    int32_t *color_row = nullptr;                 // device, ncolors + 1
    std::vector<int64_t> color_rows, color_nnz;   // per color: rows, off-diagonal entries
    int64_t offdiag_nnz = 0;
    bool coarsest = false;
    int64_t slots = 0, nnz_nat = 0;
    std::vector<int32_t> color_slice;      // host copy of slice boundaries per color
    std::vector<int32_t> color_row_h;      // host copy of row boundaries per color
    std::vector<int32_t> color_w, color_off;  // per color: uniform rounds (0: none), first slot
    std::vector<int32_t> pat_ptr, pat_idx; // natural CSR pattern (host)
    std::vector<int32_t> store_h;          // natural entry -> storage (host)
    std::vector<int32_t> color_h;          // natural color ids (host)
    int32_t *perm = nullptr, *store = nullptr;
    // sliced ELL (smoothed levels)
    int32_t *slice_row0 = nullptr, *slice_off = nullptr, *cols = nullptr, *rowlen = nullptr,
            *row_slice = nullptr, *row_base = nullptr;
    double *vals = nullptr, *diag = nullptr;
    float *vals32 = nullptr, *diag32 = nullptr;
    // coarsest: A_H (dense_a), its Cholesky factor (dense), G^{-1} (dense_w)
    // and A_H^{-1} (dense_inv), all column-major
    double *dense = nullptr, *dense_a = nullptr, *dense_w = nullptr, *dense_inv = nullptr;
    // transfers to the next level and the Galerkin plan
    int32_t *pc = nullptr, *rptr = nullptr, *ridx = nullptr, *rs_off = nullptr, *rs_idx = nullptr;
    // slice orders of the whole-level passes on large levels (nullptr: slice order)
    int32_t *slice_order = nullptr, *rs_order = nullptr;
    double *rs_w = nullptr;
    float *rs_w32 = nullptr;
    int rs_lanes = 4;
    double *pw = nullptr, *rw = nullptr;
    float *pw32 = nullptr, *rw32 = nullptr;
    int32_t *tptr = nullptr, *plan1ptr = nullptr, *plan2ptr = nullptr, *optr = nullptr, *opos = nullptr;
    uint16_t *plan1 = nullptr, *plan2 = nullptr;
    int tmax = 0, cmax = 0;           // longest T row, most local slots of a coarse row
    // LDS-tail records (levels small enough for the one-workgroup tail)
    bool tl = false;
    int tl_lg = 0, tl_npass = 0, tl_pass0 = 0, tl_nwave = 0, tl_wave0 = 0, tl_rk = 0;
    int64_t tl_nrec = 0;
    int32_t *tl_src = nullptr, *tl_cols = nullptr, *tl_ridx = nullptr;
    smg::TailRec<double> *tl_rec = nullptr;
    smg::TailRec<float> *tl_rec32 = nullptr;
    double *tl_rw = nullptr;
    float *tl_rw32 = nullptr;
    // work vectors, n x 4 (permuted order)
    double *x = nullptr, *b = nullptr, *r = nullptr;
    float *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;
    double *xj = nullptr;                  // Jacobi's second iterate (allocated when selected)
    double *sq_vals = nullptr, *sq_diag = nullptr;   // split Galerkin: levels of Q (dense on the coarsest)
    double *sm_vals = nullptr, *sm_diag = nullptr;   // and of M
    float *xj32 = nullptr;
};

struct MeshDev {
    bool attached = false;
    int n = 0, m = 0, nedges = 0;
    int32_t *faces = nullptr, *vf_ptr = nullptr, *vf_face = nullptr, *slot_a = nullptr,
            *slot_b = nullptr, *eoe = nullptr, *diag_pos = nullptr, *rowptr = nullptr,
            *cols = nullptr;
};

struct CycleGraph {
    int k, precision;
    hipStream_t stream;
    hipGraphExec_t exec;
};

smg_status fail(smg_status st, const std::string &msg);

}  // namespace smg

struct smg_solver_s {
    int device = 0, nlev = 0, mu_pre = 2, mu_post = 2;
    int smoother = 0;              // SMG_SMOOTH_GS or SMG_SMOOTH_JACOBI
    double omega = 0.0;            // Jacobi factor for every level; <= 0: per level from lambda estimates
    double *d_omega = nullptr;     // per level factor (device), set by jacobi_factors
    bool split_ready = false, split_ready_alloc = false;   // split Galerkin levels kept
    double *jac_v = nullptr, *jac_u = nullptr, *jac_sums = nullptr;   // power-step scratch
    // first level run by the one-workgroup LDS tail, per precision (0 FP64,
    // 1 FP32) and right-hand-side count k (index k); nlev - 1 = no tail
    int tail_first[2][5] = {};
    smg::LdsLevel<double> *lds64 = nullptr;   // device descriptors, one per level
    smg::LdsLevel<float> *lds32 = nullptr;
    int32_t *tpass = nullptr;                  // pass table of all tail levels
    int32_t *twave = nullptr;                  // wavefront table of all tail levels
    std::vector<size_t> tail_lds[2][5];        // LDS bytes of a tail from level l
    // one-XCD team V-cycle from team_level (0: off), team_size workgroups,
    // levels as TailLevel descriptors, its barrier counter
    int team_level = 0, team_size = 16;
    smg::TailLevel<double> *team64 = nullptr;
    smg::TailLevel<float> *team32 = nullptr;
    unsigned *team_ctr = nullptr;
    bool values_set = false;
    std::vector<smg::DevLevel> lev;
    smg::MeshDev mesh;
    double *tbuf = nullptr;        // Galerkin T = A P scratch
    double *partial = nullptr;     // per-block reduction partials
    int64_t npartial = 0;
    double *norms = nullptr;       // reduced (sum r^2, max |r|) per column
    int *flag = nullptr;           // [0] non-finite, [1] not SPD
    double *h_norms = nullptr;     // pinned, coherent: written by the norm reduction itself
    double *d_hnorms = nullptr;    // device address of h_norms
    double norm_seq = 0.0;         // tag the next norm reduction writes after its norms
    // preconditioned CG (allocated at its first use): x, p, A p on level 0
    // (n x 4 each) and column scalars: r.z at [0] / [8] (alternating), p.Ap at [16]
    double *cg_x = nullptr, *cg_p = nullptr, *cg_ap = nullptr, *cg_s = nullptr;
    int *h_flag = nullptr;         // pinned
    smg::DevMem owned;               // every device buffer of the solver
    std::vector<smg::CycleGraph> graphs;
    hipStream_t gstream = nullptr;  // capture/replay stream for cycle graphs
    // per-launch profiling
    int prof_kind = -1, prof_level = -1;
    std::vector<hipEvent_t> prof_pool;
    std::vector<double> prof_bytes_pending;      // bytes of each recorded pair
    std::vector<int64_t> prof_launches_pending;  // launches each recorded pair spans
    bool prof_group = false;                     // one pair per relaxation call, not per launch
    size_t prof_used = 0;
    double prof_ms = 0.0, prof_bytes = 0.0;
    int64_t prof_launches = 0;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // phase timing of a solve (smg_solve_params.timed): an event at every
    // change of phase, tagged with the phase it starts
    bool ph_on = false;
    int ph_cur = -1;
    std::vector<hipEvent_t> ph_pool;
    std::vector<int> ph_tag;
    double ms_prepare = 0.0;                     // device time of the last value refresh
    hipEvent_t ev_prep0 = nullptr, ev_prep1 = nullptr;
    ~smg_solver_s();
};

namespace smg {
smg_status refresh_values(smg_solver_s *s, const double *d_a0_vals, hipStream_t st);
smg_status jacobi_factors(smg_solver_s *s, hipStream_t st);
smg_status galerkin_values(smg_solver_s *s, const double *d_a0_vals, hipStream_t st);
smg_status finish_values(smg_solver_s *s, hipStream_t st);
// parts of one cycle: all of it, only the first level's pre-relaxation, or
// everything after that pre-relaxation
enum CyclePart { kCycleWhole = 0, kCyclePre = 1, kCycleAfterPre = 2 };
template <typename T>
smg_status vcycle_from(smg_solver_s *s, int l, int k, hipStream_t st, int part = kCycleWhole,
                       bool sym = false);
template <typename T>
smg_status residual_level(smg_solver_s *s, int l, int k, bool norms, hipStream_t st);
smg_status cycle_enqueue(smg_solver_s *s, int k, int precision, hipStream_t st, int part = kCycleWhole);
smg_status get_cycle_graph(smg_solver_s *s, int k, int precision, hipStream_t st,
                           hipGraphExec_t *out);
// profiling helpers: begin returns the event pair index or -1; prof_ev gives
// the start (0) / stop (1) event to hand to the launch (null when not profiled)
int prof_begin(smg_solver_s *s, int kind, int level, double bytes, hipStream_t st, int64_t launches = 1);
hipEvent_t prof_ev(smg_solver_s *s, int idx, int which);
smg_status prof_collect(smg_solver_s *s);
// phase timing: phase_mark records an event on st when the phase changes
// (timed solves only); phase_sum closes the record and adds the intervals
// between the events into ms[SMG_PHASE_*]
void phase_mark(smg_solver_s *s, hipStream_t st, int phase);
smg_status phase_sum(smg_solver_s *s, hipStream_t st, double *ms);
smg_status smg_solve_single_level(smg_solver_s *s, const double *d_b, double *d_x, int k,
                                  const smg_solve_params *p, smg_solve_info *info,
                                  hipStream_t st);
}  // namespace smg
