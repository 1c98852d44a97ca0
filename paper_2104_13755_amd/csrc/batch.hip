// Batched solve of many independent meshes (first version: the meshes'
// solves are enqueued one after another on the caller's stream).
#include "smg.h"

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "runtime.h"

using namespace smg;

struct smg_batch_s {
    std::vector<smg_solver> solvers;
    smg_batch_opts opts{};
};

extern "C" smg_status smg_batch_create(const smg_solver *solvers, int32_t count,
                                       const smg_batch_opts *o, smg_batch *out) {
    if (!solvers || count < 1 || !out) return fail(SMG_ERR_INVALID_ARG, "smg_batch_create: bad arguments");
    auto *b = new smg_batch_s;
    b->solvers.assign(solvers, solvers + count);
    if (o) b->opts = *o;
    *out = b;
    return SMG_OK;
}

extern "C" void smg_batch_destroy(smg_batch b) { delete b; }

extern "C" smg_status smg_batch_solve(smg_batch b, const double *const *d_b, double *const *d_x,
                                      const int32_t *k, const smg_solve_params *p,
                                      smg_solve_info *infos, smg_stream stream) {
    if (!b || !d_b || !d_x || !k || !p) return fail(SMG_ERR_INVALID_ARG, "smg_batch_solve: null argument");
    smg_status worst = SMG_OK;
    for (size_t i = 0; i < b->solvers.size(); ++i) {
        smg_status st = smg_solve(b->solvers[i], d_b[i], d_x[i], k[i], p, infos ? &infos[i] : nullptr, stream);
        if (st != SMG_OK && worst == SMG_OK) worst = st;
    }
    return worst;
}

extern "C" smg_status smg_batch_autotune(smg_batch b, int32_t budget_ms, smg_stream stream) {
    (void)budget_ms;
    (void)stream;
    if (!b) return fail(SMG_ERR_INVALID_ARG, "null batch");
    return SMG_OK;
}
