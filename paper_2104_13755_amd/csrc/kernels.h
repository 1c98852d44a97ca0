// Device kernels of the surface-multigrid V-cycle (gfx950) and their launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace smg {

// Sliced-ELL level matrix (off-diagonal part) + diagonal, rows color-major.
template <typename T>
struct SellView {
    int n;
    int lpr;                     // lanes per row
    const int32_t *slice_row0;   // nslices + 1 (sentinel n)
    const int32_t *slice_off;    // nslices + 1
    const int32_t *cols;
    const T *vals;
    const T *diag;
    // order in which the wavefronts of a whole-level pass (residual, CG
    // product) take the slices, so that each XCD works on one region of
    // every color (nullptr: slice order)
    const int32_t *order = nullptr;
};

struct TransferView {             // P_l (ELL-3, SoA) and R_l = P_l^T (sliced ELL, rs_lanes lanes per row)
    int n, nc, rs_lanes;
    const int32_t *pc;
    const int32_t *rs_off, *rs_idx;
    const int32_t *rs_order = nullptr;   // as SellView::order, for the restriction's slices
};

// --- relaxation / residual / transfers (K right-hand sides, 1..4) ---
// ev0/ev1 (optional): events stamped by the dispatch itself when the kernel
// starts and ends (hipExtLaunchKernelGGL), for per-launch timing.
struct ColorSpan {
    int s_begin, s_end;          // the color's slices
    int row0, row_end;           // its permuted rows
    int off0;                    // slot offset of its first slice
    int w;                       // rounds of every slice when all are equal, else 0 (slice table)
};
template <typename T>
hipError_t launch_gs_color(const SellView<T> &A, const ColorSpan &c, const T *b, T *x, int k,
                           hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// damped Jacobi sweep over `nslices` slices: xo = x + omega D^{-1} (b - A x),
// omega read from device memory (the level's factor)
template <typename T>
hipError_t launch_jacobi(const SellView<T> &A, int nslices, const T *b, const T *x, T *xo, const double *omega,
                         int k, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Dirichlet reduced system (App. B): for each unknown row r (natural index
// uidx[r]) the values of its unknown columns into uvals[uptr[r]..] in row
// order, and rhs[r] = b_i - sum over known j of A_ij x_j (k columns)
hipError_t launch_dirichlet_reduce(int nu, const int32_t *uidx, const int32_t *rowptr, const int32_t *cols,
                                   const double *vals, const uint8_t *known, const double *x, const double *b, int k,
                                   const int32_t *uptr, double *uvals, double *rhs, hipStream_t st);
// out = a x + b y over n doubles
hipError_t launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out,
                        hipStream_t st);
// first sweep from x = 0: xo = omega b / A_ii
template <typename T>
hipError_t launch_jacobi_first(int n, int k, const T *diag, const T *b, T *xo, const double *omega, hipStream_t st);
// *omega_l = 2 / (1 + lambda), lambda the Rayleigh quotient after
// kJacobiPowerSteps power steps v <- D^{-1} A v from the golden-ratio start
// vector of the natural row indices (perm: permuted -> natural); v, u are n
// scratch doubles, sums two doubles (FP64 level matrix)
constexpr int kJacobiPowerSteps = 20;
hipError_t launch_jacobi_factor(const SellView<double> &A, int n, int nslices, const int32_t *perm, double *v,
                                double *u, double *partial, double *sums, double *omega_l, hipStream_t st);
// r = b - A x over `nslices` slices; if partial != nullptr also writes
// per-block (sum r^2, max |r|) per column into partial[blk * 2k ..]; the
// block count is returned in *nblk.
template <typename T>
hipError_t launch_residual(const SellView<T> &A, int nslices, const T *b, const T *x, T *r,
                           int k, double *partial, int *nblk, hipStream_t st,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// rc = R r; xc (optional): cleared alongside (the next level's iterate)
template <typename T>
hipError_t launch_restrict(const TransferView &P, const T *rw, const T *r, T *rc, int k,
                           hipStream_t st, T *xc = nullptr);
template <typename T>
hipError_t launch_prolong_add(const TransferView &P, const T *pw, const T *e, T *x, int k,
                              hipStream_t st);

// --- reductions ---
// column sums of squares and max-abs of a dense n x k array (FP64)
hipError_t launch_colnorm_partial(const double *v, int n, int k, double *partial, int *nblk,
                                  hipStream_t st);
// out[0..k) = column sums, out[k..2k) = column maxima; the same values also go
// to host_out (device address of mapped, coherent host memory) when given,
// followed by host_out[2k] = seq once they are visible to the host.
hipError_t launch_reduce_partial(const double *partial, int nblk, int k, double *out,
                                 hipStream_t st, double *host_out = nullptr, double seq = 0.0);

// --- conjugate gradients preconditioned by a V-cycle (level 0, FP64) ---
// ap = A p; per-block partials of p . ap (sums at [blk][q]) into partial
hipError_t launch_cg_spmv(const SellView<double> &A, int nslices, const double *p, double *ap, int k,
                          double *partial, int *nblk, hipStream_t st);
// alpha = rz / pap per column (0 if pap is 0): x += alpha p, r -= alpha ap;
// partials of r . r and max |r|
hipError_t launch_cg_update(int n, const double *rz, const double *pap, const double *p, const double *ap,
                            double *x, double *r, int k, double *partial, int *nblk, hipStream_t st);
// partials of r . z; z = z64, or z32 * zscale[k + q] when z32 is given
hipError_t launch_cg_dot(int n, const double *r, const double *z64, const float *z32, const double *zscale,
                         int k, double *partial, int *nblk, hipStream_t st);
// p = z + (rz_new / rz_old) p (p = z when rz_old is null); clears z
hipError_t launch_cg_direction(int n, const double *rz_new, const double *rz_old, double *z64, float *z32,
                               const double *zscale, double *p, int k, hipStream_t st);

// --- coarsest level ---
hipError_t launch_cholesky(double *A, int n, int *flag, hipStream_t st);
// Ainv = (G G^T)^{-1} from the Cholesky factor G (W: n x n scratch)
hipError_t launch_coarse_inverse(const double *G, int n, double *W, double *Ainv, hipStream_t st);
// x = A_H^{-1} b in FP64; Tin/Tout double or float (FP32 inner cycles convert here)
template <typename Tin, typename Tout>
hipError_t launch_coarse_solve(const double *Ainv, int n, const Tin *b, Tout *x, int k,
                               hipStream_t st);

// --- single-workgroup V-cycle over the small levels ---
template <typename T>
struct TailLevel {
    int n, ncolors, lpr;
    int grp;                      // lanes cooperating on one row (1,2,4,8) in one-workgroup code
    const int32_t *color_row;     // ncolors + 1 permuted row boundaries
    const int32_t *slice_row0, *slice_off, *row_slice, *rowlen, *cols;
    const T *vals, *diag;
    T *x, *b, *r;
    const int32_t *pc;            // prolongation to the next level (SoA ELL-3)
    const T *pw;
    const int32_t *rptr, *ridx;   // restriction into the next level
    const T *rw;
    const int32_t *row_base;      // first slot of every row (slice_off + row offset in its slice * lpr)
};

// --- one-workgroup tail with every iterate in LDS ---
// Levels first..nlev-1 of a cycle in one workgroup of kTailThreads threads:
// x of every tail level and b of the coarsest live in LDS; matrices are read
// as pass records (see TailLayout in hier.h); b and r of the smoothed tail
// levels stay in global memory (b of the first level is the caller's).
constexpr int kTailThreads = 1024;
// one matrix entry of a pass record stream (column in the level's permuted numbering)
template <typename T> struct TailRec;
template <> struct alignas(8) TailRec<float> { int32_t col; float val; };
template <> struct alignas(16) TailRec<double> { int32_t col, pad; double val; };
template <typename T>
struct LdsLevel {
    int n, lg_grp;                    // rows; log2 of the lanes per row
    int pass0, npass;                 // this level's passes in the pass table
    int wave0;                        // this level's first entry in the wavefront table
    int nsum;                         // rows of all finer levels (LDS offsets)
    const TailRec<T> *rec;            // pass records
    const T *diag;
    T *b, *r;                         // n x k, permuted order
    T *x;                             // n x k; read and written for the first level only
    const int32_t *pc;                // prolongation from the next level (SoA ELL-3)
    const T *pw;
    int rk, nc;                       // restriction into the next level: ELL rk x nc
    const int32_t *ridx;
    const T *rw;
};
// passes: 4 ints per pass (row0, nrows, last-of-color << 16, first wavefront);
// waves: 2 ints per wavefront (record offset, rounds); lds_bytes from
// tail_lds_bytes().
template <typename T>
hipError_t launch_tail_lds(const LdsLevel<T> *lv, const int32_t *passes, const int32_t *waves,
                           int first, int nlev, int mu_pre, int mu_post, const double *Ainv, int k,
                           size_t lds_bytes, hipStream_t st,
                           bool post_desc = false, bool per_column = false);
// One step of the tail on level l alone (same device code and thread mapping
// as launch_tail_lds with per_column, one workgroup per right-hand side):
// relax `sweeps` sweeps of lv[l].x (desc: colors descending), the residual
// into lv[l].r, the restriction into lv[l + 1].b, the prolongation
// lv[l].x += P lv[l + 1].x, or on the coarsest level lv[l].x = Ainv lv[l].b.
// lds_bytes from tail_step_lds_bytes().
enum { kTailStepRelax = 0, kTailStepResidual = 1, kTailStepRestrict = 2, kTailStepProlong = 3,
       kTailStepCoarse = 4 };
template <typename T>
hipError_t launch_tail_step(const LdsLevel<T> *lv, const int32_t *passes, const int32_t *waves, int l, int nlev,
                            int op, int sweeps, bool desc, const double *Ainv, int k, size_t lds_bytes,
                            hipStream_t st);
inline size_t tail_step_lds_bytes(int npass, int nwave, int n, int nc, size_t value_bytes) {
    const size_t tables = ((size_t)npass * 16 + (size_t)nwave * 8 + 15) / 16 * 16;
    return tables + ((size_t)n + (size_t)nc) * value_bytes;   // one column per workgroup
}
// grant k_tail_lds<*, T> `bytes` of dynamic LDS
template <typename T>
hipError_t tail_lds_allow(size_t bytes);
// LDS bytes of a tail from level `first`: pass and wavefront tables + x of
// every tail level + b of the coarsest, rows padded to kp = (k == 3 ? 4 : k).
inline size_t tail_lds_bytes(int npass, int nwave, int64_t rows_x, int n_coarsest, int k,
                             size_t value_bytes) {
    const int kp = k == 3 ? 4 : k;
    const size_t tables = ((size_t)npass * 16 + (size_t)nwave * 8 + 15) / 16 * 16;
    return tables + ((size_t)rows_x + (size_t)n_coarsest) * kp * value_bytes;
}
// rec64[i] = {cols[i], src[i] >= 0 ? vals[src[i]] : 0}, rec32 likewise from vals32
hipError_t launch_gather_records(const int32_t *src, const int32_t *cols, int64_t n,
                                 const double *vals, const float *vals32, TailRec<double> *rec64,
                                 TailRec<float> *rec32, hipStream_t st);

// --- batched solve: one workgroup per mesh, whole FP32-in-FP64 solve ---
struct BatchMesh {
    int k, nlev, mu_pre, mu_post, max_cycles, precision;   // precision: 0 FP64, 1 FP32 + FP64 IR
    int team;                         // workgroups cooperating on this mesh (<= 64)
    int local;                        // 1: the team's workgroups sit on one XCD (same index mod 8)
    double rtol;
    TailLevel<double> l0;             // level 0 in FP64 (x, b, r, matrix)
    const TailLevel<float> *lv32;     // every level in FP32 (device array)
    const TailLevel<double> *lv64;    // every level in FP64 (device array)
    const double *Ainv;               // coarsest inverse
    const int32_t *perm0;             // level-0 color-major position -> vertex
    const double *b_user;             // n x k, caller order
    double *x_user;                   // n x k, caller order
    double *out;                      // [cycles, rel_res[k]]
};
// launch-latency probes: kind 0 an empty kernel, 1 out[t] = v[idx[t]] for
// t < n (two dependent loads and a store), grid nblk x 64 threads
hipError_t launch_floor(int kind, int nblk, const int32_t *idx, const float *v, float *out, int n, hipStream_t st);
hipError_t launch_delay(int iters, hipStream_t st);
// Alg. "V-cycle" from level `first` to the coarsest by one team of m
// workgroups (1024 threads) on one XCD meeting at L2-local barriers; lv: the
// levels as TailLevel descriptors (device array); cb: 64 unsigned of team
// control, 256-byte aligned (cleared by the launch); flag[0] becomes nonzero if a barrier wait
// timed out.  m <= 16 keeps every workgroup resident on the XCD.
template <typename T>
hipError_t launch_team_vcycle(const TailLevel<T> *lv, int first, int nlev, int mu_pre, int mu_post,
                              const double *Ainv, unsigned *cb, int *flag, int m, int k, hipStream_t st);
// team_mesh / team_rank: mesh and member index of every workgroup (mesh -1:
// an idle workgroup that exits at once); ctrs (count * kBatchCtrStride: per
// mesh a barrier counter and the XCD of an XCD-local team, 256 bytes apart)
// and aborts (count entries) are cleared by the launch;
// partials: count * 512.
constexpr int kBatchCtrStride = 64;
hipError_t launch_batch_solve(const BatchMesh *meshes, const int32_t *team_mesh,
                              const int32_t *team_rank, int nblocks_total, int threads,
                              unsigned *ctrs, int *aborts, double *partials, int count,
                              hipStream_t st);
// resident workgroups of the batched kernel per compute unit
int batch_blocks_per_cu(int threads);

// --- hierarchy values ---
hipError_t launch_scatter_values(const double *src, const int32_t *store, int64_t nnz,
                                 double *vals, double *diag, int *flag, hipStream_t st);
// T = A P and A_{l+1} = P^T T, one thread per row accumulating in its own
// LDS slots (tmax: longest T row; cmax: most local slots of a coarse row;
// either at most kGalerkinMaxSlots).  Storage of level l+1 is overwritten
// entry by entry (opos >= 0 -> vals[opos], else diag[-1 - opos]).
constexpr int kGalerkinMaxSlots = 320;
hipError_t launch_galerkin_t(int n, int tmax, const int32_t *tptr, const int32_t *plan1ptr,
                             const uint16_t *plan1, const int32_t *row_slice,
                             const int32_t *slice_row0, const int32_t *slice_off, int lpr,
                             const int32_t *rowlen, const int32_t *cols, const double *vals,
                             const double *diag, const double *pw, double *Tbuf, hipStream_t st);
hipError_t launch_galerkin_c(int nc, int cmax, const int32_t *plan2ptr, const uint16_t *plan2,
                             const int32_t *rptr, const int32_t *ridx, const double *rw,
                             const int32_t *tptr, const double *Tbuf, const int32_t *optr,
                             const int32_t *opos, double *vals, double *diag, hipStream_t st);

// --- elementwise helpers ---
template <typename T>
hipError_t launch_fill(T *p, T v, int64_t n, hipStream_t st);
hipError_t launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t st);
// dst[r*k + q] = src[perm[r]*k + q]  (gather into permuted order) and inverse,
// converting the value type on the way (double -> double / float, and back)
template <typename Ts, typename Td>
hipError_t launch_gather_rows(const int32_t *perm, const Ts *src, Td *dst, int n, int k, hipStream_t st);
template <typename Ts, typename Td>
hipError_t launch_scatter_rows(const int32_t *perm, const Ts *src, Td *dst, int n, int k, hipStream_t st);
hipError_t launch_check_finite(const double *v, int64_t n, int *flag, hipStream_t st);
// FP64 iterative-refinement glue
hipError_t launch_ir_down(const double *r64, const double *norms, float *r32, int n, int k,
                          hipStream_t st);
// x64 += s d32 (s = max|r| per column), then d32 = 0 for the next cycle
hipError_t launch_ir_up(float *d32, const double *norms, double *x64, int n, int k,
                        hipStream_t st);

// --- assembly and adjoint helpers ---
struct MeshView {
    int n;
    const int32_t *vf_ptr, *vf_face;     // vertex -> incident faces (CSR)
    const int32_t *faces;                // m x 3
    const int32_t *slot_a, *slot_b;      // per (vertex, incident face): CSR entry of the
                                         // edges (v, next corner) and (v, previous corner)
    const int32_t *edge_of_entry;        // CSR entry -> canonical edge id (-1 on the diagonal)
    const int32_t *diag_pos;             // CSR entry of (v, v)
    const int32_t *rowptr;
};
hipError_t launch_assemble(const MeshView &M, const double *V, double t, const double *mass_scale,
                           const float *edge_w, double *a_vals, double *l_vals, double *mass,
                           hipStream_t st);
hipError_t launch_spmv_dot(const int32_t *rowptr, const int32_t *cols, const double *vals,
                           const double *lam, const double *u, int n, double *partial,
                           int *nblk, hipStream_t st);
hipError_t launch_mass_grad(const double *lam, const double *m, const double *u, double *out,
                            int n, hipStream_t st);

}  // namespace smg
