/*
 * smg.h -- C ABI of the MI355X surface-multigrid library (libsmg.so).
 *
 * Solves A x = b on a triangle mesh with the Galerkin multigrid V-cycle of
 * Liu, Zhang, Ben-Chen, Jacobson, "Surface Multigrid via Intrinsic
 * Prolongation" (ACM TOG 40(4), 2021): Alg. "Galerkin Surface Multigrid
 * Solver" (outer loop) and Alg. "V-cycle" (pre-relaxation, restriction P^T r,
 * coarse-grid correction with A_{l+1} = P_l^T A_l P_l (Eq. gca), prolongation
 * P c, post-relaxation, direct coarsest solve), with the intrinsic
 * prolongations P_l of Sec. 4 (successive self-parameterization, at most three
 * barycentric weights per row, Sec. 4.5) and multicolor Gauss-Seidel
 * relaxation (App. A, Alg. "Graph Coloring").
 *
 * Conventions for every entry point:
 *  - Returns SMG_OK (0) or a negative smg_status; nothing is thrown across the
 *    ABI.  smg_last_error() gives a thread-local message for the last failure.
 *  - Indices are 0-based int32.  Vectors with k right-hand sides are n x k,
 *    row-major (the k values of one vertex are adjacent), 1 <= k <= 4.
 *  - Pointers named d_* are device pointers on the solver's device; h_* and
 *    unprefixed arrays are host pointers.  The caller owns every pointer it
 *    passes; the library never frees them and keeps none after returning,
 *    except where stated.  The library owns its internal device buffers: it
 *    takes them in smg_solver_create / smg_batch_create from the allocator of
 *    the solver's context (hipMalloc by default, or the caller's functions,
 *    see smg_ctx_create) and returns them in the matching destroy call.  Of
 *    the other entry points only smg_solver_attach_mesh (the mesh arrays)
 *    and the first smg_split_prepare (two copies of the level values) take
 *    more; solves, cycles, steps and value refreshes take none.
 *  - stream is a hipStream_t (NULL = default stream).  Work is enqueued on it;
 *    calls that return values to the host synchronize that stream.
 *  - Vectors of level l are in that level's natural vertex numbering (level 0:
 *    the caller's vertex order; level l > 0: the coarse numbering of the
 *    hierarchy).  The library's internal color-major permutation is never
 *    visible at the ABI.
 */
#ifndef SMG_H
#define SMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t smg_status;
enum {
    SMG_OK = 0,
    SMG_ERR_INVALID_ARG = -1,    /* bad size, null pointer, out-of-range index */
    SMG_ERR_OOM = -2,            /* device or host allocation failed */
    SMG_ERR_HIP = -3,            /* a HIP runtime call failed */
    SMG_ERR_NOT_SPD = -4,        /* coarsest Cholesky met a pivot <= 0 */
    SMG_ERR_NO_CONVERGENCE = -5, /* cycle cap reached; x holds the last iterate */
    SMG_ERR_NONFINITE = -6,      /* NaN/Inf in b or in the matrix values */
    SMG_ERR_STATE = -7,          /* call out of order (e.g. solve before set_values) */
    SMG_ERR_PRECOMPUTE = -8      /* hierarchy construction failed */
};

enum { SMG_FP64 = 0, SMG_FP32_IR = 1 };   /* precision of smg_solve / smg_vcycle */
enum { SMG_SMOOTH_GS = 0, SMG_SMOOTH_JACOBI = 1 };   /* relaxation, smg_set_smoother */

typedef struct smg_ctx_s *smg_ctx;         /* device + allocator of solvers */
typedef struct smg_hier_s *smg_hier;       /* host-side hierarchy (prolongations) */
typedef struct smg_solver_s *smg_solver;   /* device-resident solver of one mesh */
typedef struct smg_batch_s *smg_batch;     /* many solvers in one launch schedule */
typedef void *smg_stream;                  /* hipStream_t */

/* ------------------------------------------------------------------------ */
/* Host precompute (CPU, geometry only; paper Alg. "Galerkin Surface Multigrid
 * Solver", second line, and Sec. 5 "Successive Self-Parameterization").     */

typedef struct {
    int32_t n_levels;      /* total levels incl. the finest; 0 = rule below      */
    int32_t min_coarse;    /* rule: decimate while floor(n/4 + 1/2) >= min_coarse
                              (Sec. 5 defaults: ratio 0.25, coarsest >= 500)     */
    int32_t collapses;     /* which edges may collapse: SMG_COLLAPSE_ALL (the
                              method); SMG_COLLAPSE_INTERIOR (both endpoints
                              interior) and SMG_COLLAPSE_STRAIGHT (those plus
                              boundary edges whose previous, own and next
                              boundary vertices lie on one line; no collapse
                              with exactly one boundary endpoint) restrict it
                              to collapses whose flattening of a flat disc is
                              the planar embedding (used by tests)             */
} smg_pre_opts;

enum { SMG_COLLAPSE_ALL = 0, SMG_COLLAPSE_INTERIOR = 1, SMG_COLLAPSE_STRAIGHT = 2 };

/* Build P_1..P_H by mid-point edge collapse with joint LSCM flattening
 * (Sec. 4.1-4.4) and the barycentric query (App. C, Fig. baryQuery).
 * V: n x 3 double, F: m x 3 int32, a consistently oriented manifold mesh with
 * or without boundary.  opts may be NULL (n_levels 0, min_coarse 500).
 * *out is owned by the caller and released with smg_hier_free.
 * Errors: INVALID_ARG (bad sizes or indices, a face repeating a vertex, a
 * non-finite coordinate), PRECOMPUTE (non-manifold input). */
smg_status smg_pre_build(const double *V, int32_t n, const int32_t *F, int32_t m,
                         const smg_pre_opts *opts, smg_hier *out);

/* Wrap externally computed prolongations: level l has sizes[l] vertices,
 * P_l is sizes[l] x 3 in ELL form (p_cols[l], p_w[l]); a slot with weight 0
 * or column < 0 is unused.  Weights must be finite and >= 0, and every row
 * needs one positive weight (else INVALID_ARG).  Data are copied. */
smg_status smg_hier_from_prolongations(int32_t n_levels, const int32_t *sizes,
                                       const int32_t *const *p_cols,
                                       const double *const *p_w, smg_hier *out);

/* Write / read a hierarchy (sizes, vertex positions when known, P_l, the
 * decimation statistics) as a versioned binary file with a checksum, so the
 * geometry-only precompute is done once per mesh (Sec. 5) and reused.  A
 * loaded hierarchy is checked like smg_hier_from_prolongations and gives the
 * same solver layout as the one saved.  *out is released with
 * smg_hier_free.  Errors: INVALID_ARG (null, I/O error, wrong magic or
 * version, truncated file, checksum mismatch, invalid prolongation). */
smg_status smg_hier_save(smg_hier h, const char *path);
smg_status smg_hier_load(const char *path, smg_hier *out);

int32_t smg_hier_num_levels(smg_hier h);
int32_t smg_hier_level_size(smg_hier h, int32_t level);
/* Copy P_level (n_level x 3 ELL, unused slots: col -1, weight 0). */
smg_status smg_hier_get_prolongation(smg_hier h, int32_t level, int32_t *cols, double *w);
/* Per-level decimation statistics: collapses, failed tests, interior,
 * one-boundary, boundary case 1/2/3 counts, largest clamped barycentric. */
smg_status smg_hier_stats(smg_hier h, int32_t level, double *stats8);
void smg_hier_free(smg_hier h);

/* Greedy coloring of the off-diagonal graph of a CSR pattern (App. A, Alg.
 * "Graph Coloring": descending degree, ties by ascending index; first palette
 * color free among painted neighbours, moved to the palette's back; else a
 * new color).  color: n ids (host).  Returns the number of colors, or a
 * negative smg_status. */
int32_t smg_color_pattern(int32_t n, const int32_t *rowptr, const int32_t *cols, int32_t *color);

/* CSR pattern {diagonal} U {mesh edges}, columns ascending.  Call with
 * cols == NULL to get *nnz; then with cols of capacity *nnz. */
smg_status smg_mesh_pattern(int32_t n, const int32_t *F, int32_t m, int32_t *rowptr,
                            int32_t *cols, int32_t *nnz);

/* Host assembly (Sec. 6 systems A = M + t L, assembled once): the cotangent
 * Laplacian L (L_ij = -1/2 (cot alpha + cot beta) over the faces at edge ij,
 * one term on a boundary edge; L_ii = -sum_j L_ij) in the CSR order of
 * (rowptr, cols) = smg_mesh_pattern(F), and the lumped mass M_ii = (area of
 * the faces at i) / 3.  L_vals: rowptr[n] doubles, M_diag: n doubles, both
 * caller-sized host arrays.  Errors: INVALID_ARG (null, bad index, a
 * degenerate face, a pattern missing a diagonal or a face edge). */
smg_status smg_pre_assemble(const double *V, int32_t n, const int32_t *F, int32_t m, const int32_t *rowptr,
                            const int32_t *cols, double *L_vals, double *M_diag);

/* ------------------------------------------------------------------------ */
/* Context: the device and the allocator of every internal device buffer.  */

/* alloc returns `bytes` of device memory on the context's device (NULL on
 * failure), aligned to at least 256 bytes; free returns a block with the
 * size it was taken with.  They are called only inside smg_solver_create,
 * smg_batch_create and the destroy calls, on the calling thread (e.g. torch's
 * caching allocator from Python). */
typedef void *(*smg_alloc_fn)(size_t bytes, void *user);
typedef void (*smg_free_fn)(void *p, size_t bytes, void *user);
/* alloc and free both NULL: hipMalloc / hipFree.  The context must outlive
 * every solver created in it.  Errors: INVALID_ARG (bad device, only one
 * function given). */
smg_status smg_ctx_create(int32_t device, smg_alloc_fn alloc, smg_free_fn free_fn, void *user, smg_ctx *out);
void smg_ctx_destroy(smg_ctx ctx);

/* ------------------------------------------------------------------------ */
/* Device solver.                                                           */

typedef struct {
    int32_t mu_pre;        /* pre-relaxation sweeps (Sec. 5 default 2)  */
    int32_t mu_post;       /* post-relaxation sweeps (Sec. 5 default 2) */
    int32_t tail_rows;     /* levels with at most this many rows (and all
                              coarser ones) run in one single-workgroup kernel
                              per cycle, their iterates held in LDS (a level
                              joins only if the whole tail fits one
                              workgroup's LDS for the call's precision and
                              k); 0 = 4096, < 0 = never                     */
    int32_t lanes_per_row[16]; /* per level 1/2/4/8 lanes per matrix row in
                              the relaxation/residual kernels and, on levels
                              of the one-workgroup tail, in its passes; 0 =
                              rule (kernels: 1 if the mean row has < 10
                              entries, else 8; tail: the widest group up to
                              4 that fits a whole color in one pass); launch shape
                              only: results do not depend on it beyond
                              summation order                              */
    int32_t team_level;    /* > 0: this level and all coarser ones run in one
                              kernel by a team of workgroups on one XCD that
                              meet at L2-local barriers (between colors and
                              phases) instead of kernel boundaries; 0 = off
                              (per-color launches, then the LDS tail)     */
    int32_t team_size;     /* workgroups of that team, 1..16 (0 = 16)       */
} smg_opts;

/* Upload a hierarchy for the level-0 pattern (a0_rowptr, a0_cols: host CSR,
 * n0 = hierarchy level-0 size rows, diagonal present, columns ascending).
 * Builds on the host: R_l = P_l^T, the symbolic Galerkin patterns and their
 * numeric plans, the coloring of every smoothed level (App. A) and the
 * color-major layout; then copies everything to device `device`.
 * opts may be NULL (2/2).  The coarsest level is factored densely and may
 * have at most 16384 rows (INVALID_ARG beyond).  Every device buffer any
 * later call needs (work vectors of CG and of damped Jacobi included) is
 * taken here.  Errors: INVALID_ARG, OOM, HIP. */
smg_status smg_solver_create(int32_t device, smg_hier h, const int32_t *a0_rowptr,
                             const int32_t *a0_cols, const smg_opts *opts, smg_solver *out);
/* The same on the device of ctx, with its allocator. */
smg_status smg_solver_create_ctx(smg_ctx ctx, smg_hier h, const int32_t *a0_rowptr,
                                 const int32_t *a0_cols, const smg_opts *opts, smg_solver *out);
void smg_solver_destroy(smg_solver s);

/* Enable on-device assembly for the mesh faces F (m x 3, host). The level-0
 * pattern must be smg_mesh_pattern(F). */
smg_status smg_solver_attach_mesh(smg_solver s, const int32_t *F, int32_t m);

/* On-device A_0 = diag(s .* m) + t L_w (cotan Laplacian with optional per-edge
 * weights, lumped mass; the system of the paper's Sec. 6 examples):
 *   d_V: n x 3 positions; d_mass_scale: n (NULL = 1); d_edge_w: one weight per
 *   edge of the canonical sorted edge list (i < j, lexicographic) (NULL = 1).
 * Writes d_a0_vals (nnz, CSR order) and, if non-NULL, d_l_vals (L_w in CSR
 * order) and d_mass (n, unscaled lumped mass).  Requires attach_mesh. */
smg_status smg_assemble(smg_solver s, const double *d_V, double t, const double *d_mass_scale,
                        const float *d_edge_w, double *d_a0_vals, double *d_l_vals,
                        double *d_mass, smg_stream stream);

/* Set A_0 (d_a0_vals in the CSR order given at create) and refresh the whole
 * hierarchy on the device: Galerkin A_{l+1} = P_l^T A_l P_l for every level
 * (Eq. gca; "store the system matrix hierarchy", Sec. 5), FP32 copies, and the
 * dense FP64 Cholesky factor of the coarsest A_H.  Errors: NOT_SPD, HIP. */
smg_status smg_set_values(smg_solver s, const double *d_a0_vals, smg_stream stream);

int32_t smg_num_levels(smg_solver s);
int32_t smg_level_size(smg_solver s, int32_t level);
int64_t smg_level_nnz(smg_solver s, int32_t level);
/* Colors of level `level` (host array of n_level ids, may be NULL); returns
 * the number of colors (0 for the coarsest level). */
int32_t smg_level_colors(smg_solver s, int32_t level, int32_t *color);
/* Host copy of A_level in CSR (natural numbering, ascending columns,
 * structural pattern incl. explicit zeros).  Sizes from smg_level_nnz. */
smg_status smg_get_level_matrix(smg_solver s, int32_t level, int32_t *rowptr, int32_t *cols,
                                double *vals);
/* Host copy of the coarsest factor G (A_H = G G^T), n_H x n_H column-major,
 * upper part zero. */
smg_status smg_get_coarse_factor(smg_solver s, double *G);

/* --- one step of the V-cycle on level l (for parity checks) ---
 * precision SMG_FP64 runs the step on the FP64 level matrices.  SMG_FP32_IR
 * runs the kernels of the FP32 inner cycles: the FP64 input vectors are
 * rounded to FP32, the step reads the FP32 copies of the level matrices and
 * of P_l, accumulates in FP32, and its FP32 result is returned widened to
 * FP64 (exactly).  Vectors stay FP64 at the ABI. */
/* r = b - A_l x  (Alg. "V-cycle", restriction line, inner term) */
smg_status smg_residual(smg_solver s, int32_t level, int32_t precision, const double *d_b, const double *d_x,
                        double *d_r, int32_t k, smg_stream stream);
/* `sweeps` multicolor Gauss-Seidel sweeps in place on x (App. A); the
 * per-color launches on every level (the one-workgroup tail of the cycle
 * runs only inside smg_vcycle / smg_solve) */
smg_status smg_smooth(smg_solver s, int32_t level, int32_t precision, const double *d_b, double *d_x, int32_t k,
                      int32_t sweeps, smg_stream stream);
/* rc = P_l^T r  (restriction, R = P^T, Eq. gca) */
smg_status smg_restrict(smg_solver s, int32_t level, int32_t precision, const double *d_r, double *d_rc,
                        int32_t k, smg_stream stream);
/* x += P_l e  (prolong correction and update) */
smg_status smg_prolong_add(smg_solver s, int32_t level, int32_t precision, const double *d_e, double *d_x,
                           int32_t k, smg_stream stream);
/* x = A_H^{-1} b, the coarsest direct solve: A_H^{-1} is formed once per
 * smg_set_values from the Cholesky factor G (A_H^{-1} = G^{-T} G^{-1}) and
 * applied as a dense product with FP64 accumulation (SMG_FP32_IR: b rounded
 * to FP32 on entry and x to FP32 on exit, as inside the FP32 cycles) */
smg_status smg_coarse_solve(smg_solver s, int32_t precision, const double *d_b, double *d_x, int32_t k,
                            smg_stream stream);
/* One step of the one-workgroup tail: the device code that smg_solve and
 * smg_vcycle run, in one workgroup per right-hand side with the iterates in
 * LDS, for the levels with at most tail_rows rows (those from which every
 * coarser level fits one workgroup's LDS for the precision and k; else
 * INVALID_ARG).  It runs one step alone on one level with the same thread
 * mapping and summation order as inside the tail, so chaining these calls
 * in the order of Alg. "V-cycle" reproduces the tail's result exactly.
 *   SMG_TAIL_RELAX     d_in = b, d_out = x (in/out): |sweeps| multicolor
 *                      Gauss-Seidel sweeps, colors descending if sweeps < 0
 *   SMG_TAIL_RESIDUAL  d_in = b, d_in2 = x, d_out = r = b - A_l x
 *   SMG_TAIL_RESTRICT  d_in = r (level l), d_out = P_l^T r (level l + 1)
 *   SMG_TAIL_PROLONG   d_in = e (level l + 1), d_out = x (in/out) += P_l e
 *   SMG_TAIL_COARSE    level = coarsest: d_in = b, d_out = A_H^{-1} b
 * Vectors are n_level x k FP64 at the ABI, rounded to FP32 on entry for
 * SMG_FP32_IR as in smg_residual.  Errors: INVALID_ARG, STATE. */
/* The finest level of the one-workgroup tail for this precision and k
 * (num_levels - 1 when no smoothed level is in it); -1 on a bad argument. */
int32_t smg_tail_first_level(smg_solver s, int32_t precision, int32_t k);
enum { SMG_TAIL_RELAX = 0, SMG_TAIL_RESIDUAL = 1, SMG_TAIL_RESTRICT = 2, SMG_TAIL_PROLONG = 3,
       SMG_TAIL_COARSE = 4 };
smg_status smg_tail_step(smg_solver s, int32_t level, int32_t step, int32_t precision, const double *d_in,
                         const double *d_in2, double *d_out, int32_t k, int32_t sweeps, smg_stream stream);
/* One cycle at level 0 in place on x, in the launch shape smg_solve uses.
 * SMG_FP64: one V-cycle (Alg. "V-cycle").  SMG_FP32_IR: one refinement step
 * of the mixed solve: r = b - A x and sigma_q = max_i |r_iq| in FP64, one
 * FP32 V-cycle from zero on fp32(r / sigma) (FP32 relaxation, residuals,
 * transfers and tail, FP64 coarsest product), then x += sigma * d in FP64
 * (a column with sigma = 0 is left unchanged).  A one-level hierarchy takes
 * SMG_FP64 only (its cycle is the direct solve). */
smg_status smg_vcycle(smg_solver s, int32_t precision, const double *d_b, double *d_x, int32_t k,
                      smg_stream stream);

/* --- the solve (Alg. "Galerkin Surface Multigrid Solver") --- */
typedef struct {
    double rtol;           /* stop when max_c ||b_c - A x_c|| / ||b_c|| <= rtol */
    int32_t max_cycles;    /* cap (SMG_ERR_NO_CONVERGENCE when reached)         */
    int32_t precision;     /* SMG_FP64 or SMG_FP32_IR                            */
    int32_t fixed_cycles;  /* > 0: run exactly this many cycles, no stop test   */
    int32_t use_graph;     /* 1: replay each cycle from a captured hipGraph     */
    int32_t timed;         /* 1: fill info->ms_phase (an event at every change
                              of phase on the stream; cycles run eagerly)     */
} smg_solve_params;

/* Phases of a solve, as Tab. "profile" of the paper splits the time */
enum { SMG_PHASE_PREPARE = 0,   /* A_{l+1} = P^T A P and coarsest factor (the last
                                   smg_set_values / smg_split_combine)          */
       SMG_PHASE_RELAX = 1,     /* Gauss-Seidel / Jacobi sweeps; the one-workgroup
                                   tail (mostly relaxation passes) counts here  */
       SMG_PHASE_TRANSFER = 2,  /* residuals feeding the restriction,
                                   restriction, prolongation                    */
       SMG_PHASE_NORM = 3,      /* level-0 FP64 residual and its column norms
                                   (the stop test and the refinement residual)  */
       SMG_PHASE_OTHER = 4 };   /* coarsest solves outside the tail, refinement
                                   scaling and update, set-up of the solve      */

typedef struct {
    int32_t cycles;        /* V-cycles run (outer refinement steps for FP32_IR) */
    int32_t k;
    double rel_res[4];     /* final FP64 relative residual per column           */
    double ms;             /* wall time of the solve on the stream              */
    double ms_phase[5];    /* device time by SMG_PHASE_* (index); [0] always,
                              [1..4] when params->timed, else 0               */
} smg_solve_info;

/* x = A^{-1} b from x0 = 0.  SMG_FP32_IR runs relaxation, residual and
 * transfers of every cycle in FP32 (FP32 accumulation) inside an FP64
 * iterative-refinement loop: FP64 outer residual, FP64 coarsest Cholesky,
 * FP64 update.  info may be NULL.  Errors: STATE, NONFINITE, NO_CONVERGENCE.
 * The calling thread polls (busy-waits) for each cycle's residual norms; with
 * SMG_FP32_IR and no graph the next cycle's first part is already queued
 * while it does, and its result is discarded when the stop test ends the
 * solve (x is always the iterate of info->cycles cycles). */
smg_status smg_solve(smg_solver s, const double *d_b, double *d_x, int32_t k,
                     const smg_solve_params *p, smg_solve_info *info, smg_stream stream);

/* --- Dirichlet conditions (App. B) ---
 * x_k = c on the known vertices: solve A_uu x_u = b_u - A_uk c.  The
 * multigrid hierarchy of the reduced system keeps every level except the
 * finest transfer, whose rows become P_{u:} (the rows of P_0 of the
 * unknowns); coarse vertices that then receive no weight are removed with
 * the matching rows of the next prolongation (level by level).
 * smg_hier_dirichlet: known = n_0 flags (natural order, nonzero = known);
 * unknown_idx (n_0 capacity) receives the unknowns' natural indices in
 * ascending order, *n_unknown their count; *out a new hierarchy (free with
 * smg_hier_free).  Errors: INVALID_ARG (null, all known).
 * smg_dirichlet_pattern (host): the CSR pattern of A_uu from A's pattern
 * (rows/columns of the unknowns, order kept); u_rowptr needs n + 1 and
 * u_cols nnz(A) capacity.  Errors: INVALID_ARG.
 * smg_dirichlet_reduce (device, on `stream`): A_uu values in that pattern
 * (d_u_rowptr = the pattern's row pointers on the device) and
 * rhs = b_u - A_uk x_k for k columns (d_x, d_b: n_0 x k, the known entries
 * of d_x used).  All pointers device, inputs from the same known mask.
 * Errors: INVALID_ARG. */
smg_status smg_hier_dirichlet(smg_hier h, const uint8_t *known, smg_hier *out, int32_t *unknown_idx,
                              int32_t *n_unknown);
smg_status smg_dirichlet_pattern(int32_t n, const int32_t *rowptr, const int32_t *cols, const uint8_t *known,
                                 int32_t *u_rowptr, int32_t *u_cols, int32_t *n_unknown, int32_t *nnz_unknown);
smg_status smg_dirichlet_reduce(int32_t n_unknown, const int32_t *d_unknown_idx, const int32_t *d_rowptr,
                                const int32_t *d_cols, const double *d_vals, const uint8_t *d_known,
                                const double *d_x, const double *d_b, int32_t k, const int32_t *d_u_rowptr,
                                double *d_u_vals, double *d_rhs, smg_stream stream);

/* --- split Galerkin (App. E): P^T (a Q + b M) P = a P^T Q P + b P^T M P ---
 * smg_split_prepare runs the Galerkin products of two level-0 matrices on
 * the solver's pattern (device CSR values in smg_set_values order; e.g. the
 * cotan Laplacian and the lumped mass) and keeps every level of both (two
 * extra copies of the level values).  smg_split_combine then sets the
 * values to a Q + b M on every level with one a x + b y per level plus the
 * FP32 copies, LDS-tail records, coarsest Cholesky/inverse (and Jacobi
 * factors), i.e. a change of a and b needs no assembly and no Galerkin
 * product.  prepare leaves no values set; combine waits for the device.
 * Errors: INVALID_ARG, STATE (combine before prepare), NONFINITE (prepare),
 * NOT_SPD (combine), OOM. */
smg_status smg_split_prepare(smg_solver s, const double *d_q_vals, const double *d_m_vals, smg_stream stream);
smg_status smg_split_combine(smg_solver s, double a, double b, smg_stream stream);

/* --- relaxation method (App. "Ablation Study") ---
 * SMG_SMOOTH_GS (default): multicolor Gauss-Seidel (App. A), one launch per
 * color, the small levels in one workgroup.  SMG_SMOOTH_JACOBI: damped
 * Jacobi x <- x + omega_l D^{-1} (b - A x), one launch per sweep on every
 * level.  omega in (0, 2) sets omega_l = omega on every level; omega <= 0
 * (the paper gives no factor) sets omega_l = 2 / (1 + lambda_l) with
 * lambda_l the Rayleigh quotient of A_l after 20 power steps
 * v <- D_l^{-1} A_l v from v_i = frac(0.6180339887498949 (i + 1)) - 1/2
 * (i the natural row index), recomputed whenever the values change.
 * Applies to every later smooth, V-cycle, solve and PCG call of s (the
 * Jacobi V-cycle is symmetric as it is); its second iterate per level is
 * taken at smg_solver_create.  Waits for the
 * device and drops captured cycle graphs.  Batches take GS solvers only.
 * Errors: INVALID_ARG (omega >= 2 or NaN, unknown kind), OOM. */
smg_status smg_set_smoother(smg_solver s, int32_t kind, double omega);
/* *omega = the Jacobi factor of a smoothed level (host; waits for the
 * device).  Errors: INVALID_ARG, STATE (GS selected or values not set). */
smg_status smg_get_jacobi_omega(smg_solver s, int32_t level, double *omega);

/* --- conjugate gradients preconditioned by one V-cycle (the combination
 * proposed in Sec. "Limitations & Future Work") ---
 * x = A^{-1} b from x0 = 0, one CG run per column (textbook preconditioned
 * CG).  The preconditioner is one V-cycle from zero whose post-relaxation
 * visits the colors in descending order, the adjoint of the pre-relaxation,
 * so that it is symmetric positive definite (needs mu_pre == mu_post).
 * Stops when max_c ||r_c|| / ||b_c|| <= p->rtol for the recurrence residual
 * r; p->max_cycles caps the iterations (one V-cycle each), p->fixed_cycles
 * > 0 runs exactly that many.  p->precision: SMG_FP64, or SMG_FP32_IR for
 * an FP32 V-cycle on r scaled by max |r| per column (vectors, dot products
 * and updates stay FP64).  p->use_graph must be 0.  info->cycles =
 * iterations, info->rel_res = final recurrence residuals.  Its three n x 4
 * FP64 work vectors are taken at smg_solver_create.  Errors: INVALID_ARG, STATE,
 * NONFINITE, NO_CONVERGENCE, OOM. */
smg_status smg_pcg_solve(smg_solver s, const double *d_b, double *d_x, int32_t k,
                         const smg_solve_params *p, smg_solve_info *info, smg_stream stream);

/* --- adjoint helpers for A = diag(s.*m) + t L (differentiation) --- */
/* *h_out = lambda^T L u over the level-0 pattern (d_l_vals in CSR order), k = 1 */
smg_status smg_spmv_dot(smg_solver s, const double *d_l_vals, const double *d_lambda,
                        const double *d_u, double *h_out, smg_stream stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the value of
 * smg_spmv_dot, lambda^T L u, with no solver and no allocation.  d_rowptr
 * (n + 1), d_cols and d_vals (rowptr[n] entries) are the CSR matrix, d_lambda
 * and d_u length n, all device memory owned by the caller; the sum is written
 * to d_out[0] (device) on `stream`, with the kernels and summation order of
 * smg_spmv_dot (the same value bit for bit).  Its per-block partial sums live
 * in a static 1 MiB device array (one per GPU, kept until the process ends):
 * n may be at most 16,776,960 rows (INVALID_ARG above that, before any
 * launch).  Every call on one GPU shares that array, so calls that overlap on
 * one GPU (different streams or host threads) race; calls in one stream order
 * are safe.  Errors: INVALID_ARG, HIP. */
smg_status smg_spmv_dot_noalloc(int32_t n, const int32_t *d_rowptr, const int32_t *d_cols,
                                const double *d_vals, const double *d_lambda, const double *d_u,
                                double *d_out, smg_stream stream);
/* d_out[i] = -lambda_i * m_i * u_i */
smg_status smg_mass_grad(smg_solver s, const double *d_lambda, const double *d_m,
                         const double *d_u, double *d_out, smg_stream stream);

/* --- per-launch kernel timing (HIP events on the launch stream) --- */
enum { SMG_PROF_GS = 0, SMG_PROF_RESIDUAL = 1, SMG_PROF_RESTRICT = 2, SMG_PROF_PROLONG = 3,
       SMG_PROF_COARSE = 4, SMG_PROF_GALERKIN = 5, SMG_PROF_GROUP = 0x100 };
/* Time every launch of kernel `kind` on level `level` (-1: every level; any
 * precision) with start/stop events stamped by the dispatch itself, until
 * disabled (kind < 0).  kind | SMG_PROF_GROUP (Gauss-Seidel only) instead
 * puts one event pair around each relaxation call's launches (every sweep
 * and color of one level's pre- or post-relaxation): the time then includes
 * the gaps between those back-to-back launches, and the launch count is
 * every launch inside.  Solves with use_graph run their cycles eagerly while
 * profiling is on. */
smg_status smg_profile_enable(smg_solver s, int32_t kind, int32_t level);
/* Totals since enable: summed launch durations (ms), launch count, and the
 * algorithmic bytes of those launches (what a CSR sweep must move: z (s + 4)
 * + 4 (n + 1) + 3 k n s for a relaxation sweep or a residual over n rows
 * with z matrix entries, diagonal included, s = 8 or 4 bytes per value, k
 * right-hand sides, neighbour values of x counted once; a color of a sweep
 * counts its own rows' share, the first color the extra row pointer).
 * Synchronizes the device. */
smg_status smg_profile_read(smg_solver s, double *total_ms, int64_t *launches, double *bytes);

/* Launch latency on this device, for the latency bound of the per-color
 * launches: `launches` (1..4000) back-to-back launches on `stream` with the
 * grid of level `level`'s widest color (one 64-thread workgroup per slice),
 * of an empty kernel (kind 0) or of a kernel whose threads load an index
 * (the level's own column array), then the value it points to, and store it
 * (kind 1: the dependent chain of a relaxation launch), or that chain with
 * the level's two FP32 work vectors alternating as source and destination,
 * so each launch gathers values the previous one wrote (kind 2, as
 * successive color launches do; both vectors are zero again on return).
 * The launches are queued behind a bounded sleep kernel that outlasts their
 * enqueueing, so
 * *us = the device's launch-to-launch time (one event pair around them all);
 * *us_host (may be NULL) = host time to enqueue one launch.  Synchronizes the
 * stream.  Errors: INVALID_ARG, HIP. */
smg_status smg_launch_floor(smg_solver s, int32_t kind, int32_t level, int32_t launches, smg_stream stream,
                            double *us, double *us_host);

/* ------------------------------------------------------------------------ */
/* Batching: many solvers in one persistent launch.                          */

typedef struct {
    int32_t threads;          /* workgroup size: 256, 512, 1024; 0 = tuned/default */
    int32_t lanes_level0;     /* lanes per row on level 0: 1 or 2; 0 = tuned/default */
    int32_t lanes_coarse;     /* lanes per row on the Galerkin levels: 1,2,4,8; 0 = tuned/default */
    int32_t team_max;         /* most workgroups per mesh (1..64); 0 = tuned/default */
    const char *cache_file;   /* autotune cache (read at create, written by autotune); may be NULL */
    int32_t device_teams;     /* 0: each team's workgroups on one XCD, meeting at barriers in
                                 that XCD's L2 (when the teams can be placed so); 1: teams
                                 anywhere, barriers through device-scope atomics */
    int32_t balance;          /* 1: workgroups per mesh by level-0 entries x the last solve's
                                 cycles (from the second solve on); 0: by entries (or tuned) */
} smg_batch_opts;

/* Group solvers (same device, at least two levels each) for batched solves:
 * one persistent kernel runs every mesh's whole solve.  Each mesh is worked
 * by a team of workgroups (1..team_max, in proportion to its size, all
 * resident at once; largest meshes first) that loops over its own V-cycles
 * with barriers between dependent phases and the convergence test on the
 * device; converged meshes stop.  Unless o->device_teams, whole teams are
 * packed onto the 8 XCDs (workgroups i and i + 8 are dispatched to the same
 * XCD) so that a team's barriers stay in its XCD's L2; a team found spread
 * over XCDs fails the solve (HIP).  The solvers must outlive the batch.
 * Errors: INVALID_ARG, OOM. */
smg_status smg_batch_create(const smg_solver *solvers, int32_t count, const smg_batch_opts *o,
                            smg_batch *out);
void smg_batch_destroy(smg_batch b);
/* Solve mesh i: x_i = A_i^{-1} b_i (k[i] columns, caller order), precision
 * SMG_FP32_IR (FP32 cycles, FP64 residual / update / coarsest solve) or
 * SMG_FP64, all meshes in ONE kernel launch replayed from a hipGraph
 * (captured on the first call and after a launch-shape change).  infos
 * (count entries) may be NULL; fixed_cycles and use_graph are ignored.
 * Returns NO_CONVERGENCE if any mesh hit max_cycles (its x is the last
 * iterate), NONFINITE if any residual became non-finite, HIP if a team
 * barrier wait timed out (every wait is bounded; the kernel always ends). */
smg_status smg_batch_solve(smg_batch b, const double *const *d_b, double *const *d_x,
                           const int32_t *k, const smg_solve_params *p, smg_solve_info *infos,
                           smg_stream stream);
/* Autotuner: re-runs the last smg_batch_solve for candidate launch shapes
 * (workgroups per mesh, workgroup size, lanes per row on level 0 and on the
 * Galerkin levels; teams sized by level-0 entries or, with the last solve's
 * cycle counts, by entries x cycles, so the meshes that take longest get the
 * larger teams; a cached work-sized shape takes effect from the second solve),
 * keeps the fastest whose solve converged, and writes it to the cache file
 * if one was given.  It never changes mu, the levels, the coloring or the
 * color order.  budget_ms bounds the search.  The last solve's x buffers end
 * up holding a solve in the chosen shape (the original shape when no
 * candidate converged).  Errors: STATE (no previous solve), and the errors of
 * smg_batch_solve other than NO_CONVERGENCE and NONFINITE, which only
 * disqualify a shape (the final solve in the chosen shape reports them). */
smg_status smg_batch_autotune(smg_batch b, int32_t budget_ms, smg_stream stream);
/* Current launch shape into shape5: threads, lanes_level0, lanes_coarse,
 * team_max, balance (1: teams sized by entries x cycles). */
smg_status smg_batch_shape(smg_batch b, int32_t *shape5);

const char *smg_status_string(smg_status st);
const char *smg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SMG_H */
