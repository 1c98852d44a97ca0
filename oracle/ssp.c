/*
 * ORACLE (test infrastructure only; never linked by the product library).
 *
 * Plain FP64 successive self-parameterization for ONE decimation level:
 * mid-point edge collapses of a manifold triangle mesh, each followed by the
 * joint LSCM flattening of the edge 1-ring before the collapse and the vertex
 * 1-ring after it (paper Sec. 4.1 "Successive Self-Parameterization", Sec. 4.2
 * "Joint Flattening", Eq. jointEnergy, Sec. 4.3 "Boundary Edges",
 * Sec. 4.4 mid-point collapse + LSCM, App. C).  Every fine vertex is carried
 * through each collapse as (face, barycentric) via the shared UV domain
 * (Fig. baryQuery), which yields the rows of the prolongation P (Sec. 4.5:
 * three barycentric weights per row).
 *
 * Readings where the paper is silent (same readings as the design notes):
 *  - priority: squared 3D edge length, shortest first, ties by (min id, max id);
 *    an edge that fails is retried only after a collapse whose new 1-ring
 *    contains one of its endpoints;
 *  - validity: link condition, no interior edge between two boundary
 *    vertices, no vertex left without faces, non-singular LSCM, and every UV
 *    triangle of both patches with signed area > 1e-12 * scale^2;
 *  - gauge: interior / one-boundary collapses pin the two ring vertices farthest
 *    apart in 3D at (0,0) and (d,0); boundary-edge collapses put the colinear
 *    vertices on v = 0 and pin u of the first and last to 0 and to the 3D
 *    length of the boundary chain between them;
 *  - query: a point goes to the after-patch triangle with the largest minimum
 *    barycentric coordinate (ties: lowest face id); negative coordinates are
 *    clamped to 0 and the row renormalized; at the end weights < 1e-12 are
 *    dropped and the row renormalized.
 * What pins this file: on a flat disc with interior collapses every row must
 * be the planar barycentric coordinates of the fine vertex in the coarse
 * triangle that contains it, in the xy plane and after a rigid motion into a
 * tilted plane; the same holds when boundary-edge collapses on straight
 * boundary runs are allowed too (there the third boundary case, the new
 * vertex on the line through i and j, meets every constraint with zero
 * energy, so it must win); every collapse of a curved disc (interior,
 * one-boundary and all three boundary-edge cases) is re-solved from the 3D
 * triangles by an independent least-squares formulation of the conformal
 * energy, which must give the same per-case energies, the same winning case
 * and the same UV positions; on any mesh, rows are nonnegative, sum to 1,
 * have at most three entries, leave no coarse column empty, keep the Euler
 * characteristic, and are bitwise unchanged by a power-of-two scale and
 * unchanged to rounding by a rigid motion.  The rows on curved meshes have
 * no closed form or printed values to compare with: parity unpinned there
 * beyond these checks.
 * Compile with -ffp-contract=off.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------- small growable int list ---------- */
typedef struct { int *a; int n, cap; } ilist;

static void il_push(ilist *l, int v) {
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 8;
        l->a = (int *)realloc(l->a, sizeof(int) * (size_t)l->cap);
    }
    l->a[l->n++] = v;
}

/* ---------- binary min-heap of edges ---------- */
typedef struct { double len2; int a, b; } hent;
typedef struct { hent *e; long n, cap; } heap;

static int h_less(const hent *x, const hent *y) {
    if (x->len2 != y->len2) return x->len2 < y->len2;
    if (x->a != y->a) return x->a < y->a;
    return x->b < y->b;
}
static void h_push(heap *h, hent v) {
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->e = (hent *)realloc(h->e, sizeof(hent) * (size_t)h->cap);
    }
    long i = h->n++;
    h->e[i] = v;
    while (i > 0) {
        long p = (i - 1) / 2;
        if (!h_less(&h->e[i], &h->e[p])) break;
        hent t = h->e[i]; h->e[i] = h->e[p]; h->e[p] = t;
        i = p;
    }
}
static hent h_pop(heap *h) {
    hent top = h->e[0];
    h->e[0] = h->e[--h->n];
    long i = 0;
    for (;;) {
        long l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->n && h_less(&h->e[l], &h->e[s])) s = l;
        if (r < h->n && h_less(&h->e[r], &h->e[s])) s = r;
        if (s == i) break;
        hent t = h->e[i]; h->e[i] = h->e[s]; h->e[s] = t;
        i = s;
    }
    return top;
}

/* ---------- mesh state ---------- */
typedef struct {
    int nv, capv;
    double *X;       /* 3 * capv positions */
    char *valive;
    ilist *vf;       /* incident alive faces per vertex */
    int nf;
    int *F;          /* 3 * nf, updated in place */
    char *falive;
} mesh;

static double len2(const mesh *M, int a, int b) {
    double dx = M->X[3 * a] - M->X[3 * b];
    double dy = M->X[3 * a + 1] - M->X[3 * b + 1];
    double dz = M->X[3 * a + 2] - M->X[3 * b + 2];
    return dx * dx + dy * dy + dz * dz;
}

/* neighbours of v with multiplicity (how many incident faces contain them) */
static int neighbours(const mesh *M, int v, int *ids, int *cnt, int cap) {
    int n = 0;
    const ilist *L = &M->vf[v];
    for (int t = 0; t < L->n; ++t) {
        const int *f = &M->F[3 * L->a[t]];
        for (int c = 0; c < 3; ++c) {
            int w = f[c];
            if (w == v) continue;
            int s = 0;
            while (s < n && ids[s] != w) ++s;
            if (s == n) {
                if (n == cap) return -1;
                ids[n] = w; cnt[n] = 0; ++n;
            }
            cnt[s]++;
        }
    }
    return n;
}

static int is_boundary_vertex(const mesh *M, int v) {
    int ids[256], cnt[256];
    int n = neighbours(M, v, ids, cnt, 256);
    for (int s = 0; s < n; ++s) if (cnt[s] == 1) return 1;
    return 0;
}

/* the boundary neighbour of v other than `other` (v must be a boundary vertex) */
static int other_boundary_neighbour(const mesh *M, int v, int other) {
    int ids[256], cnt[256];
    int n = neighbours(M, v, ids, cnt, 256);
    for (int s = 0; s < n; ++s)
        if (cnt[s] == 1 && ids[s] != other) return ids[s];
    return -1;
}

/* ---------- dense linear algebra (Gaussian elimination, partial pivoting) ---------- */
static int gauss_solve(double *A, double *b, int n) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = fabs(A[c * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > best) { best = fabs(A[r * n + c]); piv = r; }
        if (!(best > 1e-300)) return -1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) { double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * b[k];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/* ---------- joint LSCM ---------- */
#define MAXD 96          /* max joint DOFs per patch pair */
#define MAXF 96          /* max faces per patch */

typedef struct {
    int nfb, nfa;
    int fb_id[MAXF], fb_v[MAXF][3];  /* before faces: ids, vertex ids */
    int fa_id[MAXF], fa_v[MAXF][3];  /* after faces (i, j replaced by k) */
    int fb_d[MAXF][3], fa_d[MAXF][3];/* DOF per corner */
    int nd;                          /* joint DOFs */
    double U[MAXD][2];               /* solved UV per DOF */
    double energy, scale;
} jpatch;

/* Add the LSCM rows of triangle with 3D corners (P0,P1,P2) and DOFs d[3] to the
 * least-squares matrix R (rows x 2nd). Row pair encodes
 *   (W0 U0 + W1 U1 + W2 U2) / (2 sqrt(area)),  W_j = (x_l - x_k) + i (y_l - y_k)
 * in the triangle's own orthonormal frame, so the squared residual is
 * area * |dU/dx + i dU/dy|^2, the conformal (LSCM) energy of the triangle. */
static int lscm_rows(const double *P0, const double *P1, const double *P2, const int *d,
                     double *R, int row, int ncol) {
    double e1[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
    double e2[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
    double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    double cx = e1[1] * e2[2] - e1[2] * e2[1];
    double cy = e1[2] * e2[0] - e1[0] * e2[2];
    double cz = e1[0] * e2[1] - e1[1] * e2[0];
    double cn = sqrt(cx * cx + cy * cy + cz * cz);
    if (!(l1 > 0.0) || !(cn > 0.0)) return -1;
    double x[3] = {0.0, l1, (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) / l1};
    double y[3] = {0.0, 0.0, cn / l1};
    double area = 0.5 * cn;
    double s = 1.0 / (2.0 * sqrt(area));
    double *re = &R[(size_t)row * ncol];
    double *im = &R[(size_t)(row + 1) * ncol];
    for (int j = 0; j < 3; ++j) {
        int k = (j + 1) % 3, l = (j + 2) % 3;
        double wr = (x[l] - x[k]) * s, wi = (y[l] - y[k]) * s;
        int cu = 2 * d[j], cv = 2 * d[j] + 1;
        /* (wr + i wi)(u + i v) = (wr u - wi v) + i (wi u + wr v) */
        re[cu] += wr; re[cv] -= wi;
        im[cu] += wi; im[cv] += wr;
    }
    return 0;
}

static double tri_area2(const double *a, const double *b, const double *c) {
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

/* Solve the joint flattening for a DOF assignment already stored in jp.
 * fixed[c] >= 0 marks column c (2*dof + coord) as fixed with value val[c]. */
static int joint_solve(const mesh *M, jpatch *jp, const int *fixed, const double *val) {
    int ncol = 2 * jp->nd;
    int nrow = 2 * (jp->nfb + jp->nfa);
    double *R = (double *)calloc((size_t)nrow * ncol, sizeof(double));
    int row = 0;
    for (int t = 0; t < jp->nfb; ++t) {
        const int *v = jp->fb_v[t];
        if (lscm_rows(&M->X[3 * v[0]], &M->X[3 * v[1]], &M->X[3 * v[2]], jp->fb_d[t], R, row, ncol)) { free(R); return -1; }
        row += 2;
    }
    for (int t = 0; t < jp->nfa; ++t) {
        const int *v = jp->fa_v[t];
        if (lscm_rows(&M->X[3 * v[0]], &M->X[3 * v[1]], &M->X[3 * v[2]], jp->fa_d[t], R, row, ncol)) { free(R); return -1; }
        row += 2;
    }
    /* free-column index */
    int fidx[2 * MAXD], nfree = 0;
    for (int c = 0; c < ncol; ++c) fidx[c] = fixed[c] ? -1 : nfree++;
    double *N = (double *)calloc((size_t)nfree * nfree, sizeof(double));
    double *rhs = (double *)calloc((size_t)nfree, sizeof(double));
    for (int r = 0; r < nrow; ++r) {
        const double *Rr = &R[(size_t)r * ncol];
        double fixsum = 0.0;
        for (int c = 0; c < ncol; ++c) if (fixed[c]) fixsum += Rr[c] * val[c];
        for (int c = 0; c < ncol; ++c) {
            if (fixed[c] || Rr[c] == 0.0) continue;
            int fc = fidx[c];
            rhs[fc] -= Rr[c] * fixsum;
            for (int c2 = 0; c2 < ncol; ++c2) {
                if (fixed[c2] || Rr[c2] == 0.0) continue;
                N[fc * nfree + fidx[c2]] += Rr[c] * Rr[c2];
            }
        }
    }
    int rc = gauss_solve(N, rhs, nfree);
    if (rc == 0) {
        double z[2 * MAXD];
        for (int c = 0; c < ncol; ++c) z[c] = fixed[c] ? val[c] : rhs[fidx[c]];
        for (int d = 0; d < jp->nd; ++d) { jp->U[d][0] = z[2 * d]; jp->U[d][1] = z[2 * d + 1]; }
        double e = 0.0;
        for (int r = 0; r < nrow; ++r) {
            double s = 0.0;
            for (int c = 0; c < ncol; ++c) s += R[(size_t)r * ncol + c] * z[c];
            e += s * s;
        }
        jp->energy = e;
        /* orientation / degeneracy test on both patches */
        double eps = 1e-12 * jp->scale * jp->scale;
        for (int t = 0; t < jp->nfb && rc == 0; ++t) {
            const int *d = jp->fb_d[t];
            if (!(0.5 * tri_area2(jp->U[d[0]], jp->U[d[1]], jp->U[d[2]]) > eps)) rc = -2;
        }
        for (int t = 0; t < jp->nfa && rc == 0; ++t) {
            const int *d = jp->fa_d[t];
            if (!(0.5 * tri_area2(jp->U[d[0]], jp->U[d[1]], jp->U[d[2]]) > eps)) rc = -2;
        }
    }
    free(R); free(N); free(rhs);
    return rc;
}

/* ---------- level driver ---------- */

/* Which edges may collapse.  ALL is the method; the other two are test
 * options that restrict it to collapses with a closed-form result on a flat
 * disc: INTERIOR keeps edges with both endpoints interior; STRAIGHT keeps
 * those plus boundary edges whose previous, own and next boundary vertices
 * (p, i, j, q) lie on one straight line, and no one-boundary collapse. */
enum { COLLAPSE_ALL = 0, COLLAPSE_INTERIOR = 1, COLLAPSE_STRAIGHT = 2 };

/* Probe record of one committed collapse (test infrastructure): doubles
 *   [0..9]   kind (0 interior, 1 one-boundary, 2 boundary edge), chosen case,
 *            i, j, p, q, k, ring size nr, before-face count nfb, case count
 *   ring     PR_RING: ring vertex ids (ascending)
 *   faces    PR_FACE: 3 vertex ids per before face (ascending face id)
 *   per case PR_CASE: flatten status (0 ok), energy, UV of each ring vertex,
 *            UV of i and j in the before patch, UV of k in the after patch. */
#define PR_HDR 10
#define PR_RING PR_HDR
#define PR_FACE (PR_RING + MAXD)
#define PR_CASE0 (PR_FACE + 3 * MAXF)
#define PR_CASE_SIZE (2 + 2 * MAXD + 6)
#define PR_SIZE (PR_CASE0 + 3 * PR_CASE_SIZE)

/* p, i, j, q on one line in this order: consecutive segments parallel (sine
 * of their angle below 1e-9) and pointing the same way. */
static int straight_run(const mesh *M, int p, int i, int j, int q) {
    int pts[4] = {p, i, j, q};
    for (int s = 0; s < 2; ++s) {
        const double *A = &M->X[3 * pts[s]], *B = &M->X[3 * pts[s + 1]], *C = &M->X[3 * pts[s + 2]];
        double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        double w[3] = {C[0] - B[0], C[1] - B[1], C[2] - B[2]};
        double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz = u[0] * w[1] - u[1] * w[0];
        double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double nw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (!(sqrt(cx * cx + cy * cy + cz * cz) <= 1e-9 * nu * nw)) return 0;
        if (!(u[0] * w[0] + u[1] * w[1] + u[2] * w[2] > 0.0)) return 0;
    }
    return 1;
}
typedef struct {
    long collapses, fails, case_int, case_one, case_b1, case_b2, case_b3;
    double max_clamp;
} sstats;

static double dist3(const mesh *M, int a, int b) { return sqrt(len2(M, a, b)); }

/*
 * Decimate (n, X, m, F) to `target` vertices.
 * Outputs: *nc coarse vertices (Xc, 3*nc), *mc coarse faces (Fc), and for each
 * fine vertex v three coarse columns Pc[3v..] and weights Pw[3v..] (weight 0
 * marks an unused slot, column then -1).  stats (7 longs + 1 double) optional.
 * mode is one of the COLLAPSE_* sets above.
 * probe (optional, test infrastructure): room for probe_cap records of
 * PR_SIZE doubles; the first committed collapses are recorded there, their
 * count in *probe_n, and every vertex position created (3 * (2n + 8)
 * doubles, new vertex ids continue after n) in Xall.
 * Returns 0, or <0 on failure.
 */
int oracle_ssp_level_probe(int n, const double *X, int m, const int *F, int target, int mode,
                           int *nc, double *Xc, int *mc, int *Fc, int *Pc, double *Pw, double *stats_out,
                           double *probe, int probe_cap, int *probe_n, double *Xall) {
    mesh M;
    M.nv = n; M.capv = 2 * n + 8;
    M.X = (double *)malloc(sizeof(double) * 3 * (size_t)M.capv);
    memcpy(M.X, X, sizeof(double) * 3 * (size_t)n);
    M.valive = (char *)calloc((size_t)M.capv, 1);
    memset(M.valive, 1, (size_t)n);
    M.vf = (ilist *)calloc((size_t)M.capv, sizeof(ilist));
    M.nf = m;
    M.F = (int *)malloc(sizeof(int) * 3 * (size_t)m);
    memcpy(M.F, F, sizeof(int) * 3 * (size_t)m);
    M.falive = (char *)malloc((size_t)m);
    memset(M.falive, 1, (size_t)m);
    for (int f = 0; f < m; ++f)
        for (int c = 0; c < 3; ++c) il_push(&M.vf[F[3 * f + c]], f);

    /* query state: every fine vertex starts in its lowest-id incident face */
    int *qface = (int *)malloc(sizeof(int) * (size_t)n);
    double *qbar = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int *fhead = (int *)malloc(sizeof(int) * (size_t)m);
    int *qnext = (int *)malloc(sizeof(int) * (size_t)n);
    int *moved = (int *)malloc(sizeof(int) * (size_t)n);
    for (int f = 0; f < m; ++f) fhead[f] = -1;
    for (int v = 0; v < n; ++v) {
        int best = -1;
        for (int t = 0; t < M.vf[v].n; ++t) if (best < 0 || M.vf[v].a[t] < best) best = M.vf[v].a[t];
        if (best < 0) return -10;  /* isolated vertex */
        qface[v] = best;
        for (int c = 0; c < 3; ++c) qbar[3 * v + c] = (F[3 * best + c] == v) ? 1.0 : 0.0;
        qnext[v] = fhead[best];
        fhead[best] = v;
    }

    heap H = {0, 0, 0};
    for (int f = 0; f < m; ++f)
        for (int c = 0; c < 3; ++c) {
            int a = F[3 * f + c], b = F[3 * f + (c + 1) % 3];
            hent e = {len2(&M, a, b), a < b ? a : b, a < b ? b : a};
            h_push(&H, e);
        }

    sstats st;
    memset(&st, 0, sizeof(st));
    int alive = n;
    jpatch *jp = (jpatch *)malloc(sizeof(jpatch));
    jpatch *jbest = (jpatch *)malloc(sizeof(jpatch));

    while (alive > target && H.n > 0) {
        hent e = h_pop(&H);
        int a = e.a, b = e.b;
        if (!M.valive[a] || !M.valive[b]) continue;
        /* faces containing both endpoints */
        int fab[4], nfab = 0;
        for (int t = 0; t < M.vf[a].n; ++t) {
            int f = M.vf[a].a[t];
            const int *fv = &M.F[3 * f];
            if (fv[0] == b || fv[1] == b || fv[2] == b) { if (nfab < 4) fab[nfab] = f; nfab++; }
        }
        if (nfab == 0 || nfab > 2) { st.fails++; continue; }
        int bnd_a = is_boundary_vertex(&M, a), bnd_b = is_boundary_vertex(&M, b);
        int edge_bnd = (nfab == 1);
        if (mode == COLLAPSE_INTERIOR && (bnd_a || bnd_b)) { st.fails++; continue; }
        if (mode == COLLAPSE_STRAIGHT && !edge_bnd && (bnd_a || bnd_b)) { st.fails++; continue; }
        if (!edge_bnd && bnd_a && bnd_b) { st.fails++; continue; }
        /* link condition */
        int ida[256], cna[256], idb[256], cnb[256];
        int na = neighbours(&M, a, ida, cna, 256), nb = neighbours(&M, b, idb, cnb, 256);
        if (na < 0 || nb < 0) { st.fails++; continue; }
        int opp[2], nopp = 0;
        for (int t = 0; t < nfab; ++t) {
            const int *fv = &M.F[3 * fab[t]];
            for (int c = 0; c < 3; ++c) if (fv[c] != a && fv[c] != b) opp[nopp++] = fv[c];
        }
        int shared = 0, linkok = 1;
        for (int s = 0; s < na; ++s) {
            if (ida[s] == b) continue;
            for (int r = 0; r < nb; ++r)
                if (idb[r] == ida[s]) {
                    shared++;
                    int isopp = 0;
                    for (int t = 0; t < nopp; ++t) if (opp[t] == ida[s]) isopp = 1;
                    if (!isopp) linkok = 0;
                }
        }
        if (!linkok || shared != nopp) { st.fails++; continue; }
        int earok = 1;
        for (int t = 0; t < nopp; ++t) if (M.vf[opp[t]].n < 2) earok = 0;
        if (!earok) { st.fails++; continue; }

        /* label the endpoints */
        int i = a, j = b, kind;   /* kind: 0 interior, 1 one-boundary, 2 boundary edge */
        int p = -1, q = -1;
        if (edge_bnd) {
            kind = 2;
            const int *fv = &M.F[3 * fab[0]];
            for (int c = 0; c < 3; ++c)
                if (fv[c] == a && fv[(c + 1) % 3] == b) { i = a; j = b; }
                else if (fv[c] == b && fv[(c + 1) % 3] == a) { i = b; j = a; }
            p = other_boundary_neighbour(&M, i, j);
            q = other_boundary_neighbour(&M, j, i);
            if (p < 0 || q < 0 || p == q || p == j || q == i) { st.fails++; continue; }
            if (mode == COLLAPSE_STRAIGHT && !straight_run(&M, p, i, j, q)) { st.fails++; continue; }
        } else if (bnd_a || bnd_b) {
            kind = 1;
            if (bnd_a) { j = a; i = b; } else { i = a; j = b; }
        } else {
            kind = 0;
        }
        int k = M.nv;  /* id of the new vertex */
        if (k >= M.capv) { st.fails++; continue; }
        M.X[3 * k + 0] = 0.5 * (M.X[3 * i + 0] + M.X[3 * j + 0]);
        M.X[3 * k + 1] = 0.5 * (M.X[3 * i + 1] + M.X[3 * j + 1]);
        M.X[3 * k + 2] = 0.5 * (M.X[3 * i + 2] + M.X[3 * j + 2]);

        /* before faces: union of faces of i and j, ascending id */
        int fb[MAXF], nfb = 0, overflow = 0;
        for (int pass = 0; pass < 2; ++pass) {
            const ilist *L = &M.vf[pass ? j : i];
            for (int t = 0; t < L->n; ++t) {
                int f = L->a[t], dup = 0;
                for (int s = 0; s < nfb; ++s) if (fb[s] == f) dup = 1;
                if (dup) continue;
                if (nfb == MAXF) { overflow = 1; break; }
                fb[nfb++] = f;
            }
        }
        if (overflow) { st.fails++; continue; }
        for (int s = 1; s < nfb; ++s) { int v = fb[s], r = s - 1; while (r >= 0 && fb[r] > v) { fb[r + 1] = fb[r]; --r; } fb[r + 1] = v; }
        /* ring vertices ascending */
        int ring[MAXD], nr = 0;
        for (int s = 0; s < nfb; ++s)
            for (int c = 0; c < 3; ++c) {
                int w = M.F[3 * fb[s] + c], dup = 0;
                if (w == i || w == j) continue;
                for (int r = 0; r < nr; ++r) if (ring[r] == w) dup = 1;
                if (!dup) { if (nr == MAXD - 4) { overflow = 1; break; } ring[nr++] = w; }
            }
        if (overflow) { st.fails++; continue; }
        for (int s = 1; s < nr; ++s) { int v = ring[s], r = s - 1; while (r >= 0 && ring[r] > v) { ring[r + 1] = ring[r]; --r; } ring[r + 1] = v; }

        int ncase = (kind == 2) ? 3 : 1;
        int chosen = -1;
        double *rec = (probe && *probe_n < probe_cap) ? &probe[(size_t)(*probe_n) * PR_SIZE] : NULL;
        if (rec) {
            for (int s = 0; s < PR_SIZE; ++s) rec[s] = NAN;
            rec[0] = kind; rec[2] = i; rec[3] = j; rec[4] = p; rec[5] = q; rec[6] = k;
            rec[7] = nr; rec[8] = nfb; rec[9] = ncase;
            for (int s = 0; s < nr; ++s) rec[PR_RING + s] = ring[s];
            for (int s = 0; s < nfb; ++s)
                for (int c = 0; c < 3; ++c) rec[PR_FACE + 3 * s + c] = M.F[3 * fb[s] + c];
        }
        for (int cs = 0; cs < ncase; ++cs) {
            /* DOFs: ring 0..nr-1, i = nr, j = nr+1, k = nr+2 unless aliased */
            int di = nr, dj = nr + 1, dk;
            int nd;
            if (kind == 0) { dk = nr + 2; nd = nr + 3; }
            else if (kind == 1) { dk = dj; nd = nr + 2; }
            else if (cs == 0) { dk = di; nd = nr + 2; }
            else if (cs == 1) { dk = dj; nd = nr + 2; }
            else { dk = nr + 2; nd = nr + 3; }
            jp->nd = nd;
            jp->nfb = 0; jp->nfa = 0;
            for (int s = 0; s < nfb; ++s) {
                int f = fb[s];
                const int *fv = &M.F[3 * f];
                int hasi = 0, hasj = 0;
                for (int c = 0; c < 3; ++c) { if (fv[c] == i) hasi = 1; if (fv[c] == j) hasj = 1; }
                jp->fb_id[jp->nfb] = f;
                for (int c = 0; c < 3; ++c) {
                    int w = fv[c], d;
                    if (w == i) d = di; else if (w == j) d = dj;
                    else { d = 0; while (ring[d] != w) ++d; }
                    jp->fb_v[jp->nfb][c] = w;
                    jp->fb_d[jp->nfb][c] = d;
                }
                jp->nfb++;
                if (hasi && hasj) continue;  /* removed by the collapse */
                jp->fa_id[jp->nfa] = f;
                for (int c = 0; c < 3; ++c) {
                    int w = fv[c];
                    if (w == i || w == j) { jp->fa_v[jp->nfa][c] = k; jp->fa_d[jp->nfa][c] = dk; }
                    else { jp->fa_v[jp->nfa][c] = w; jp->fa_d[jp->nfa][c] = jp->fb_d[jp->nfb - 1][c]; }
                }
                jp->nfa++;
            }
            int fixed[2 * MAXD];
            double val[2 * MAXD];
            memset(fixed, 0, sizeof(int) * 2 * (size_t)nd);
            memset(val, 0, sizeof(double) * 2 * (size_t)nd);
            if (kind != 2) {
                /* gauge: the two ring vertices farthest apart in 3D */
                int pa = -1, pb = -1;
                double best = -1.0;
                for (int s = 0; s < nr; ++s)
                    for (int r = s + 1; r < nr; ++r) {
                        double d2 = len2(&M, ring[s], ring[r]);
                        if (d2 > best) { best = d2; pa = s; pb = r; }
                    }
                if (pa < 0) { chosen = -1; break; }
                double d = sqrt(best);
                fixed[2 * pa] = fixed[2 * pa + 1] = 1;
                fixed[2 * pb] = fixed[2 * pb + 1] = 1;
                val[2 * pb] = d;
                jp->scale = d;
            } else {
                int dp = 0, dq = 0;
                while (ring[dp] != p) ++dp;
                while (ring[dq] != q) ++dq;
                double lpi = dist3(&M, p, i), lij = dist3(&M, i, j), ljq = dist3(&M, j, q);
                int first, last;
                double span;
                if (cs == 0) {        /* k on i: i, j, q colinear */
                    fixed[2 * di + 1] = fixed[2 * dj + 1] = fixed[2 * dq + 1] = 1;
                    first = di; last = dq; span = lij + ljq;
                } else if (cs == 1) { /* k on j: p, i, j colinear */
                    fixed[2 * dp + 1] = fixed[2 * di + 1] = fixed[2 * dj + 1] = 1;
                    first = dp; last = dj; span = lpi + lij;
                } else {              /* k on line ij: p, i, k, j, q colinear */
                    fixed[2 * dp + 1] = fixed[2 * di + 1] = fixed[2 * dk + 1] = 1;
                    fixed[2 * dj + 1] = fixed[2 * dq + 1] = 1;
                    first = dp; last = dq; span = lpi + lij + ljq;
                }
                fixed[2 * first] = 1; val[2 * first] = 0.0;
                fixed[2 * last] = 1; val[2 * last] = span;
                jp->scale = span;
            }
            int rc = joint_solve(&M, jp, fixed, val);
            if (rec) {
                double *cr = &rec[PR_CASE0 + cs * PR_CASE_SIZE];
                cr[0] = rc;
                cr[1] = jp->energy;
                for (int s = 0; s < nr; ++s) { cr[2 + 2 * s] = jp->U[s][0]; cr[3 + 2 * s] = jp->U[s][1]; }
                double *tail = &cr[2 + 2 * MAXD];
                tail[0] = jp->U[di][0]; tail[1] = jp->U[di][1];
                tail[2] = jp->U[dj][0]; tail[3] = jp->U[dj][1];
                tail[4] = jp->U[dk][0]; tail[5] = jp->U[dk][1];
            }
            if (rc != 0) continue;
            if (chosen < 0 || jp->energy < jbest->energy) {
                chosen = cs;
                memcpy(jbest, jp, sizeof(jpatch));
            }
        }
        if (chosen < 0) { st.fails++; continue; }

        /* ---- commit: carry query points through the shared UV domain ---- */
        double max_clamp = st.max_clamp;
        int nmoved = 0;
        for (int s = 0; s < jbest->nfb; ++s) {
            int f = jbest->fb_id[s];
            for (int pt = fhead[f]; pt >= 0; pt = qnext[pt]) {
                double uv[2] = {0.0, 0.0};
                for (int c = 0; c < 3; ++c) {
                    /* slot c of qbar follows the face's current vertex order */
                    const double *U = jbest->U[jbest->fb_d[s][c]];
                    uv[0] += qbar[3 * pt + c] * U[0];
                    uv[1] += qbar[3 * pt + c] * U[1];
                }
                int bestf = -1;
                double bestmin = -INFINITY, bb[3] = {0, 0, 0};
                for (int r = 0; r < jbest->nfa; ++r) {
                    const double *U0 = jbest->U[jbest->fa_d[r][0]];
                    const double *U1 = jbest->U[jbest->fa_d[r][1]];
                    const double *U2 = jbest->U[jbest->fa_d[r][2]];
                    double A = tri_area2(U0, U1, U2);
                    double l0 = tri_area2(uv, U1, U2) / A;
                    double l1 = tri_area2(U0, uv, U2) / A;
                    double l2 = tri_area2(U0, U1, uv) / A;
                    double mn = fmin(l0, fmin(l1, l2));
                    if (bestf < 0 || mn > bestmin || (mn == bestmin && jbest->fa_id[r] < jbest->fa_id[bestf])) {
                        bestmin = mn; bestf = r; bb[0] = l0; bb[1] = l1; bb[2] = l2;
                    }
                }
                double sum = 0.0;
                for (int c = 0; c < 3; ++c) {
                    if (bb[c] < 0.0) { if (-bb[c] > max_clamp) max_clamp = -bb[c]; bb[c] = 0.0; }
                    sum += bb[c];
                }
                for (int c = 0; c < 3; ++c) qbar[3 * pt + c] = bb[c] / sum;
                qface[pt] = jbest->fa_id[bestf];
                moved[nmoved++] = pt;
            }
            fhead[f] = -1;
        }
        st.max_clamp = max_clamp;
        for (int s = 0; s < nmoved; ++s) {
            int pt = moved[s];
            qnext[pt] = fhead[qface[pt]];
            fhead[qface[pt]] = pt;
        }
        /* topology update: faces keep their ids, i and j become k */
        for (int s = 0; s < jbest->nfb; ++s) {
            int f = jbest->fb_id[s];
            int kept = -1;
            for (int r = 0; r < jbest->nfa; ++r) if (jbest->fa_id[r] == f) kept = r;
            if (kept >= 0) {
                for (int c = 0; c < 3; ++c) M.F[3 * f + c] = jbest->fa_v[kept][c];
            } else {
                M.falive[f] = 0;
                for (int c = 0; c < 3; ++c) {
                    ilist *L = &M.vf[jbest->fb_v[s][c]];
                    for (int t = 0; t < L->n; ++t) if (L->a[t] == f) { L->a[t] = L->a[--L->n]; break; }
                }
            }
        }
        M.valive[i] = M.valive[j] = 0;
        M.vf[i].n = 0;
        M.vf[j].n = 0;
        M.valive[k] = 1;
        for (int r = 0; r < jbest->nfa; ++r) il_push(&M.vf[k], jbest->fa_id[r]);
        M.nv++;
        alive--;
        st.collapses++;
        if (rec) { rec[1] = chosen; (*probe_n)++; }
        if (kind == 0) st.case_int++;
        else if (kind == 1) st.case_one++;
        else if (chosen == 0) st.case_b1++;
        else if (chosen == 1) st.case_b2++;
        else st.case_b3++;
        /* re-enable / re-key every edge with an endpoint in the new 1-ring of k */
        int nbk[256], cnk[256];
        int nk = neighbours(&M, k, nbk, cnk, 256);
        for (int s = -1; s < nk; ++s) {
            int x = (s < 0) ? k : nbk[s];
            int nbx[256], cnx[256];
            int nx = neighbours(&M, x, nbx, cnx, 256);
            for (int r = 0; r < nx; ++r) {
                int y = nbx[r];
                hent ne = {len2(&M, x, y), x < y ? x : y, x < y ? y : x};
                h_push(&H, ne);
            }
        }
    }

    /* ---- outputs: compact coarse ids in ascending old id ---- */
    int *newid = (int *)malloc(sizeof(int) * (size_t)M.nv);
    int cnt = 0;
    for (int v = 0; v < M.nv; ++v) {
        newid[v] = -1;
        if (M.valive[v]) {
            newid[v] = cnt;
            for (int c = 0; c < 3; ++c) Xc[3 * cnt + c] = M.X[3 * v + c];
            cnt++;
        }
    }
    *nc = cnt;
    int fc = 0;
    for (int f = 0; f < m; ++f) {
        if (!M.falive[f]) continue;
        for (int c = 0; c < 3; ++c) Fc[3 * fc + c] = newid[M.F[3 * f + c]];
        fc++;
    }
    *mc = fc;
    for (int v = 0; v < n; ++v) {
        int f = qface[v];
        double w[3], sum = 0.0;
        for (int c = 0; c < 3; ++c) { w[c] = qbar[3 * v + c] < 1e-12 ? 0.0 : qbar[3 * v + c]; sum += w[c]; }
        for (int c = 0; c < 3; ++c) {
            Pw[3 * v + c] = w[c] / sum;
            Pc[3 * v + c] = (w[c] > 0.0) ? newid[M.F[3 * f + c]] : -1;
        }
    }
    if (stats_out) {
        stats_out[0] = (double)st.collapses; stats_out[1] = (double)st.fails;
        stats_out[2] = (double)st.case_int; stats_out[3] = (double)st.case_one;
        stats_out[4] = (double)st.case_b1; stats_out[5] = (double)st.case_b2;
        stats_out[6] = (double)st.case_b3; stats_out[7] = st.max_clamp;
    }
    if (Xall) memcpy(Xall, M.X, sizeof(double) * 3 * (size_t)M.nv);
    free(newid); free(moved);
    free(jp); free(jbest);
    free(H.e);
    free(qface); free(qbar); free(fhead); free(qnext);
    for (int v = 0; v < M.capv; ++v) free(M.vf[v].a);
    free(M.vf); free(M.X); free(M.valive); free(M.F); free(M.falive);
    return 0;
}

int oracle_ssp_level(int n, const double *X, int m, const int *F, int target, int mode,
                     int *nc, double *Xc, int *mc, int *Fc, int *Pc, double *Pw, double *stats_out) {
    return oracle_ssp_level_probe(n, X, m, F, target, mode, nc, Xc, mc, Fc, Pc, Pw, stats_out,
                                  NULL, 0, NULL, NULL);
}
