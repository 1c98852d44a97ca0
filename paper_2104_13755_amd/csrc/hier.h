// Host-side data structures of the surface-multigrid library.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace smg {

// One decimation level produced by the successive self-parameterization.
struct LevelOut {
    std::vector<double> X;        // coarse positions, 3 per vertex
    std::vector<int32_t> F;       // coarse triangles, 3 per face
    std::vector<int32_t> pcols;   // fine vertex -> 3 coarse columns (-1 unused)
    std::vector<double> pw;       // matching barycentric weights (0 unused)
    double stats[8];
};

// collapses: 0 every edge, 1 edges with both endpoints interior, 2 those plus
// boundary edges on straight boundary runs (no one-boundary collapse).
int ssp_decimate_level(const std::vector<double> &X, const std::vector<int32_t> &F, int target,
                       int collapses, LevelOut &out);

// Greedy coloring of a CSR pattern's off-diagonal graph (Alg. "Graph Coloring").
int greedy_coloring(int n, const int32_t *rowptr, const int32_t *cols, std::vector<int32_t> &color);

// Plain CSR pattern (+ optional values).
struct Csr {
    int n = 0, m = 0;
    std::vector<int32_t> ptr, idx;
};

// Symbolic Galerkin pattern of P^T A P (rows/cols in natural coarse numbering,
// ascending columns).  P given row-wise as ELL-3 (col < 0 unused).
Csr galerkin_pattern(const Csr &A, int nc, const std::vector<int32_t> &pcols);

// Sliced-ELL layout of the off-diagonal part of a level whose rows are
// permuted color-major.  A slice is one wavefront: 64 / lpr rows, each row
// spread over lpr adjacent lanes (entry e of a row sits in lane e % lpr of its
// group, element e / lpr), elements stored column-major (64 slots apart).
struct SellLayout {
    int n = 0;                       // rows
    int lpr = 1;                     // lanes per row (1, 2, 4 or 8)
    int nslices = 0;
    std::vector<int32_t> slice_row0; // first permuted row of each slice
    std::vector<int32_t> slice_off;  // nslices + 1 element offsets (multiples of 64)
    std::vector<int32_t> cols;       // permuted column per slot (padding: own row)
    std::vector<int32_t> rowlen;     // off-diagonal entries per permuted row
    std::vector<int32_t> color_row;  // ncolors + 1 row boundaries (permuted)
    std::vector<int32_t> color_slice;// ncolors + 1 slice boundaries
    std::vector<int32_t> color_w;    // per color: rounds of every slice, 0 = per-slice widths
    std::vector<int32_t> row_slice;  // slice index of each permuted row
    std::vector<int32_t> pptr, pidx; // permuted rows' off-diagonal columns, ascending
    int64_t slots() const { return slice_off.empty() ? 0 : slice_off.back(); }
    // slot of the e-th off-diagonal entry of permuted row r
    int32_t slot(int r, int e) const {
        const int s = row_slice[r];
        return slice_off[s] + (e / lpr) * 64 + (r - slice_row0[s]) * lpr + (e % lpr);
    }
};

// Everything the device needs for one level, built on the host.
struct LevelHost {
    int n = 0;
    bool coarsest = false;
    Csr pat;                         // natural-order pattern of A_l (with diagonal)
    std::vector<int32_t> color;      // natural index -> color (smoothed levels)
    int ncolors = 0;
    std::vector<int32_t> perm;       // permuted position -> natural index
    std::vector<int32_t> iperm;      // natural index -> permuted position
    SellLayout sell;
    // natural CSR entry -> storage position: >= 0 SELL slot, < 0 -> diag of
    // permuted row (-1 - r).  On the coarsest level: dense column-major index.
    std::vector<int32_t> store;
    // prolongation to the next level, permuted both ways, SoA ELL-3
    std::vector<int32_t> pc;         // 3 * n (slot m at m*n + r)
    std::vector<double> pw;
    // restriction R = P^T, CSR over permuted coarse rows
    std::vector<int32_t> rptr, ridx;
    std::vector<double> rw;
    // the same R as sliced ELL with rs_lanes lanes per coarse row: 64 /
    // rs_lanes rows per slice, entry e of row a (slice s, g = a % rows per
    // slice) at rs_off[s] + 64 (e / rs_lanes) + g rs_lanes + e % rs_lanes
    // (padding: index of the row's first entry or 0, weight 0)
    int rs_lanes = 4;
    std::vector<int32_t> rs_off, rs_idx;
    std::vector<double> rs_w;
    // Galerkin plan to the next level: T = A P, then A_next = P^T T.  Each row
    // of T and of A_next is accumulated in its own local slots (a row owner
    // adds its contributions in a fixed order, so results are deterministic).
    std::vector<int32_t> tptr;       // n + 1
    std::vector<int32_t> plan1ptr;   // n + 1 (3 per source entry: diag + rowlen)
    std::vector<uint16_t> plan1;     // offset within the T row
    int tmax = 0;                    // longest T row
    std::vector<int32_t> plan2ptr;   // n_next + 1
    std::vector<uint16_t> plan2;     // local slot within the coarse row
    std::vector<int32_t> optr;       // n_next + 1: local slots of each coarse row
    std::vector<int32_t> opos;       // local slot -> storage position in level l+1 (see `store`)
    int cmax = 0;                    // most local slots of a coarse row
};

// Record layout of one smoothed level for the one-workgroup tail kernel,
// whose iterate lives in LDS.  Rows of a color are processed in passes of
// `threads / grp` rows, each row by `grp` adjacent lanes (thread t of a pass:
// row row0 + t / grp).  Each wavefront w of a pass reads its own rounds of
// records in pairs, record (k, lane) at wave offset + 128 (k / 2) + 2 lane +
// k % 2 (a lane's two records of a pair are adjacent: one 16-byte load in
// FP32), holding entry k * grp + t % grp of the thread's row (padding: column
// 0, weight 0).  The
// restriction into the next level is an ELL of width rk, entry k of coarse row
// a at k * nc + a (padding: index 0, weight 0).
struct TailLayout {
    int grp = 1;
    std::vector<int32_t> pass;    // 4 per pass: row0, nrows, (last of its color) << 16, first wave
    std::vector<int32_t> wave;    // 2 per wavefront: record offset, pairs of rounds
    std::vector<int32_t> src;     // record -> SELL slot of the level (-1 padding)
    std::vector<int32_t> cols;    // record -> permuted column
    int rk = 0, nc = 0;
    std::vector<int32_t> ridx;    // rk * nc
    std::vector<double> rw;
};
// threads: workgroup size of the tail kernel; nc: rows of the next level;
// grp > 0 forces the lanes per row (else the widest group up to 4 that fits
// a whole color in one pass).
void build_tail_layout(const LevelHost &L, int nc, int threads, int grp, TailLayout &out);
// Bounds of every index the tail kernel derives from a layout of a level with
// n rows (records, pass rows, restriction); false + message if one is out.
bool check_tail_layout(const TailLayout &T, int n, int threads, std::string &err);

struct HierHost {
    int nlev = 0;
    std::vector<int> sizes;
    std::vector<std::vector<double>> X;        // vertex positions per level (3 each) when known
    std::vector<std::vector<int32_t>> pcols;   // natural ELL-3 per level
    std::vector<std::vector<double>> pw;
    std::vector<std::array<double, 8>> stats;
};

// Cotangent Laplacian values and lumped mass on a CSR pattern that holds the
// diagonal and every mesh edge (assemble_host.cpp); false + message on a
// degenerate face or a pattern without an edge of a face.
bool host_assemble(const double *V, int n, const int32_t *F, int m, const int32_t *rowptr, const int32_t *cols,
                   double *L, double *M, std::string &err);

// Versioned binary file of a hierarchy (hier_io.cpp); false + message on an
// I/O error or a malformed file.
bool hier_write(const HierHost &H, const char *path, std::string &err);
bool hier_read(const char *path, HierHost &H, std::string &err);

// Lanes per row for a level whose rows average `avg` off-diagonal entries.
int default_lanes_per_row(double avg);

// Build every LevelHost from the level-0 pattern and the prolongations.
// lpr[l] > 0 forces the lanes per row of level l (else the default rule).
// Inside a color, rows of Galerkin levels with at most sort_rows rows are
// ordered by descending length (the one-workgroup tail reads them by
// wavefront); all other levels follow a Morton curve through the vertex
// positions when H.X holds them (neighbours' iterates then share cache
// lines), else the natural order.
int build_levels(const HierHost &H, const Csr &A0, const std::vector<int> &lpr, int sort_rows,
                 std::vector<LevelHost> &levels, std::string &err);

}  // namespace smg
