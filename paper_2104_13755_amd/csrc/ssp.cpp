// Host precompute: intrinsic prolongation by successive self-parameterization.
//
// Implements the hierarchy construction of "Surface Multigrid via Intrinsic
// Prolongation": mid-point edge collapses (Sec. 4.4), each followed by the
// joint flattening of the edge 1-ring before and the vertex 1-ring after the
// collapse into one shared UV domain (Sec. 4.2, Eq. jointEnergy) with the LSCM
// energy (Sec. 4.4), the boundary-edge cases of Sec. 4.3, and the online
// barycentric query of App. C / Fig. baryQuery that carries every fine vertex
// through the collapses of its level.  The result per level is the
// prolongation P_l whose rows hold the barycentric coordinates of a fine
// vertex in its coarse triangle (Sec. 4.5).
//
// The paper leaves several choices open; this file takes these readings:
//   * priority = squared 3D edge length, smallest first, ties by (lo, hi) id;
//     an edge that fails a test is retried only after a later collapse puts
//     one of its endpoints into the new 1-ring;
//   * a collapse is valid iff the link condition holds, it does not join two
//     boundary vertices through an interior edge, no opposite vertex loses its
//     last face, the LSCM system is non-singular, and every UV triangle of both
//     patches has signed area > 1e-12 scale^2;
//   * gauge for interior and one-boundary collapses: the two ring vertices
//     farthest apart in 3D are pinned at (0,0) and (d,0); boundary-edge
//     collapses (three cases, Fig. jointVar_case2) put their colinear vertices
//     on v = 0 and pin u of the first and last colinear vertex to 0 and to the
//     3D length of the boundary chain between them; the valid case of least
//     energy wins (ties: lower case number);
//   * query: the after-patch triangle with the largest minimum barycentric
//     coordinate (ties: lowest triangle id), negatives clamped to 0 and
//     renormalized; final weights below 1e-12 dropped and renormalized.
// Arithmetic that decides integers (priorities, thresholds) is written
// without contraction; the library is built with -ffp-contract=off.

#include "hier.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <limits>
#include <unordered_set>
#include <vector>

namespace smg {
namespace {

struct Surface {
    std::vector<double> X;                 // 3 per vertex (grows by one per collapse)
    std::vector<std::array<int, 3>> tri;   // triangle corners, updated in place
    std::vector<uint8_t> tri_alive, vert_alive;
    std::vector<std::vector<int>> star;    // vertex -> alive incident triangles

    double sqdist(int a, int b) const {
        const double dx = X[3 * a] - X[3 * b];
        const double dy = X[3 * a + 1] - X[3 * b + 1];
        const double dz = X[3 * a + 2] - X[3 * b + 2];
        return dx * dx + dy * dy + dz * dz;
    }
    // a, b, c, d in this order on one straight line: the polyline is as long
    // as the segment from a to d (to 1e-12 relative; a bend by an angle t
    // lengthens it by about t^2 / 2 of the shorter side)
    bool on_one_line(int a, int b, int c, int d) const {
        const double chain = std::sqrt(sqdist(a, b)) + std::sqrt(sqdist(b, c)) + std::sqrt(sqdist(c, d));
        return chain - std::sqrt(sqdist(a, d)) <= 1e-12 * chain;
    }
    // neighbour -> number of incident triangles shared with v
    void link(int v, std::vector<std::pair<int, int>> &out) const {
        out.clear();
        for (int t : star[v])
            for (int c = 0; c < 3; ++c) {
                const int w = tri[t][c];
                if (w == v) continue;
                bool found = false;
                for (auto &pr : out)
                    if (pr.first == w) { pr.second++; found = true; break; }
                if (!found) out.push_back({w, 1});
            }
    }
};

struct Cand {
    double key;
    int lo, hi;
};
struct CandAfter {   // a comes after b in the collapse order
    bool operator()(const Cand &a, const Cand &b) const {
        if (a.key != b.key) return a.key > b.key;
        if (a.lo != b.lo) return a.lo > b.lo;
        return a.hi > b.hi;
    }
};

// Min-heap with four children per node (fewer levels, children in one cache line).
class Heap4 {
  public:
    bool empty() const { return h_.empty(); }
    const Cand &top() const { return h_[0]; }
    void push(const Cand &c) {
        size_t i = h_.size();
        h_.push_back(c);
        while (i > 0) {
            const size_t p = (i - 1) / 4;
            if (!CandAfter()(h_[p], c)) break;
            h_[i] = h_[p];
            i = p;
        }
        h_[i] = c;
    }
    void pop() {
        const Cand last = h_.back();
        h_.pop_back();
        const size_t n = h_.size();
        if (n == 0) return;
        size_t i = 0;
        for (;;) {
            const size_t c0 = 4 * i + 1;
            if (c0 >= n) break;
            size_t m = c0;
            const size_t ce = std::min(n, c0 + 4);
            for (size_t c = c0 + 1; c < ce; ++c) if (CandAfter()(h_[m], h_[c])) m = c;
            if (!CandAfter()(last, h_[m])) break;
            h_[i] = h_[m];
            i = m;
        }
        h_[i] = last;
    }
  private:
    std::vector<Cand> h_;
};

// One patch pair sharing a joint UV variable.
struct Joint {
    int ndof = 0;
    std::vector<int> before_id, after_id;                 // triangle ids
    std::vector<std::array<int, 3>> before_v, after_v;    // vertex ids (after: i,j -> k)
    std::vector<std::array<int, 3>> before_d, after_d;    // joint DOF per corner
    std::vector<std::array<double, 2>> uv;                // per DOF
    double energy = 0.0, scale = 1.0;
};

// Conformal-energy rows of one triangle in its own orthonormal frame:
// coefficient of (u_c, v_c) in Re and Im of (sum_c W_c U_c)/(2 sqrt(area)),
// W_c = (x_{c+2} - x_{c+1}) + i (y_{c+2} - y_{c+1}).
static bool conformal_rows(const double *p0, const double *p1, const double *p2,
                           double re[6], double im[6]) {
    const double ax = p1[0] - p0[0], ay = p1[1] - p0[1], az = p1[2] - p0[2];
    const double bx = p2[0] - p0[0], by = p2[1] - p0[1], bz = p2[2] - p0[2];
    const double la = std::sqrt(ax * ax + ay * ay + az * az);
    const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const double nn = std::sqrt(nx * nx + ny * ny + nz * nz);
    if (!(la > 0.0) || !(nn > 0.0)) return false;
    const double lx[3] = {0.0, la, (ax * bx + ay * by + az * bz) / la};
    const double ly[3] = {0.0, 0.0, nn / la};
    const double inv = 1.0 / (2.0 * std::sqrt(0.5 * nn));
    for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        const double wr = (lx[c2] - lx[c1]) * inv, wi = (ly[c2] - ly[c1]) * inv;
        re[2 * c] = wr;  re[2 * c + 1] = -wi;
        im[2 * c] = wi;  im[2 * c + 1] = wr;
    }
    return true;
}

static inline double orient2(const double *a, const double *b, const double *c) {
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

// Buffers of flatten(), reused across collapses.
struct FlatWork {
    std::vector<int> slot;
    std::vector<double> N, g;
    std::vector<std::array<double, 12>> rows;   // conformal rows (re, im) per triangle, in accumulation order
};

// Minimise the summed conformal energy of both patches with some coordinates
// fixed.  Normal equations N z_free = -J_free^T J_fixed z_fixed, solved by a
// dense Cholesky factorisation.
static bool flatten(const Surface &S, Joint &J, const std::vector<int> &fixed,
                    const std::vector<double> &fixval, FlatWork &w) {
    const int ncol = 2 * J.ndof;
    std::vector<int> &slot = w.slot;
    slot.assign(ncol, -1);
    int nfree = 0;
    for (int c = 0; c < ncol; ++c) if (!fixed[c]) slot[c] = nfree++;
    std::vector<double> &N = w.N, &g = w.g;
    N.assign((size_t)nfree * nfree, 0.0);
    g.assign(nfree, 0.0);
    w.rows.clear();
    auto accumulate = [&](const std::array<int, 3> &v, const std::array<int, 3> &d) -> bool {
        w.rows.emplace_back();
        double *re = w.rows.back().data(), *im = re + 6;
        if (!conformal_rows(&S.X[3 * v[0]], &S.X[3 * v[1]], &S.X[3 * v[2]], re, im)) return false;
        int col[6];
        for (int c = 0; c < 3; ++c) { col[2 * c] = 2 * d[c]; col[2 * c + 1] = 2 * d[c] + 1; }
        for (const double *row : {re, im}) {
            double known = 0.0;
            for (int a = 0; a < 6; ++a) if (fixed[col[a]]) known += row[a] * fixval[col[a]];
            for (int a = 0; a < 6; ++a) {
                const int sa = slot[col[a]];
                if (sa < 0) continue;
                g[sa] -= row[a] * known;
                for (int b = 0; b < 6; ++b) {
                    const int sb = slot[col[b]];
                    if (sb >= 0) N[(size_t)sa * nfree + sb] += row[a] * row[b];
                }
            }
        }
        return true;
    };
    for (size_t t = 0; t < J.before_v.size(); ++t) if (!accumulate(J.before_v[t], J.before_d[t])) return false;
    for (size_t t = 0; t < J.after_v.size(); ++t) if (!accumulate(J.after_v[t], J.after_d[t])) return false;
    // Cholesky N = C C^T (lower, in place), then two triangular solves
    double nmax = 0.0;
    for (int a = 0; a < nfree; ++a) nmax = std::max(nmax, N[(size_t)a * nfree + a]);
    for (int a = 0; a < nfree; ++a) {
        double diag = N[(size_t)a * nfree + a];
        for (int q = 0; q < a; ++q) diag -= N[(size_t)a * nfree + q] * N[(size_t)a * nfree + q];
        if (!(diag > 1e-14 * nmax)) return false;
        const double c = std::sqrt(diag);
        N[(size_t)a * nfree + a] = c;
        for (int b = a + 1; b < nfree; ++b) {
            double s = N[(size_t)b * nfree + a];
            for (int q = 0; q < a; ++q) s -= N[(size_t)b * nfree + q] * N[(size_t)a * nfree + q];
            N[(size_t)b * nfree + a] = s / c;
        }
    }
    for (int a = 0; a < nfree; ++a) {
        double s = g[a];
        for (int q = 0; q < a; ++q) s -= N[(size_t)a * nfree + q] * g[q];
        g[a] = s / N[(size_t)a * nfree + a];
    }
    for (int a = nfree - 1; a >= 0; --a) {
        double s = g[a];
        for (int q = a + 1; q < nfree; ++q) s -= N[(size_t)q * nfree + a] * g[q];
        g[a] = s / N[(size_t)a * nfree + a];
    }
    J.uv.assign(J.ndof, {0.0, 0.0});
    for (int c = 0; c < ncol; ++c) J.uv[c / 2][c % 2] = fixed[c] ? fixval[c] : g[slot[c]];
    // energy of the solution, and the orientation test of every UV triangle
    double e = 0.0;
    size_t tri = 0;
    auto add_energy = [&](const std::array<int, 3> &d) {
        const double *re = w.rows[tri].data(), *im = re + 6;
        ++tri;
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < 3; ++c) {
            sr += re[2 * c] * J.uv[d[c]][0] + re[2 * c + 1] * J.uv[d[c]][1];
            si += im[2 * c] * J.uv[d[c]][0] + im[2 * c + 1] * J.uv[d[c]][1];
        }
        e += sr * sr + si * si;
    };
    for (size_t t = 0; t < J.before_v.size(); ++t) add_energy(J.before_d[t]);
    for (size_t t = 0; t < J.after_v.size(); ++t) add_energy(J.after_d[t]);
    J.energy = e;
    const double min_area = 1e-12 * J.scale * J.scale;
    for (const auto *dl : {&J.before_d, &J.after_d})
        for (const auto &d : *dl)
            if (!(0.5 * orient2(J.uv[d[0]].data(), J.uv[d[1]].data(), J.uv[d[2]].data()) > min_area))
                return false;
    return true;
}

}  // namespace

int ssp_decimate_level(const std::vector<double> &Xin, const std::vector<int32_t> &Fin, int target,
                       int collapses, LevelOut &out) {
    const int n = (int)(Xin.size() / 3);
    const int m = (int)(Fin.size() / 3);
    Surface S;
    S.X = Xin;
    S.X.reserve(3 * (size_t)(2 * n + 8));
    S.tri.resize(m);
    S.tri_alive.assign(m, 1);
    S.vert_alive.assign(n, 1);
    S.star.assign(n, {});
    for (int t = 0; t < m; ++t) {
        for (int c = 0; c < 3; ++c) {
            const int v = Fin[3 * t + c];
            if (v < 0 || v >= n) return -1;
            S.tri[t][c] = v;
            S.star[v].push_back(t);
        }
    }
    // each fine vertex starts in its lowest-id triangle with a one-hot weight
    std::vector<int> where(n);
    std::vector<std::array<double, 3>> bary(n);
    std::vector<std::vector<int>> bucket(m);
    for (int v = 0; v < n; ++v) {
        if (S.star[v].empty()) return -2;   // isolated vertex
        const int t = *std::min_element(S.star[v].begin(), S.star[v].end());
        where[v] = t;
        for (int c = 0; c < 3; ++c) bary[v][c] = S.tri[t][c] == v ? 1.0 : 0.0;
        bucket[t].push_back(v);
    }
    // Candidates in priority order.  An edge of the input keeps its length
    // for the whole level (a collapse creates a new vertex id), so the input
    // edges are sorted once and read in order; edges created by collapses and
    // re-enabled edges go through a heap, and each pop takes the smaller head
    // of the two under the same total order.
    std::vector<Cand> init;
    init.reserve(3 * (size_t)m);
    for (int t = 0; t < m; ++t)
        for (int c = 0; c < 3; ++c) {
            const int a = S.tri[t][c], b = S.tri[t][(c + 1) % 3];
            init.push_back({S.sqdist(a, b), std::min(a, b), std::max(a, b)});
        }
    std::sort(init.begin(), init.end(), [](const Cand &x, const Cand &y) { return CandAfter()(y, x); });
    init.erase(std::unique(init.begin(), init.end(),
                           [](const Cand &x, const Cand &y) { return x.lo == y.lo && x.hi == y.hi; }),
               init.end());
    size_t cursor = 0;
    Heap4 pq;
    auto next_cand = [&](Cand &out) {
        const bool from_init = cursor < init.size() && (pq.empty() || CandAfter()(pq.top(), init[cursor]));
        if (from_init) {
            out = init[cursor++];
        } else {
            if (pq.empty()) return false;
            out = pq.top();
            pq.pop();
        }
        return true;
    };

    double st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int alive = n;
    // Edges that failed a validity test.  They leave the queue and come back
    // only when a collapse changes their neighbourhood; every other edge keeps
    // its single queue entry (its length never changes: new vertices get new
    // ids), so re-inserting it would only add an equal-key duplicate.
    // nfailed[v] counts the failed edges at v, so the re-enable scan skips
    // vertices that have none.
    std::unordered_set<uint64_t> failed;
    std::vector<int> nfailed(n, 0);
    auto ekey = [](int lo, int hi) { return ((uint64_t)(uint32_t)lo << 32) | (uint32_t)hi; };
    auto fail_edge = [&](int lo, int hi) {
        if (failed.insert(ekey(lo, hi)).second) { nfailed[lo]++; nfailed[hi]++; }
        st[1]++;
    };
    std::vector<std::pair<int, int> > la, lb;
    std::vector<int> before, ring, moved, opp, opps, na, nb, common, fixed;
    std::vector<double> val;
    FlatWork work;
    struct AfterTri { const double *A, *B, *C; double area; };
    std::vector<AfterTri> after_uv;   // corners and signed area of each after triangle
    Joint cur, best;
    Cand cd;
    while (alive > target && next_cand(cd)) {
        const int a = cd.lo, b = cd.hi;
        if (!S.vert_alive[a] || !S.vert_alive[b]) continue;
        int shared_tris[3], nshared = 0;
        for (int t : S.star[a]) {
            const auto &f = S.tri[t];
            if (f[0] == b || f[1] == b || f[2] == b) { if (nshared < 3) shared_tris[nshared] = t; ++nshared; }
        }
        if (nshared < 1 || nshared > 2) { fail_edge(a, b); continue; }
        // a vertex is on the boundary iff an edge at it has one triangle
        S.link(a, la);
        S.link(b, lb);
        auto boundary_of = [](const std::vector<std::pair<int, int> > &l) {
            for (auto &pr : l) if (pr.second == 1) return true;
            return false;
        };
        const bool ba = boundary_of(la), bb = boundary_of(lb);
        const bool boundary_edge = nshared == 1;
        if (collapses == 1 && (ba || bb)) { fail_edge(a, b); continue; }
        if (collapses == 2 && !boundary_edge && (ba || bb)) { fail_edge(a, b); continue; }
        if (!boundary_edge && ba && bb) { fail_edge(a, b); continue; }
        // link condition: common neighbours == opposite corners of the shared triangles
        opp.clear();
        for (int q = 0; q < nshared; ++q)
            for (int c = 0; c < 3; ++c) {
                const int w = S.tri[shared_tris[q]][c];
                if (w != a && w != b) opp.push_back(w);
            }
        na.clear();
        nb.clear();
        common.clear();
        for (auto &pr : la) if (pr.first != b) na.push_back(pr.first);
        for (auto &pr : lb) if (pr.first != a) nb.push_back(pr.first);
        std::sort(na.begin(), na.end());
        std::sort(nb.begin(), nb.end());
        std::set_intersection(na.begin(), na.end(), nb.begin(), nb.end(), std::back_inserter(common));
        opps = opp;
        std::sort(opps.begin(), opps.end());
        if (common != opps) { fail_edge(a, b); continue; }
        bool ear = false;
        for (int o : opp) if (S.star[o].size() < 2) ear = true;
        if (ear) { fail_edge(a, b); continue; }

        int i = a, j = b, kind = 0, p = -1, q = -1;
        if (boundary_edge) {
            kind = 2;
            const auto &f = S.tri[shared_tris[0]];
            for (int c = 0; c < 3; ++c) {
                if (f[c] == a && f[(c + 1) % 3] == b) { i = a; j = b; }
                else if (f[c] == b && f[(c + 1) % 3] == a) { i = b; j = a; }
            }
            auto boundary_neighbour_except = [](const std::vector<std::pair<int, int> > &l, int other) {
                for (auto &pr : l) if (pr.second == 1 && pr.first != other) return pr.first;
                return -1;
            };
            p = boundary_neighbour_except(i == a ? la : lb, j);
            q = boundary_neighbour_except(j == a ? la : lb, i);
            if (p < 0 || q < 0 || p == q || p == j || q == i) { fail_edge(a, b); continue; }
            if (collapses == 2 && !S.on_one_line(p, i, j, q)) { fail_edge(a, b); continue; }
        } else if (ba || bb) {
            kind = 1;
            if (ba) { j = a; i = b; } else { i = a; j = b; }
        }
        const int k = (int)(S.X.size() / 3);
        // patches
        before.clear();
        for (int t : S.star[i]) before.push_back(t);
        for (int t : S.star[j]) before.push_back(t);
        std::sort(before.begin(), before.end());
        before.erase(std::unique(before.begin(), before.end()), before.end());
        ring.clear();
        for (int t : before)
            for (int c = 0; c < 3; ++c) {
                const int w = S.tri[t][c];
                if (w != i && w != j) ring.push_back(w);
            }
        std::sort(ring.begin(), ring.end());
        ring.erase(std::unique(ring.begin(), ring.end()), ring.end());
        const int nr = (int)ring.size();
        auto ring_dof = [&](int w) { return (int)(std::lower_bound(ring.begin(), ring.end(), w) - ring.begin()); };
        const double kx = 0.5 * (S.X[3 * i] + S.X[3 * j]);
        const double ky = 0.5 * (S.X[3 * i + 1] + S.X[3 * j + 1]);
        const double kz = 0.5 * (S.X[3 * i + 2] + S.X[3 * j + 2]);
        S.X.push_back(kx); S.X.push_back(ky); S.X.push_back(kz);

        const int ncases = kind == 2 ? 3 : 1;
        int chosen = -1;
        for (int cs = 0; cs < ncases; ++cs) {
            const int di = nr, dj = nr + 1;
            int dk;
            if (kind == 0) { dk = nr + 2; cur.ndof = nr + 3; }
            else if (kind == 1) { dk = dj; cur.ndof = nr + 2; }
            else if (cs == 0) { dk = di; cur.ndof = nr + 2; }
            else if (cs == 1) { dk = dj; cur.ndof = nr + 2; }
            else { dk = nr + 2; cur.ndof = nr + 3; }
            cur.before_id.clear(); cur.before_v.clear(); cur.before_d.clear();
            cur.after_id.clear(); cur.after_v.clear(); cur.after_d.clear();
            for (int t : before) {
                const auto f = S.tri[t];
                std::array<int, 3> d{}, av{}, ad{};
                bool has_i = false, has_j = false;
                for (int c = 0; c < 3; ++c) {
                    if (f[c] == i) { d[c] = di; has_i = true; }
                    else if (f[c] == j) { d[c] = dj; has_j = true; }
                    else d[c] = ring_dof(f[c]);
                    av[c] = (f[c] == i || f[c] == j) ? k : f[c];
                    ad[c] = (f[c] == i || f[c] == j) ? dk : d[c];
                }
                cur.before_id.push_back(t); cur.before_v.push_back(f); cur.before_d.push_back(d);
                if (has_i && has_j) continue;
                cur.after_id.push_back(t); cur.after_v.push_back(av); cur.after_d.push_back(ad);
            }
            fixed.assign(2 * cur.ndof, 0);
            val.assign(2 * cur.ndof, 0.0);
            if (kind != 2) {
                int pa = -1, pb = -1;
                double far2 = -1.0;
                for (int s = 0; s < nr; ++s)
                    for (int r = s + 1; r < nr; ++r) {
                        const double d2 = S.sqdist(ring[s], ring[r]);
                        if (d2 > far2) { far2 = d2; pa = s; pb = r; }
                    }
                if (pa < 0) break;
                const double d = std::sqrt(far2);
                fixed[2 * pa] = fixed[2 * pa + 1] = fixed[2 * pb] = fixed[2 * pb + 1] = 1;
                val[2 * pb] = d;
                cur.scale = d;
            } else {
                const int dp = ring_dof(p), dq = ring_dof(q);
                const double lpi = std::sqrt(S.sqdist(p, i)), lij = std::sqrt(S.sqdist(i, j)),
                             ljq = std::sqrt(S.sqdist(j, q));
                int first, last, nline;
                double span;
                int line[5];
                if (cs == 0) { line[0] = di; line[1] = dj; line[2] = dq; nline = 3; first = di; last = dq; span = lij + ljq; }
                else if (cs == 1) { line[0] = dp; line[1] = di; line[2] = dj; nline = 3; first = dp; last = dj; span = lpi + lij; }
                else {
                    line[0] = dp; line[1] = di; line[2] = dk; line[3] = dj; line[4] = dq;
                    nline = 5; first = dp; last = dq; span = lpi + lij + ljq;
                }
                for (int s = 0; s < nline; ++s) fixed[2 * line[s] + 1] = 1;
                fixed[2 * first] = 1; val[2 * first] = 0.0;
                fixed[2 * last] = 1; val[2 * last] = span;
                cur.scale = span;
            }
            if (!flatten(S, cur, fixed, val, work)) continue;
            if (chosen < 0 || cur.energy < best.energy) { chosen = cs; std::swap(best, cur); }
        }
        if (chosen < 0) { S.X.resize(3 * (size_t)k); fail_edge(a, b); continue; }

        // move the query points of the before patch into the after patch
        moved.clear();
        after_uv.clear();
        for (size_t r = 0; r < best.after_id.size(); ++r) {
            const double *A = best.uv[best.after_d[r][0]].data();
            const double *B = best.uv[best.after_d[r][1]].data();
            const double *C = best.uv[best.after_d[r][2]].data();
            after_uv.push_back({A, B, C, orient2(A, B, C)});
        }
        for (size_t s = 0; s < best.before_id.size(); ++s) {
            const int t = best.before_id[s];
            for (int v : bucket[t]) {
                double u0 = 0.0, u1 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    u0 += bary[v][c] * best.uv[best.before_d[s][c]][0];
                    u1 += bary[v][c] * best.uv[best.before_d[s][c]][1];
                }
                const double pt[2] = {u0, u1};
                int win = -1;
                double win_min = 0.0, wl[3] = {0, 0, 0};
                for (size_t r = 0; r < after_uv.size(); ++r) {
                    const double *A = after_uv[r].A, *B = after_uv[r].B, *C = after_uv[r].C;
                    const double area = after_uv[r].area;
                    const double l0 = orient2(pt, B, C) / area;
                    const double l1 = orient2(A, pt, C) / area;
                    const double l2 = orient2(A, B, pt) / area;
                    const double mn = std::min(l0, std::min(l1, l2));
                    if (win < 0 || mn > win_min ||
                        (mn == win_min && best.after_id[r] < best.after_id[win])) {
                        win = (int)r; win_min = mn; wl[0] = l0; wl[1] = l1; wl[2] = l2;
                    }
                }
                double sum = 0.0;
                for (int c = 0; c < 3; ++c) {
                    if (wl[c] < 0.0) { st[7] = std::max(st[7], -wl[c]); wl[c] = 0.0; }
                    sum += wl[c];
                }
                for (int c = 0; c < 3; ++c) bary[v][c] = wl[c] / sum;
                where[v] = best.after_id[win];
                moved.push_back(v);
            }
            bucket[t].clear();
        }
        for (int v : moved) bucket[where[v]].push_back(v);
        // topology update
        for (size_t s = 0; s < best.before_id.size(); ++s) {
            const int t = best.before_id[s];
            auto it = std::find(best.after_id.begin(), best.after_id.end(), t);
            if (it != best.after_id.end()) {
                S.tri[t] = best.after_v[it - best.after_id.begin()];
            } else {
                S.tri_alive[t] = 0;
                for (int c = 0; c < 3; ++c) {
                    auto &sv = S.star[best.before_v[s][c]];
                    sv.erase(std::find(sv.begin(), sv.end(), t));
                }
            }
        }
        S.vert_alive[i] = S.vert_alive[j] = 0;
        S.star[i].clear();
        S.star[j].clear();
        S.vert_alive.push_back(1);
        nfailed.push_back(0);
        S.star.push_back(best.after_id);
        --alive;
        st[0]++;
        if (kind == 0) st[2]++;
        else if (kind == 1) st[3]++;
        else st[4 + chosen]++;
        // queue the new edges at k and re-enable failed edges whose
        // neighbourhood (an endpoint in the new 1-ring of k) changed
        S.link(k, la);
        for (auto &pr : la) pq.push({S.sqdist(k, pr.first), pr.first, k});
        if (!failed.empty())
            for (auto &pr : la) {
                const int x = pr.first;
                if (nfailed[x] == 0) continue;
                S.link(x, lb);
                for (auto &qr : lb) {
                    const int y = qr.first;
                    auto it = failed.find(ekey(std::min(x, y), std::max(x, y)));
                    if (it != failed.end()) {
                        failed.erase(it);
                        nfailed[x]--;
                        nfailed[y]--;
                        pq.push({S.sqdist(x, y), std::min(x, y), std::max(x, y)});
                    }
                }
            }
    }

    // compact the coarse mesh (ascending old ids / triangle ids)
    const int nv = (int)(S.X.size() / 3);
    std::vector<int> cid(nv, -1);
    out.X.clear();
    int nc = 0;
    for (int v = 0; v < nv; ++v)
        if (S.vert_alive[v]) {
            cid[v] = nc++;
            for (int c = 0; c < 3; ++c) out.X.push_back(S.X[3 * v + c]);
        }
    out.F.clear();
    for (int t = 0; t < m; ++t)
        if (S.tri_alive[t])
            for (int c = 0; c < 3; ++c) out.F.push_back(cid[S.tri[t][c]]);
    out.pcols.assign(3 * (size_t)n, -1);
    out.pw.assign(3 * (size_t)n, 0.0);
    for (int v = 0; v < n; ++v) {
        double w[3], sum = 0.0;
        for (int c = 0; c < 3; ++c) { w[c] = bary[v][c] < 1e-12 ? 0.0 : bary[v][c]; sum += w[c]; }
        for (int c = 0; c < 3; ++c) {
            out.pw[3 * v + c] = w[c] / sum;
            out.pcols[3 * v + c] = w[c] > 0.0 ? cid[S.tri[where[v]][c]] : -1;
        }
    }
    std::memcpy(out.stats, st, sizeof(st));
    return 0;
}

}  // namespace smg
