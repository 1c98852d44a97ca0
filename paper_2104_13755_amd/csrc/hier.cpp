// Host setup of the device hierarchy: coloring (App. A, Alg. "Graph
// Coloring"), color-major permutation, sliced-ELL layout, restriction
// R = P^T, and the symbolic Galerkin products A_{l+1} = P_l^T A_l P_l (Eq. gca)
// with the plans that let the device recompute their values for any A_0.
#include "hier.h"

#include <algorithm>
#include <array>
#include <numeric>

namespace smg {

// Alg. "Graph Coloring": descending degree (ties ascending index); first
// palette color absent among painted neighbours, moved to the palette's back;
// otherwise a new color appended.  Colors are numbered by creation.
int greedy_coloring(int n, const int32_t *rowptr, const int32_t *cols, std::vector<int32_t> &color) {
    std::vector<int32_t> degree(n);
    for (int i = 0; i < n; ++i) {
        int d = 0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) d += cols[p] != i;
        degree[i] = d;
    }
    // descending degree, ties ascending index: a counting sort by degree
    int maxd = 0;
    for (int i = 0; i < n; ++i) maxd = std::max(maxd, degree[i]);
    std::vector<int32_t> start(maxd + 2, 0), order(n);
    for (int i = 0; i < n; ++i) start[maxd - degree[i] + 1]++;
    for (int d = 0; d <= maxd; ++d) start[d + 1] += start[d];
    for (int i = 0; i < n; ++i) order[start[maxd - degree[i]]++] = i;
    color.assign(n, -1);
    std::vector<int32_t> palette;
    std::vector<int32_t> taken;   // taken[c] == node + 1 marks color c as used around node
    for (int node : order) {
        for (int p = rowptr[node]; p < rowptr[node + 1]; ++p) {
            const int nb = cols[p];
            if (nb != node && color[nb] >= 0) taken[color[nb]] = node + 1;
        }
        auto it = std::find_if(palette.begin(), palette.end(), [&](int c) { return taken[c] != node + 1; });
        int c;
        if (it == palette.end()) {
            c = (int)taken.size();
            taken.push_back(0);
            palette.push_back(c);
        } else {
            c = *it;
            palette.erase(it);
            palette.push_back(c);
        }
        color[node] = c;
    }
    return (int)taken.size();
}

Csr galerkin_pattern(const Csr &A, int nc, const std::vector<int32_t> &pcols) {
    const int n = A.n;
    // R = P^T structure
    std::vector<int32_t> rptr(nc + 1, 0);
    for (int i = 0; i < n; ++i)
        for (int m = 0; m < 3; ++m) if (pcols[3 * i + m] >= 0) rptr[pcols[3 * i + m] + 1]++;
    for (int a = 0; a < nc; ++a) rptr[a + 1] += rptr[a];
    std::vector<int32_t> ridx(rptr[nc]);
    std::vector<int32_t> fill(rptr.begin(), rptr.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int m = 0; m < 3; ++m) if (pcols[3 * i + m] >= 0) ridx[fill[pcols[3 * i + m]]++] = i;
    // columns of T = A P per fine row (each fine row feeds up to three coarse rows)
    std::vector<int32_t> tptr(n + 1, 0), tidx, mark(nc, -1);
    tidx.reserve((size_t)A.ptr[n] * 2);
    for (int i = 0; i < n; ++i) {
        for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
            const int j = A.idx[p];
            for (int m = 0; m < 3; ++m) {
                const int b = pcols[3 * j + m];
                if (b >= 0 && mark[b] != i) { mark[b] = i; tidx.push_back(b); }
            }
        }
        tptr[i + 1] = (int32_t)tidx.size();
    }
    Csr C;
    C.n = C.m = nc;
    C.ptr.assign(nc + 1, 0);
    std::fill(mark.begin(), mark.end(), -1);
    std::vector<int32_t> row;
    for (int a = 0; a < nc; ++a) {
        row.clear();
        for (int q = rptr[a]; q < rptr[a + 1]; ++q) {
            const int i = ridx[q];
            for (int t = tptr[i]; t < tptr[i + 1]; ++t) {
                const int b = tidx[t];
                if (mark[b] != a) { mark[b] = a; row.push_back(b); }
            }
        }
        std::sort(row.begin(), row.end());
        C.idx.insert(C.idx.end(), row.begin(), row.end());
        C.ptr[a + 1] = (int32_t)C.idx.size();
    }
    return C;
}

// Measured on MI355X (1M-vertex torus hierarchy): one lane per row for the
// ~6-entry rows of a mesh Laplacian, eight lanes for the 20-30-entry rows of
// the Galerkin levels (shorter dependent-load chains, more waves in flight).
int default_lanes_per_row(double avg) {
    return avg < 10.0 ? 1 : 8;
}

static void build_sell(LevelHost &L, int lpr) {
    SellLayout &S = L.sell;
    const int n = L.n;
    S.n = n;
    S.lpr = lpr;
    const int rps = 64 / lpr;   // rows per slice
    // permuted off-diagonal pattern, ascending permuted columns
    S.pptr.assign(n + 1, 0);
    S.rowlen.assign(n, 0);
    for (int r = 0; r < n; ++r) {
        const int i = L.perm[r];
        S.rowlen[r] = (L.pat.ptr[i + 1] - L.pat.ptr[i]) - 1;
        S.pptr[r + 1] = S.pptr[r] + S.rowlen[r];
    }
    S.pidx.resize(S.pptr[n]);
    for (int r = 0; r < n; ++r) {
        const int i = L.perm[r];
        int o = S.pptr[r];
        for (int p = L.pat.ptr[i]; p < L.pat.ptr[i + 1]; ++p)
            if (L.pat.idx[p] != i) S.pidx[o++] = L.iperm[L.pat.idx[p]];
        std::sort(S.pidx.begin() + S.pptr[r], S.pidx.begin() + S.pptr[r + 1]);
    }
    // slices of 64 rows that never straddle two colors
    S.slice_row0.clear();
    S.slice_off.assign(1, 0);
    S.color_slice.assign(1, 0);
    S.row_slice.assign(n, 0);
    S.color_w.assign(L.ncolors, 0);
    std::vector<int> ws;
    for (int c = 0; c < L.ncolors; ++c) {
        // a color whose slices all take its widest slice's rounds costs at
        // most a quarter more slots; then every slice's offset follows from
        // its index and a relaxation needs no slice table
        ws.clear();
        int64_t sum = 0;
        int wmax = 0;
        for (int r0 = S.color_row[c]; r0 < S.color_row[c + 1]; r0 += rps) {
            const int r1 = std::min(r0 + rps, S.color_row[c + 1]);
            int w = 0;
            for (int r = r0; r < r1; ++r) w = std::max(w, (S.rowlen[r] + lpr - 1) / lpr);
            ws.push_back(w);
            sum += w;
            wmax = std::max(wmax, w);
        }
        if (4 * (int64_t)wmax * (int64_t)ws.size() <= 5 * sum) {
            S.color_w[c] = wmax;
            std::fill(ws.begin(), ws.end(), wmax);
        }
        int q = 0;
        for (int r0 = S.color_row[c]; r0 < S.color_row[c + 1]; r0 += rps, ++q) {
            const int r1 = std::min(r0 + rps, S.color_row[c + 1]);
            for (int r = r0; r < r1; ++r) S.row_slice[r] = (int)S.slice_row0.size();
            S.slice_row0.push_back(r0);
            S.slice_off.push_back(S.slice_off.back() + 64 * ws[q]);
        }
        S.color_slice.push_back((int)S.slice_row0.size());
    }
    S.nslices = (int)S.slice_row0.size();
    S.cols.assign(S.slots(), 0);
    for (int s = 0; s < S.nslices; ++s) {
        const int w = (S.slice_off[s + 1] - S.slice_off[s]) / 64;
        for (int t = 0; t < 64; ++t) {
            const int r = S.slice_row0[s] + t / lpr, j = t % lpr;
            const bool valid = r < n && S.row_slice[r] == s;
            for (int q = 0; q < w; ++q) {
                const int e = q * lpr + j;
                const int slot = S.slice_off[s] + q * 64 + t;
                if (valid && e < S.rowlen[r]) S.cols[slot] = S.pidx[S.pptr[r] + e];
                else S.cols[slot] = valid ? r : S.slice_row0[s];   // padding: weight 0
            }
        }
    }
}

// storage position of entry (r, c) of level L (permuted indices)
static int32_t store_pos(const LevelHost &L, int r, int c) {
    if (L.coarsest) return r + c * L.n;
    if (r == c) return -1 - r;
    const SellLayout &S = L.sell;
    const int32_t *b = S.pidx.data() + S.pptr[r], *e = S.pidx.data() + S.pptr[r + 1];
    const int32_t *it = std::lower_bound(b, e, c);
    if (it == e || *it != c) return INT32_MIN;
    return S.slot(r, (int)(it - b));
}

// 30-bit Morton key of each vertex: positions quantized to 1024 cells along
// the bounding box's longest side, bits of x, y, z interleaved
static std::vector<int64_t> morton_keys(const std::vector<double> &X) {
    const size_t n = X.size() / 3;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (size_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], X[3 * i + d]); hi[d] = std::max(hi[d], X[3 * i + d]); }
    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    std::vector<int64_t> key(n, 0);
    for (size_t i = 0; i < n; ++i) {
        int64_t q[3];
        for (int d = 0; d < 3; ++d) q[d] = std::min<int64_t>(1023, (int64_t)((X[3 * i + d] - lo[d]) / ext * 1023.0 + 0.5));
        int64_t k = 0;
        for (int b = 0; b < 10; ++b)
            for (int d = 0; d < 3; ++d) k |= ((q[d] >> b) & 1) << (3 * b + d);
        key[i] = k;
    }
    return key;
}

int build_levels(const HierHost &H, const Csr &A0, const std::vector<int> &lpr, int sort_rows,
                 std::vector<LevelHost> &levels, std::string &err) {
    const int nlev = H.nlev;
    levels.assign(nlev, LevelHost());
    Csr pat = A0;
    for (int l = 0; l < nlev; ++l) {
        LevelHost &L = levels[l];
        L.n = H.sizes[l];
        L.pat = pat;
        L.coarsest = l == nlev - 1;
        if (pat.n != L.n) { err = "pattern size mismatch at level " + std::to_string(l); return -1; }
        for (int i = 0; i < L.n; ++i) {   // diagonal must be present
            bool d = false;
            for (int p = pat.ptr[i]; p < pat.ptr[i + 1]; ++p) d |= pat.idx[p] == i;
            if (!d) { err = "missing diagonal entry"; return -1; }
        }
        L.perm.resize(L.n);
        L.iperm.resize(L.n);
        if (!L.coarsest) {
            L.ncolors = greedy_coloring(L.n, pat.ptr.data(), pat.idx.data(), L.color);
            std::vector<int32_t> cnt(L.ncolors + 1, 0);
            for (int i = 0; i < L.n; ++i) cnt[L.color[i] + 1]++;
            for (int c = 0; c < L.ncolors; ++c) cnt[c + 1] += cnt[c];
            L.sell.color_row = cnt;
            for (int i = 0; i < L.n; ++i) L.perm[cnt[L.color[i]]++] = i;
            if (l > 0 && L.n <= sort_rows) {   // tail levels: rows of a color by descending length
                auto len = [&](int i) { return pat.ptr[i + 1] - pat.ptr[i]; };
                for (int c = 0; c < L.ncolors; ++c)
                    std::stable_sort(L.perm.begin() + L.sell.color_row[c], L.perm.begin() + L.sell.color_row[c + 1],
                                     [&](int a, int b) { return len(a) > len(b); });
            } else if (l < (int)H.X.size() && H.X[l].size() == 3 * (size_t)L.n) {
                const std::vector<int64_t> key = morton_keys(H.X[l]);
                for (int c = 0; c < L.ncolors; ++c)
                    std::stable_sort(L.perm.begin() + L.sell.color_row[c], L.perm.begin() + L.sell.color_row[c + 1],
                                     [&](int a, int b) { return key[a] < key[b]; });
            }
        } else {
            std::iota(L.perm.begin(), L.perm.end(), 0);
        }
        for (int r = 0; r < L.n; ++r) L.iperm[L.perm[r]] = r;
        if (!L.coarsest) {
            int lanes = (l < (int)lpr.size() && lpr[l] > 0) ? lpr[l]
                        : default_lanes_per_row((double)(pat.idx.size() - L.n) / std::max(1, L.n));
            if (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8) { err = "lanes per row must be 1, 2, 4 or 8"; return -1; }
            build_sell(L, lanes);
        }
        if (l + 1 < nlev) pat = galerkin_pattern(pat, H.sizes[l + 1], H.pcols[l]);
    }
    // epos[c]: index of permuted column c in the current row's ascending
    // off-diagonal list (every column looked up is in that row's pattern)
    std::vector<int32_t> epos;
    for (int l = 0; l < nlev; ++l) {
        LevelHost &L = levels[l];
        L.store.resize(L.pat.idx.size());
        epos.assign(L.n, 0);
        for (int i = 0; i < L.n; ++i) {
            const int r = L.iperm[i];
            if (!L.coarsest)
                for (int e = L.sell.pptr[r]; e < L.sell.pptr[r + 1]; ++e) epos[L.sell.pidx[e]] = e - L.sell.pptr[r];
            for (int p = L.pat.ptr[i]; p < L.pat.ptr[i + 1]; ++p) {
                const int c = L.iperm[L.pat.idx[p]];
                L.store[p] = (L.coarsest || c == r) ? store_pos(L, r, c) : L.sell.slot(r, epos[c]);
            }
        }
        if (l + 1 == nlev) break;
        const LevelHost &C = levels[l + 1];
        const int n = L.n, nc = C.n;
        // prolongation, permuted, SoA
        L.pc.assign(3 * (size_t)n, 0);
        L.pw.assign(3 * (size_t)n, 0.0);
        for (int r = 0; r < n; ++r) {
            const int i = L.perm[r];
            int first = -1;
            for (int m = 0; m < 3; ++m)
                if (H.pcols[l][3 * i + m] >= 0 && H.pw[l][3 * i + m] > 0.0) { first = C.iperm[H.pcols[l][3 * i + m]]; break; }
            if (first < 0) { err = "empty prolongation row"; return -1; }
            for (int m = 0; m < 3; ++m) {
                const int col = H.pcols[l][3 * i + m];
                const double w = H.pw[l][3 * i + m];
                const bool used = col >= 0 && w > 0.0;
                L.pc[(size_t)m * n + r] = used ? C.iperm[col] : first;
                L.pw[(size_t)m * n + r] = used ? w : 0.0;
            }
        }
        // R = P^T over permuted coarse rows, fine rows ascending
        L.rptr.assign(nc + 1, 0);
        for (int r = 0; r < n; ++r)
            for (int m = 0; m < 3; ++m) if (L.pw[(size_t)m * n + r] > 0.0) L.rptr[L.pc[(size_t)m * n + r] + 1]++;
        for (int a = 0; a < nc; ++a) L.rptr[a + 1] += L.rptr[a];
        L.ridx.resize(L.rptr[nc]);
        L.rw.resize(L.rptr[nc]);
        {
            std::vector<int32_t> fill(L.rptr.begin(), L.rptr.end() - 1);
            for (int r = 0; r < n; ++r)
                for (int m = 0; m < 3; ++m) {
                    const double w = L.pw[(size_t)m * n + r];
                    if (w > 0.0) {
                        const int a = L.pc[(size_t)m * n + r];
                        L.ridx[fill[a]] = r;
                        L.rw[fill[a]] = w;
                        fill[a]++;
                    }
                }
        }
        {
            const int LR = L.rs_lanes, rps = 64 / LR, ns = (nc + rps - 1) / rps;
            L.rs_off.assign(ns + 1, 0);
            for (int s = 0; s < ns; ++s) {
                int wmax = 0;
                for (int a = s * rps; a < std::min(nc, s * rps + rps); ++a)
                    wmax = std::max(wmax, (L.rptr[a + 1] - L.rptr[a] + LR - 1) / LR);
                L.rs_off[s + 1] = L.rs_off[s] + 64 * wmax;
            }
            L.rs_idx.assign(L.rs_off[ns], 0);
            L.rs_w.assign(L.rs_off[ns], 0.0);
            for (int a = 0; a < nc; ++a) {
                const int s = a / rps, g = a % rps, w = (L.rs_off[s + 1] - L.rs_off[s]) / 64;
                const int len = L.rptr[a + 1] - L.rptr[a];
                for (int e = 0; e < w * LR; ++e) {
                    const size_t at = (size_t)L.rs_off[s] + 64 * (e / LR) + g * LR + e % LR;
                    L.rs_idx[at] = len ? L.ridx[L.rptr[a] + std::min(e, len - 1)] : 0;
                    L.rs_w[at] = e < len ? L.rw[L.rptr[a] + e] : 0.0;
                }
            }
        }
        // T = A P pattern per permuted fine row; plan1 maps (source, slot) -> T offset
        L.tptr.assign(n + 1, 0);
        L.plan1ptr.assign(n + 1, 0);
        L.plan1.reserve(3 * ((size_t)n + L.sell.pidx.size()));
        // the prolongation row by row (-1: unused slot), one cache line per source
        std::vector<std::array<int32_t, 3>> prow(n);
        for (int r = 0; r < n; ++r)
            for (int m = 0; m < 3; ++m) prow[r][m] = L.pw[(size_t)m * n + r] > 0.0 ? L.pc[(size_t)m * n + r] : -1;
        std::vector<int32_t> tcols;
        std::vector<int32_t> row;
        // mark[b] == r: coarse column b already in T row r, at offset pos[b]
        std::vector<int32_t> mark(nc, -1), pos(nc, 0);
        for (int r = 0; r < n; ++r) {
            row.clear();
            auto add_src = [&](int src) {
                for (int m = 0; m < 3; ++m) {
                    const int b = prow[src][m];
                    if (b >= 0 && mark[b] != r) { mark[b] = r; row.push_back(b); }
                }
            };
            add_src(r);
            for (int e = 0; e < L.sell.rowlen[r]; ++e) add_src(L.sell.pidx[L.sell.pptr[r] + e]);
            std::sort(row.begin(), row.end());
            for (size_t k = 0; k < row.size(); ++k) pos[row[k]] = (int32_t)k;
            if (row.size() > 65535) { err = "Galerkin row too long"; return -1; }
            tcols.insert(tcols.end(), row.begin(), row.end());
            L.tptr[r + 1] = (int32_t)tcols.size();
            L.tmax = std::max(L.tmax, (int)row.size());
            auto emit = [&](int src) {
                for (int m = 0; m < 3; ++m) {
                    const int b = prow[src][m];
                    L.plan1.push_back((uint16_t)(b >= 0 ? pos[b] : 0));
                }
            };
            emit(r);
            for (int e = 0; e < L.sell.rowlen[r]; ++e) emit(L.sell.pidx[L.sell.pptr[r] + e]);
            L.plan1ptr[r + 1] = (int32_t)L.plan1.size();
        }
        // local slots of coarse row a (permuted): its pattern columns (permuted,
        // ascending), each with its storage position in level l+1
        L.optr.assign(nc + 1, 0);
        L.opos.clear();
        std::vector<int32_t> ocol;   // permuted column of each local slot
        epos.assign(nc, 0);
        for (int a = 0; a < nc; ++a) {
            const int i = C.perm[a];
            const size_t o0 = ocol.size();
            for (int p = C.pat.ptr[i]; p < C.pat.ptr[i + 1]; ++p) ocol.push_back(C.iperm[C.pat.idx[p]]);
            std::sort(ocol.begin() + o0, ocol.end());
            if (!C.coarsest)
                for (int e = C.sell.pptr[a]; e < C.sell.pptr[a + 1]; ++e) epos[C.sell.pidx[e]] = e - C.sell.pptr[a];
            for (size_t k = o0; k < ocol.size(); ++k) {
                const int c = ocol[k];
                const int32_t pos = (C.coarsest || c == a) ? store_pos(C, a, c) : C.sell.slot(a, epos[c]);
                if (pos == INT32_MIN) { err = "coarse pattern without storage"; return -1; }
                L.opos.push_back(pos);
            }
            L.optr[a + 1] = (int32_t)ocol.size();
            L.cmax = std::max(L.cmax, (int)(ocol.size() - o0));
            if (ocol.size() - o0 > 65535) { err = "coarse row too long"; return -1; }
        }
        // plan2: for coarse row a, for R entry (r, w), for T entry (r, b): local slot of (a, b)
        L.plan2ptr.assign(nc + 1, 0);
        {
            size_t total = 0;
            for (int a = 0; a < nc; ++a)
                for (int q = L.rptr[a]; q < L.rptr[a + 1]; ++q) total += L.tptr[L.ridx[q] + 1] - L.tptr[L.ridx[q]];
            L.plan2.reserve(total);
        }
        std::fill(mark.begin(), mark.end(), -1);
        for (int a = 0; a < nc; ++a) {
            for (int k = L.optr[a]; k < L.optr[a + 1]; ++k) { mark[ocol[k]] = a; pos[ocol[k]] = k - L.optr[a]; }
            for (int q = L.rptr[a]; q < L.rptr[a + 1]; ++q) {
                const int r = L.ridx[q];
                for (int t = L.tptr[r]; t < L.tptr[r + 1]; ++t) {
                    if (mark[tcols[t]] != a) { err = "Galerkin plan outside the symbolic pattern"; return -1; }
                    L.plan2.push_back((uint16_t)pos[tcols[t]]);
                }
            }
            if (L.plan2.size() > (size_t)INT32_MAX) { err = "Galerkin plan too large"; return -1; }
            L.plan2ptr[a + 1] = (int32_t)L.plan2.size();
        }
    }
    return 0;
}

void build_tail_layout(const LevelHost &L, int nc, int threads, int grp, TailLayout &out) {
    const SellLayout &S = L.sell;
    out = TailLayout();
    int maxrows = 1;
    for (int c = 0; c + 1 < (int)S.color_row.size(); ++c)
        maxrows = std::max(maxrows, S.color_row[c + 1] - S.color_row[c]);
    // widest lane group up to 4 that still fits a whole color in one pass (a
    // full-size sweep: wider groups spend more in the cross-lane reduction
    // than they save in record rounds)
    int g = 1;
    while (g < 4 && (int64_t)maxrows * g * 2 <= threads) g *= 2;
    if (grp > 0) g = std::min(grp, 64);
    out.grp = g;
    const int per = threads / g;
    int64_t off = 0;
    for (int c = 0; c + 1 < (int)S.color_row.size(); ++c) {
        const int r0 = S.color_row[c], r1 = S.color_row[c + 1];
        for (int p0 = r0; p0 < r1; p0 += per) {
            const int nr = std::min(per, r1 - p0), nt = nr * g, nw = (nt + 63) / 64;
            const bool last = p0 + per >= r1;
            out.pass.insert(out.pass.end(), {p0, nr, (int)last << 16, (int32_t)(out.wave.size() / 2)});
            for (int w = 0; w < nw; ++w) {
                int kmax = 0;
                for (int t = w * 64; t < std::min(nt, w * 64 + 64); t += g)
                    kmax = std::max(kmax, (S.rowlen[p0 + t / g] + g - 1) / g);
                const int npair = (kmax + 1) / 2;   // rounds in pairs: record (k, lane) at 128 (k / 2) + 2 lane + k % 2
                out.wave.insert(out.wave.end(), {(int32_t)off, npair});
                for (int pr = 0; pr < npair; ++pr)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int h = 0; h < 2; ++h) {
                            const int k = 2 * pr + h;
                            const int t = w * 64 + lane, r = p0 + t / g, e = k * g + t % g;
                            const bool ok = t < nt && e < S.rowlen[r];
                            const int32_t slot = ok ? S.slot(r, e) : -1;
                            out.src.push_back(slot);
                            out.cols.push_back(ok ? S.cols[slot] : 0);
                        }
                off += 128 * (int64_t)npair;
            }
        }
    }
    out.nc = nc;
    for (int a = 0; a < nc; ++a) out.rk = std::max(out.rk, L.rptr[a + 1] - L.rptr[a]);
    out.ridx.assign((size_t)out.rk * nc, 0);
    out.rw.assign((size_t)out.rk * nc, 0.0);
    for (int a = 0; a < nc; ++a)
        for (int p = L.rptr[a]; p < L.rptr[a + 1]; ++p) {
            const size_t at = (size_t)(p - L.rptr[a]) * nc + a;
            out.ridx[at] = L.ridx[p];
            out.rw[at] = L.rw[p];
        }
}

bool check_tail_layout(const TailLayout &T, int n, int threads, std::string &err) {
    const int g = T.grp;
    if (g < 1 || g > 64 || (g & (g - 1))) { err = "tail: bad lane group"; return false; }
    int64_t off = 0;
    size_t wv = 0;
    for (size_t p = 0; p + 3 < T.pass.size(); p += 4) {
        const int r0 = T.pass[p], nr = T.pass[p + 1];
        const int nw = (nr * g + 63) / 64;
        if (r0 < 0 || nr < 1 || r0 + nr > n || (int64_t)nr * g > threads || T.pass[p + 3] != (int)wv) {
            err = "tail: bad pass";
            return false;
        }
        for (int w = 0; w < nw; ++w, ++wv) {
            if (2 * wv + 1 >= T.wave.size() || T.wave[2 * wv] != off || T.wave[2 * wv + 1] < 0) { err = "tail: bad wave"; return false; }
            off += 128 * (int64_t)T.wave[2 * wv + 1];
        }
    }
    if (2 * wv != T.wave.size()) { err = "tail: wave count"; return false; }
    if (off != (int64_t)T.src.size() || T.cols.size() != T.src.size()) { err = "tail: record count"; return false; }
    for (int32_t c : T.cols) if (c < 0 || c >= n) { err = "tail: record column"; return false; }
    if (T.ridx.size() != (size_t)T.rk * T.nc || T.rw.size() != T.ridx.size()) { err = "tail: restriction size"; return false; }
    for (int32_t i : T.ridx) if (i < 0 || i >= n) { err = "tail: restriction index"; return false; }
    return true;
}

}  // namespace smg
