// Test driver (host only): builds the device-side level data of a hierarchy
// with build_levels() and replays the two Galerkin plans on the CPU, row by
// row in the order the device kernels use them (T = A P per permuted fine
// row, then A_{l+1} = P^T T per permuted coarse row), starting from A_0 in the
// library's storage (sliced ELL + diagonal; dense on the coarsest level).
// Every level's values are decoded back to natural CSR through `store`.
// Then, on every smoothed level, one Gauss-Seidel sweep is replayed, in
// ascending and in descending color order, from the sliced-ELL layout the
// way the per-color launches read it (slice table, or for a color of uniform
// width its offset from the slice index), and from the one-workgroup tail's
// record layout (records read per wavefront lane as the device reads them).
// Last, per transfer, the restriction from its sliced-ELL form (P^T r) and
// the prolongation from its permuted ELL-3 form (x + P e).
//
// Input (binary, little endian): int32 nlev, lpr, sort_rows; int32 sizes[nlev];
// per level l < nlev-1: int32 pcols[3 n_l], double pw[3 n_l]; int32 nnz;
// int32 ptr[n_0 + 1], idx[nnz]; double a[nnz]; per smoothed level (natural
// order): double x0[n_l], b[n_l]; per level l < nlev-1: double e[n_{l+1}].
// Output (binary): per level: int32 nnz, ncolors; int32 ptr[n_l + 1],
// idx[nnz]; double a[nnz]; int32 color[n_l] (all -1 on the coarsest level);
// then per smoothed level: int32 grp, uniform-width colors; double x_asc[n_l], x_desc[n_l] from the
// tail records, then x_asc[n_l], x_desc[n_l] from the sliced ELL (natural);
// then per level l < nlev-1: double P^T x0[n_{l+1}], x0 + P e[n_l] (natural).
#include "hier.h"

#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace smg;

template <class T> static bool rd(FILE *f, T *p, size_t n) { return fread(p, sizeof(T), n, f) == n; }
template <class T> static void wr(FILE *f, const T *p, size_t n) { fwrite(p, sizeof(T), n, f); }

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[3];
    if (!rd(f, hdr, 3)) return 3;
    const int nlev = hdr[0];
    HierHost H;
    H.nlev = nlev;
    H.sizes.resize(nlev);
    if (!rd(f, H.sizes.data(), nlev)) return 3;
    for (int l = 0; l + 1 < nlev; ++l) {
        std::vector<int32_t> c(3 * (size_t)H.sizes[l]);
        std::vector<double> w(3 * (size_t)H.sizes[l]);
        if (!rd(f, c.data(), c.size()) || !rd(f, w.data(), w.size())) return 3;
        H.pcols.push_back(c);
        H.pw.push_back(w);
    }
    int32_t nnz;
    if (!rd(f, &nnz, 1)) return 3;
    Csr A0;
    A0.n = A0.m = H.sizes[0];
    A0.ptr.resize(A0.n + 1);
    A0.idx.resize(nnz);
    std::vector<double> a0(nnz);
    if (!rd(f, A0.ptr.data(), A0.ptr.size()) || !rd(f, A0.idx.data(), nnz) || !rd(f, a0.data(), nnz)) return 3;
    std::vector<std::vector<double>> x0(nlev), b0(nlev);
    for (int l = 0; l + 1 < nlev; ++l) {
        x0[l].resize(H.sizes[l]);
        b0[l].resize(H.sizes[l]);
        if (!rd(f, x0[l].data(), x0[l].size()) || !rd(f, b0[l].data(), b0[l].size())) return 3;
    }
    std::vector<std::vector<double>> ec(nlev);
    for (int l = 0; l + 1 < nlev; ++l) {
        ec[l].resize(H.sizes[l + 1]);
        if (!rd(f, ec[l].data(), ec[l].size())) return 3;
    }
    fclose(f);

    std::vector<LevelHost> lev;
    std::string err;
    if (build_levels(H, A0, std::vector<int>(nlev, hdr[1]), hdr[2], lev, err) != 0) {
        fprintf(stderr, "build_levels: %s\n", err.c_str());
        return 4;
    }
    // storage of every level: vals (SELL slots, or dense n x n on the coarsest) + diag
    std::vector<std::vector<double>> vals(nlev), diag(nlev);
    for (int l = 0; l < nlev; ++l) {
        const LevelHost &L = lev[l];
        vals[l].assign(L.coarsest ? (size_t)L.n * L.n : (size_t)L.sell.slots(), 0.0);
        diag[l].assign(L.n, 0.0);
    }
    auto put = [&](int l, int32_t pos, double v) {
        if (pos >= 0) vals[l][pos] = v; else diag[l][-1 - pos] = v;
    };
    for (int p = 0; p < nnz; ++p) put(0, lev[0].store[p], a0[p]);
    for (int l = 0; l + 1 < nlev; ++l) {
        const LevelHost &L = lev[l];
        const SellLayout &S = L.sell;
        const int n = L.n, nc = lev[l + 1].n;
        std::vector<double> T(L.tptr[n], 0.0);
        for (int r = 0; r < n; ++r) {
            const uint16_t *pl = L.plan1.data() + L.plan1ptr[r];
            double *acc = T.data() + L.tptr[r];
            for (int m = 0; m < 3; ++m) acc[pl[m]] += diag[l][r] * L.pw[(size_t)m * n + r];
            const int s = S.row_slice[r];
            const int base = S.slice_off[s] + (r - S.slice_row0[s]) * S.lpr;
            for (int e = 0; e < S.rowlen[r]; ++e) {
                const int slot = base + (e / S.lpr) * 64 + (e % S.lpr);
                const int c = S.cols[slot];
                for (int m = 0; m < 3; ++m) acc[pl[3 * (e + 1) + m]] += vals[l][slot] * L.pw[(size_t)m * n + c];
            }
        }
        for (int a = 0; a < nc; ++a) {
            std::vector<double> acc(L.optr[a + 1] - L.optr[a], 0.0);
            int idx = L.plan2ptr[a];
            for (int p = L.rptr[a]; p < L.rptr[a + 1]; ++p) {
                const int r = L.ridx[p];
                for (int t = L.tptr[r]; t < L.tptr[r + 1]; ++t) acc[L.plan2[idx++]] += L.rw[p] * T[t];
            }
            if (idx != L.plan2ptr[a + 1]) return 5;
            for (size_t k = 0; k < acc.size(); ++k) put(l + 1, L.opos[L.optr[a] + k], acc[k]);
        }
    }
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    for (int l = 0; l < nlev; ++l) {
        const LevelHost &L = lev[l];
        const int32_t hd[2] = {(int32_t)L.pat.idx.size(), L.ncolors};
        wr(o, hd, 2);
        wr(o, L.pat.ptr.data(), L.pat.ptr.size());
        wr(o, L.pat.idx.data(), L.pat.idx.size());
        std::vector<double> av(L.pat.idx.size());
        for (size_t p = 0; p < av.size(); ++p) {
            const int32_t pos = L.store[p];
            av[p] = pos >= 0 ? vals[l][pos] : diag[l][-1 - pos];
        }
        wr(o, av.data(), av.size());
        std::vector<int32_t> col(L.n, -1);
        if (!L.coarsest) col = L.color;
        wr(o, col.data(), col.size());
    }
    const int threads = 1024;
    for (int l = 0; l + 1 < nlev; ++l) {
        const LevelHost &L = lev[l];
        TailLayout T;
        build_tail_layout(L, lev[l + 1].n, threads, 0, T);
        if (!check_tail_layout(T, L.n, threads, err)) {
            fprintf(stderr, "level %d: %s\n", l, err.c_str());
            return 6;
        }
        const int G = T.grp, npass = (int)T.pass.size() / 4;
        int nuniform = 0;
        for (int c = 0; c < L.ncolors; ++c) nuniform += L.sell.color_w[c] > 0;
        wr(o, &G, 1);
        wr(o, &nuniform, 1);
        for (int dir = 0; dir < 2; ++dir) {
            std::vector<double> x(L.n), b(L.n);
            for (int r = 0; r < L.n; ++r) { x[r] = x0[l][L.perm[r]]; b[r] = b0[l][L.perm[r]]; }
            for (int pp = 0; pp < npass; ++pp) {
                const int p = dir ? npass - 1 - pp : pp;
                const int row0 = T.pass[4 * p], nrows = T.pass[4 * p + 1], w0 = T.pass[4 * p + 3];
                for (int g = 0; g < nrows; ++g) {
                    double acc = 0.0;
                    for (int j = 0; j < G; ++j) {
                        const int t = g * G + j, w = w0 + t / 64, lane = t % 64;
                        const int off = T.wave[2 * w], npair = T.wave[2 * w + 1];
                        for (int k = 0; k < 2 * npair; ++k) {
                            const int rec = off + 128 * (k / 2) + 2 * lane + k % 2;
                            const double v = T.src[rec] >= 0 ? vals[l][T.src[rec]] : 0.0;
                            acc += v * x[T.cols[rec]];
                        }
                    }
                    const int r = row0 + g;
                    x[r] = (b[r] - acc) / diag[l][r];
                }
            }
            std::vector<double> xn(L.n);
            for (int r = 0; r < L.n; ++r) xn[L.perm[r]] = x[r];
            wr(o, xn.data(), xn.size());
        }
        const SellLayout &S = L.sell;
        for (int dir = 0; dir < 2; ++dir) {
            std::vector<double> x(L.n), b(L.n);
            for (int r = 0; r < L.n; ++r) { x[r] = x0[l][L.perm[r]]; b[r] = b0[l][L.perm[r]]; }
            for (int cc = 0; cc < L.ncolors; ++cc) {
                const int c = dir ? L.ncolors - 1 - cc : cc;
                const int s0 = S.color_slice[c], s1 = S.color_slice[c + 1];
                for (int s = s0; s < s1; ++s) {
                    int r0, r1, off, w;
                    if (S.color_w[c] > 0) {   // uniform width: offsets from the slice index
                        w = S.color_w[c];
                        r0 = S.color_row[c] + (s - s0) * (64 / S.lpr);
                        r1 = S.color_row[c + 1];
                        off = S.slice_off[s0] + (s - s0) * 64 * w;
                    } else {
                        r0 = S.slice_row0[s];
                        r1 = S.slice_row0[s + 1];
                        off = S.slice_off[s];
                        w = (S.slice_off[s + 1] - off) / 64;
                    }
                    std::vector<double> acc(64 / S.lpr, 0.0);
                    for (int lane = 0; lane < 64; ++lane)
                        for (int k = 0; k < w; ++k) {
                            const int at = off + lane + 64 * k;
                            acc[lane / S.lpr] += vals[l][at] * x[S.cols[at]];
                        }
                    for (int g = 0; g < 64 / S.lpr && r0 + g < r1; ++g) {
                        const int r = r0 + g;
                        x[r] = (b[r] - acc[g]) / diag[l][r];
                    }
                }
            }
            std::vector<double> xn(L.n);
            for (int r = 0; r < L.n; ++r) xn[L.perm[r]] = x[r];
            wr(o, xn.data(), xn.size());
        }
    }
    for (int l = 0; l + 1 < nlev; ++l) {
        const LevelHost &L = lev[l], &C = lev[l + 1];
        const int n = L.n, nc = C.n, lr = L.rs_lanes, rps = 64 / lr;
        std::vector<double> r(n), rc(nc, 0.0);
        for (int i = 0; i < n; ++i) r[i] = x0[l][L.perm[i]];
        for (int s = 0; s * rps < nc; ++s) {
            const int w = (L.rs_off[s + 1] - L.rs_off[s]) / 64;
            for (int lane = 0; lane < 64; ++lane) {
                const int a = s * rps + lane / lr;
                if (a >= nc) continue;
                for (int k = 0; k < w; ++k) {
                    const int at = L.rs_off[s] + lane + 64 * k;
                    rc[a] += L.rs_w[at] * r[L.rs_idx[at]];
                }
            }
        }
        std::vector<double> rcn(nc);
        for (int a = 0; a < nc; ++a) rcn[C.perm[a]] = rc[a];
        wr(o, rcn.data(), rcn.size());
        std::vector<double> x(n);
        for (int i = 0; i < n; ++i) {
            const int rr = L.iperm[i];
            double v = r[rr];
            for (int m = 0; m < 3; ++m) v += L.pw[(size_t)m * n + rr] * ec[l][C.perm[L.pc[(size_t)m * n + rr]]];
            x[i] = v;
        }
        wr(o, x.data(), x.size());
    }
    fclose(o);
    return 0;
}
