// Versioned binary file of a host hierarchy (the geometry-only precompute
// is reused for every later system on the same mesh).  Layout, all values in
// the host's byte order (little-endian on the targets of this library):
//
//   "SMGHIER1"                       8 bytes, magic and format version
//   int32  nlev                      1..64
//   int32  sizes[nlev]               vertices per level, each >= 1
//   per level l:    uint8 has_X, then double X[3 sizes[l]] if has_X
//   per level l < nlev - 1:          int32 pcols[3 sizes[l]], double pw[3 sizes[l]],
//                                    double stats[8]
//   uint64 checksum                  FNV-1a over every byte before it
//
// A loaded file is checked like externally given prolongations (columns in
// range, weights finite and >= 0, a positive weight in every row) besides
// the magic, the sizes and the checksum.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hier.h"

namespace smg {
namespace {

constexpr char kMagic[8] = {'S', 'M', 'G', 'H', 'I', 'E', 'R', '1'};

struct Writer {
    FILE *f;
    uint64_t h = 1469598103934665603ull;
    bool ok = true;
    void put(const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
        if (n && std::fwrite(p, 1, n, f) != n) ok = false;
    }
};

struct Reader {
    FILE *f;
    uint64_t h = 1469598103934665603ull;
    bool ok = true;
    bool get(void *p, size_t n) {
        if (!ok) return false;
        if (n && std::fread(p, 1, n, f) != n) { ok = false; return false; }
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
        return true;
    }
};

}  // namespace

bool hier_write(const HierHost &H, const char *path, std::string &err) {
    FILE *f = std::fopen(path, "wb");
    if (!f) { err = std::string("cannot open ") + path + " for writing"; return false; }
    Writer w{f};
    w.put(kMagic, 8);
    const int32_t nlev = H.nlev;
    w.put(&nlev, 4);
    for (int l = 0; l < nlev; ++l) { const int32_t n = H.sizes[l]; w.put(&n, 4); }
    for (int l = 0; l < nlev; ++l) {
        const bool has = l < (int)H.X.size() && H.X[l].size() == 3 * (size_t)H.sizes[l];
        const uint8_t flag = has ? 1 : 0;
        w.put(&flag, 1);
        if (has) w.put(H.X[l].data(), H.X[l].size() * sizeof(double));
    }
    for (int l = 0; l + 1 < nlev; ++l) {
        w.put(H.pcols[l].data(), H.pcols[l].size() * sizeof(int32_t));
        w.put(H.pw[l].data(), H.pw[l].size() * sizeof(double));
        w.put(H.stats[l].data(), 8 * sizeof(double));
    }
    const uint64_t sum = w.h;
    if (w.ok && std::fwrite(&sum, 8, 1, f) != 1) w.ok = false;
    if (std::fclose(f) != 0) w.ok = false;
    if (!w.ok) err = std::string("write to ") + path + " failed";
    return w.ok;
}

bool hier_read(const char *path, HierHost &H, std::string &err) {
    FILE *f = std::fopen(path, "rb");
    if (!f) { err = std::string("cannot open ") + path; return false; }
    Reader r{f};
    auto bad = [&](const std::string &m) { std::fclose(f); err = m; return false; };
    char magic[8];
    if (!r.get(magic, 8) || std::memcmp(magic, kMagic, 8) != 0) return bad("not a hierarchy file (magic or version)");
    int32_t nlev = 0;
    if (!r.get(&nlev, 4) || nlev < 1 || nlev > 64) return bad("bad level count");
    H = HierHost();
    H.nlev = nlev;
    H.sizes.resize(nlev);
    for (int l = 0; l < nlev; ++l) {
        int32_t n = 0;
        if (!r.get(&n, 4) || n < 1) return bad("bad level size");
        H.sizes[l] = n;
    }
    H.X.resize(nlev);
    for (int l = 0; l < nlev; ++l) {
        uint8_t flag = 0;
        if (!r.get(&flag, 1) || flag > 1) return bad("bad position flag");
        if (flag) {
            H.X[l].resize(3 * (size_t)H.sizes[l]);
            if (!r.get(H.X[l].data(), H.X[l].size() * sizeof(double))) return bad("file truncated");
        }
    }
    H.pcols.resize(nlev - 1);
    H.pw.resize(nlev - 1);
    H.stats.resize(nlev - 1);
    for (int l = 0; l + 1 < nlev; ++l) {
        const size_t m = 3 * (size_t)H.sizes[l];
        H.pcols[l].resize(m);
        H.pw[l].resize(m);
        if (!r.get(H.pcols[l].data(), m * sizeof(int32_t)) || !r.get(H.pw[l].data(), m * sizeof(double)) ||
            !r.get(H.stats[l].data(), 8 * sizeof(double)))
            return bad("file truncated");
    }
    const uint64_t want = r.h;
    uint64_t sum = 0;
    if (std::fread(&sum, 8, 1, f) != 1) return bad("file truncated (no checksum)");
    if (sum != want) return bad("checksum mismatch");
    char extra;
    if (std::fread(&extra, 1, 1, f) == 1) return bad("trailing bytes after the checksum");
    std::fclose(f);
    // the same checks as prolongations given by a caller
    for (int l = 0; l + 1 < nlev; ++l) {
        const int n = H.sizes[l], nc = H.sizes[l + 1];
        for (int i = 0; i < n; ++i) {
            bool any = false;
            for (int c = 0; c < 3; ++c) {
                const int32_t col = H.pcols[l][3 * (size_t)i + c];
                const double w = H.pw[l][3 * (size_t)i + c];
                if (col >= nc || !std::isfinite(w) || w < 0.0 || (col < 0 && w != 0.0)) {
                    err = "prolongation entry out of range at level " + std::to_string(l);
                    return false;
                }
                any = any || (col >= 0 && w > 0.0);
            }
            if (!any) {
                err = "prolongation row " + std::to_string(i) + " of level " + std::to_string(l) + " has no weight";
                return false;
            }
        }
    }
    return true;
}

}  // namespace smg
