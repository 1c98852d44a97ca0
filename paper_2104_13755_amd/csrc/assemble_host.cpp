// Host assembly of the cotangent Laplacian and the lumped mass on the CSR
// pattern {diagonal} U {mesh edges} (for systems assembled once on the host;
// the device assembly k_assemble serves changing coefficients).
//   L_ij = -1/2 (cot alpha_ij + cot beta_ij) over the faces at edge (i, j),
//          one term on a boundary edge;   L_ii = -sum_{j != i} L_ij;
//   M_ii = sum of the areas of the faces at i, divided by 3.
// Faces are visited one by one and each corner's cotangent is scattered to
// the edge it faces (the device kernel instead gathers per row).
#include <cmath>
#include <cstdint>
#include <string>

#include "hier.h"

namespace smg {

bool host_assemble(const double *V, int n, const int32_t *F, int m, const int32_t *rowptr, const int32_t *cols,
                   double *L, double *M, std::string &err) {
    const int64_t nnz = rowptr[n];
    for (int64_t p = 0; p < nnz; ++p) L[p] = 0.0;
    for (int i = 0; i < n; ++i) M[i] = 0.0;
    // position of column c in row r (columns ascending), -1 if absent
    auto at = [&](int r, int c) -> int64_t {
        int64_t lo = rowptr[r], hi = rowptr[r + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (cols[mid] < c) lo = mid + 1; else hi = mid;
        }
        return (lo < rowptr[r + 1] && cols[lo] == c) ? lo : -1;
    };
    for (int f = 0; f < m; ++f) {
        const int32_t *t = F + 3 * (size_t)f;
        double area2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const int o = t[c], a = t[(c + 1) % 3], b = t[(c + 2) % 3];
            const double u[3] = {V[3 * a] - V[3 * o], V[3 * a + 1] - V[3 * o + 1], V[3 * a + 2] - V[3 * o + 2]};
            const double w[3] = {V[3 * b] - V[3 * o], V[3 * b + 1] - V[3 * o + 1], V[3 * b + 2] - V[3 * o + 2]};
            const double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2],
                         cz = u[0] * w[1] - u[1] * w[0];
            const double cn = std::sqrt(cx * cx + cy * cy + cz * cz);
            if (!(cn > 0.0)) { err = "degenerate face " + std::to_string(f); return false; }
            const double cot = (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) / cn;
            const int64_t pab = at(a, b), pba = at(b, a);
            if (pab < 0 || pba < 0) { err = "edge of face " + std::to_string(f) + " missing from the pattern"; return false; }
            L[pab] += -0.5 * cot;
            L[pba] += -0.5 * cot;
            if (c == 0) area2 = cn;
        }
        for (int c = 0; c < 3; ++c) M[t[c]] += area2 / 6.0;
    }
    for (int i = 0; i < n; ++i) {
        const int64_t d = at(i, i);
        if (d < 0) { err = "diagonal of row " + std::to_string(i) + " missing from the pattern"; return false; }
        double off = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            if (p != d) off += L[p];
        L[d] = -off;
    }
    return true;
}

}  // namespace smg
