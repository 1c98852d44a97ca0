// HIP kernels (gfx950, wave64) of the surface-multigrid V-cycle.
//
// Layout: every smoothed level stores the off-diagonal part of A_l in a
// sliced-ELL format with 64-row slices (one wavefront per slice, one lane per
// row, slot (lane, e) at slice_off + 64 e + lane), so the matrix stream of a
// sweep is read fully coalesced with no cross-lane reduction.  Rows are
// permuted color-major and slices never straddle two colors, so one color of a
// multicolor Gauss-Seidel sweep (App. A) is one contiguous slice range.
// Vectors with K right-hand sides are row-major n x K.
#include "kernels.h"

#include <hip/hip_ext.h>

#include <cmath>

namespace smg {
namespace {

constexpr int kBlock = 256;
constexpr int kGsBlock = 64;   // one wavefront per block: a color's slices spread over more compute units

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so neighbouring slices share an L2.
__device__ __forceinline__ int xcd_block(int bid, int nblk) {
    const int q = nblk >> 3, r = nblk & 7;
    const int x = bid & 7, i = bid >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Sum over aligned groups of g adjacent lanes (g = 1, 2, 4 or 8, the same
// in the whole wavefront) by DPP lane swaps: lane ^ 1 and lane ^ 2 inside each
// quad, then the mirror of each 8-lane half-row (lane i <-> 7 - i), so every
// lane of a group ends with the group's sum, ((a0 + a1) + (a2 + a3)) + the
// other quad's.  All lanes of a group must be active.
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_mov(T v) {
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
    } else {
        const long long u = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
        return __hiloint2double(hi, lo);
    }
}
template <int K, typename T>
__device__ __forceinline__ void group_sum(T (&acc)[K], int g) {
    constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141;   // quad_perm [1,0,3,2], [2,3,0,1]
    if (g >= 2)
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += dpp_mov<kXor1>(acc[q]);
    if (g >= 4)
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += dpp_mov<kXor2>(acc[q]);
    if (g >= 8)
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += dpp_mov<kHalfMirror>(acc[q]);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Loads and stores through pointers read from descriptors in memory, marked
// global explicitly (the compiler cannot infer it and would use flat accesses).
template <typename T>
__device__ __forceinline__ T gld(const T *p, size_t i) {
    return ((const __attribute__((address_space(1))) T *)p)[i];
}
template <typename T>
__device__ __forceinline__ void gst(T *p, size_t i, T v) {
    ((__attribute__((address_space(1))) T *)p)[i] = v;
}

// ---------------------------------------------------------------- relaxation
// Sum of one row's off-diagonal products over the lpr lanes of its group.
// Rounds are taken in chunks whose loads are all issued before any is used:
// full chunks of 8, then one chunk of 2, 4 or 8 for the rest (a round past w
// re-reads the last one with weight 0), so a row costs one matrix round trip
// and one gather round trip per chunk.  Products are added in round order.
template <int CH, int K, typename T>
__device__ __forceinline__ void gather_chunk(int o, int e, int w, const int32_t *__restrict__ cols,
                                             const T *__restrict__ vals, const T *__restrict__ x,
                                             T (&acc)[K]) {
    int c[CH];
    T a[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const int at = o + 64 * min(e + u, w - 1);
        c[u] = cols[at];
        a[u] = vals[at] * (e + u < w ? T(1) : T(0));   // padding rounds weigh 0 (values are finite)
    }
    T xv[CH][K];
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int q = 0; q < K; ++q) xv[u][q] = x[(size_t)c[u] * K + q];
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += a[u] * xv[u][q];
}
template <int K, typename T>
__device__ __forceinline__ void row_gather(int o, int w, int lpr, const int32_t *__restrict__ cols,
                                           const T *__restrict__ vals, const T *__restrict__ x,
                                           T (&acc)[K]) {
    int e = 0;
    for (; e + 8 <= w; e += 8) gather_chunk<8, K, T>(o, e, w, cols, vals, x, acc);
    const int rem = w - e;
    if (rem > 0) {
        if (rem <= 2) gather_chunk<2, K, T>(o, e, w, cols, vals, x, acc);
        else if (rem <= 4) gather_chunk<4, K, T>(o, e, w, cols, vals, x, acc);
        else gather_chunk<8, K, T>(o, e, w, cols, vals, x, acc);
    }
    group_sum<K>(acc, lpr);
}

// x_i <- (b_i - sum_{j != i} A_ij x_j) / A_ii for every row i of one color.
template <int K, typename T>
__global__ __launch_bounds__(kGsBlock) void k_gs_color(int s_begin, int s_end, int lpr,
                                                     const int32_t *__restrict__ slice_row0,
                                                     const int32_t *__restrict__ slice_off,
                                                     const int32_t *__restrict__ cols,
                                                     const T *__restrict__ vals,
                                                     const T *__restrict__ diag,
                                                     const T *__restrict__ b, T *__restrict__ x) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = s_begin + blk * (kGsBlock / 64) + (threadIdx.x >> 6);
    if (s >= s_end) return;
    const int lane = threadIdx.x & 63;
    // the slice's bounds, diagonal and b are loaded together; lanes past the
    // slice's last row work on (padding) data of its first row and store nothing
    const int r0 = slice_row0[s], r1 = slice_row0[s + 1];
    const int o0 = slice_off[s], o1 = slice_off[s + 1];
    const int row = r0 + (lane >> __builtin_ctz(lpr));
    const bool valid = row < r1;
    const int rw = valid ? row : r0;
    const int w = (o1 - o0) >> 6;
    const T d = diag[rw];
    T bq[K], acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { bq[q] = b[(size_t)rw * K + q]; acc[q] = T(0); }
    row_gather<K, T>(o0 + lane, w, lpr, cols, vals, x, acc);
    if (valid && (lane & (lpr - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) x[(size_t)row * K + q] = (bq[q] - acc[q]) / d;
    }
}

// The same update for a color whose slices all hold w rounds: a slice's rows
// and slots follow from its index, so the matrix, diagonal and b loads are
// issued together (one round trip fewer than through the slice table).
template <int K, typename T>
__global__ __launch_bounds__(kGsBlock) void k_gs_color_w(int nsl, int row0, int row_end, int off0, int w,
                                                       int lpr, const int32_t *__restrict__ cols,
                                                       const T *__restrict__ vals,
                                                       const T *__restrict__ diag,
                                                       const T *__restrict__ b, T *__restrict__ x) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = blk * (kGsBlock / 64) + (threadIdx.x >> 6);
    if (s >= nsl) return;
    const int lane = threadIdx.x & 63;
    const int lg = __builtin_ctz(lpr);
    const int r0 = row0 + (s << (6 - lg));
    const int row = r0 + (lane >> lg);
    const bool valid = row < row_end;
    const int rw = valid ? row : r0;
    const T d = diag[rw];
    T bq[K], acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { bq[q] = b[(size_t)rw * K + q]; acc[q] = T(0); }
    row_gather<K, T>(off0 + s * 64 * w + lane, w, lpr, cols, vals, x, acc);
    if (valid && (lane & (lpr - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) x[(size_t)row * K + q] = (bq[q] - acc[q]) / d;
    }
}

// Per-block column partials: partial[blk][q] = sum of v[q], [K + q] = max of m[q].
template <int K>
__device__ __forceinline__ void block_partials(const double (&v)[K], const double (&m)[K],
                                               double *__restrict__ partial) {
    __shared__ double red[2 * K][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double a = wave_sum(v[q]), b = wave_max(m[q]);
        if (lane == 0) { red[q][wv] = a; red[K + q][wv] = b; }
    }
    __syncthreads();
    if (threadIdx.x < K) {
        const int q = threadIdx.x;
        double a = 0.0, b = 0.0;
        for (int i = 0; i < kBlock / 64; ++i) { a += red[q][i]; b = fmax(b, red[K + q][i]); }
        partial[(size_t)blockIdx.x * 2 * K + q] = a;
        partial[(size_t)blockIdx.x * 2 * K + K + q] = b;
    }
}

// Damped Jacobi (the alternative relaxation of App. "Ablation Study"):
// xo_i = x_i + omega (b_i - sum_j A_ij x_j) / A_ii for every row at once.
template <int K, typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi(int nslices, int lpr, const int32_t *__restrict__ slice_row0,
                                                   const int32_t *__restrict__ slice_off,
                                                   const int32_t *__restrict__ cols,
                                                   const T *__restrict__ vals, const T *__restrict__ diag,
                                                   const T *__restrict__ b, const T *__restrict__ x,
                                                   T *__restrict__ xo, const double *__restrict__ omega_l) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = blk * (kBlock / 64) + (threadIdx.x >> 6);
    if (s >= nslices) return;
    const int lane = threadIdx.x & 63;
    const int r0 = slice_row0[s], r1 = slice_row0[s + 1];
    const int o0 = slice_off[s], o1 = slice_off[s + 1];
    const int row = r0 + (lane >> __builtin_ctz(lpr));
    const bool valid = row < r1;
    const int rw = valid ? row : r0;
    const int w = (o1 - o0) >> 6;
    const T d = diag[rw];
    const T omega = (T)*omega_l;
    T bq[K], xi[K], acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        bq[q] = b[(size_t)rw * K + q];
        xi[q] = x[(size_t)rw * K + q];
        acc[q] = T(0);
    }
    row_gather<K, T>(o0 + lane, w, lpr, cols, vals, x, acc);
    if (valid && (lane & (lpr - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) xo[(size_t)row * K + q] = xi[q] + omega * (bq[q] - (acc[q] + d * xi[q])) / d;
    }
}

// out = a x + b y (split Galerkin levels, App. E)
__global__ __launch_bounds__(kBlock) void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                                                  const double *__restrict__ y, double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) out[t] = a * x[t] + b * y[t];
}

// Reduced system of Dirichlet conditions (App. B), one thread per unknown
// row i: A_uu values in row order (the full row's entries whose column is
// unknown) and rhs = b_i - sum over known columns j of A_ij x_j.
template <int K>
__global__ __launch_bounds__(kBlock) void k_dirichlet_reduce(int nu, const int32_t *__restrict__ uidx,
                                                             const int32_t *__restrict__ rowptr,
                                                             const int32_t *__restrict__ cols,
                                                             const double *__restrict__ vals,
                                                             const uint8_t *__restrict__ known,
                                                             const double *__restrict__ x,
                                                             const double *__restrict__ b,
                                                             const int32_t *__restrict__ uptr,
                                                             double *__restrict__ uvals, double *__restrict__ rhs) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nu) return;
    const int i = uidx[r];
    double acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = b[(size_t)i * K + q];
    int o = uptr[r];
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int j = cols[p];
        const double a = vals[p];
        if (known[j]) {
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] -= a * x[(size_t)j * K + q];
        } else {
            if (o < uptr[r + 1]) uvals[o] = a;   // a pattern from another mask writes nothing past the row
            ++o;
        }
    }
#pragma unroll
    for (int q = 0; q < K; ++q) rhs[(size_t)r * K + q] = acc[q];
}

// The first Jacobi sweep from a zero iterate: xo = omega b / A_ii (no
// gathers; the same operations as a sweep with x = 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_first(int64_t nk, int k, const T *__restrict__ diag,
                                                         const T *__restrict__ b, T *__restrict__ xo,
                                                         const double *__restrict__ omega_l) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nk) return;
    const T omega = (T)*omega_l;
    xo[t] = omega * (b[t] - T(0)) / diag[t / k];
}

// Estimate of the largest eigenvalue of D^{-1} A for the Jacobi factor:
// v_r = frac(phi^-1 (natural index + 1)) - 1/2, then power steps
// v <- D^{-1} A v (FINAL = false), then partials of v . A v and v . D v
// (FINAL = true, two sums per block).
__global__ __launch_bounds__(kBlock) void k_power_start(int n, const int32_t *__restrict__ perm,
                                                        double *__restrict__ v) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    const double i = (double)perm[r] + 1.0;
    const double t = 0.6180339887498949 * i;
    v[r] = (t - floor(t)) - 0.5;
}

template <bool FINAL>
__global__ __launch_bounds__(kBlock) void k_power_step(int nslices, int lpr, const int32_t *__restrict__ slice_row0,
                                                       const int32_t *__restrict__ slice_off,
                                                       const int32_t *__restrict__ cols,
                                                       const double *__restrict__ vals,
                                                       const double *__restrict__ diag,
                                                       const double *__restrict__ v, double *__restrict__ vo,
                                                       double *__restrict__ partial) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = blk * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double sums[2] = {0.0, 0.0}, zero[2] = {0.0, 0.0};
    if (s < nslices) {
        const int r0 = slice_row0[s], r1 = slice_row0[s + 1];
        const int o0 = slice_off[s], o1 = slice_off[s + 1];
        const int row = r0 + (lane >> __builtin_ctz(lpr));
        const bool valid = row < r1;
        const int rw = valid ? row : r0;
        const int w = (o1 - o0) >> 6;
        const double d = diag[rw], vi = v[rw];
        double acc[1] = {0.0};
        row_gather<1, double>(o0 + lane, w, lpr, cols, vals, v, acc);
        if (valid && (lane & (lpr - 1)) == 0) {
            const double av = acc[0] + d * vi;
            if (FINAL) { sums[0] = vi * av; sums[1] = vi * d * vi; }
            else vo[row] = av / d;
        }
    }
    if (FINAL) block_partials<2>(sums, zero, partial);
}

// omega_l = 2 / (1 + lambda), lambda = (v . A v) / (v . D v)
__global__ void k_power_omega(const double *__restrict__ sums, double *__restrict__ omega_l) {
    if (threadIdx.x == 0) *omega_l = 2.0 / (1.0 + sums[0] / sums[1]);
}

// ------------------------------------------------------------------ residual
// r = b - A x over all slices; optional per-block column (sum r^2, max |r|).
template <int K, typename T, bool NORM>
__global__ __launch_bounds__(kBlock) void k_residual(int nslices, int lpr,
                                                     const int32_t *__restrict__ slice_row0,
                                                     const int32_t *__restrict__ slice_off,
                                                     const int32_t *__restrict__ cols,
                                                     const T *__restrict__ vals,
                                                     const T *__restrict__ diag,
                                                     const T *__restrict__ b,
                                                     const T *__restrict__ x, T *__restrict__ r,
                                                     double *__restrict__ partial,
                                                     const int32_t *__restrict__ order) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int w0 = blk * (kBlock / 64) + (threadIdx.x >> 6);
    const int s = (order != nullptr && w0 < nslices) ? order[w0] : w0;
    const int lane = threadIdx.x & 63;
    double sq[K], mx[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { sq[q] = 0.0; mx[q] = 0.0; }
    if (s < nslices) {
        const int r0 = slice_row0[s], r1 = slice_row0[s + 1];
        const int o0 = slice_off[s], o1 = slice_off[s + 1];
        const int row = r0 + (lane >> __builtin_ctz(lpr));
        const bool valid = row < r1;
        const int rw = valid ? row : r0;
        {
            const int w = (o1 - o0) >> 6;
            const T d = diag[rw];
            T bq[K], xo[K], acc[K];
#pragma unroll
            for (int q = 0; q < K; ++q) {
                bq[q] = b[(size_t)rw * K + q];
                xo[q] = x[(size_t)rw * K + q];
                acc[q] = T(0);
            }
            row_gather<K, T>(o0 + lane, w, lpr, cols, vals, x, acc);
            if (valid && (lane & (lpr - 1)) == 0) {
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    const T rv = bq[q] - (acc[q] + d * xo[q]);
                    r[(size_t)row * K + q] = rv;
                    if (NORM) { sq[q] = (double)rv * (double)rv; mx[q] = fabs((double)rv); }
                }
            }
        }
    }
    if (NORM) {
        __shared__ double red[2 * K][kBlock / 64];
        const int wv = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const double a = wave_sum(sq[q]);
            const double m = wave_max(mx[q]);
            if (lane == 0) { red[q][wv] = a; red[K + q][wv] = m; }
        }
        __syncthreads();
        if (threadIdx.x < K) {
            const int q = threadIdx.x;
            double a = 0.0, m = 0.0;
            for (int i = 0; i < kBlock / 64; ++i) { a += red[q][i]; m = fmax(m, red[K + q][i]); }
            partial[(size_t)blockIdx.x * 2 * K + q] = a;
            partial[(size_t)blockIdx.x * 2 * K + K + q] = m;
        }
    }
}

// -------------------------------------- preconditioned CG on level 0
// ap = A p over every slice (diagonal + sliced ELL); partials of p . ap.
template <int K>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(int nslices, int lpr, const int32_t *__restrict__ slice_row0,
                                                    const int32_t *__restrict__ slice_off,
                                                    const int32_t *__restrict__ cols,
                                                    const double *__restrict__ vals,
                                                    const double *__restrict__ diag,
                                                    const double *__restrict__ p, double *__restrict__ ap,
                                                    double *__restrict__ partial,
                                                    const int32_t *__restrict__ order) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int w0 = blk * (kBlock / 64) + (threadIdx.x >> 6);
    const int s = (order != nullptr && w0 < nslices) ? order[w0] : w0;
    const int lane = threadIdx.x & 63;
    double pq[K], zero[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { pq[q] = 0.0; zero[q] = 0.0; }
    if (s < nslices) {
        const int r0 = slice_row0[s], r1 = slice_row0[s + 1];
        const int o0 = slice_off[s], o1 = slice_off[s + 1];
        const int row = r0 + (lane >> __builtin_ctz(lpr));
        const bool valid = row < r1;
        const int rw = valid ? row : r0;
        const int w = (o1 - o0) >> 6;
        const double d = diag[rw];
        double pi[K], acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) { pi[q] = p[(size_t)rw * K + q]; acc[q] = 0.0; }
        row_gather<K, double>(o0 + lane, w, lpr, cols, vals, p, acc);
        if (valid && (lane & (lpr - 1)) == 0) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const double v = acc[q] + d * pi[q];
                ap[(size_t)row * K + q] = v;
                pq[q] = pi[q] * v;
            }
        }
    }
    block_partials<K>(pq, zero, partial);
}

// alpha = (r.z) / (p.Ap) per column (0 when p.Ap is 0); x += alpha p,
// r -= alpha Ap; partials of r.r and max |r|.
template <int K>
__global__ __launch_bounds__(kBlock) void k_cg_update(int n, const double *__restrict__ rz,
                                                      const double *__restrict__ pap,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ ap, double *__restrict__ x,
                                                      double *__restrict__ r, double *__restrict__ partial) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double sq[K], mx[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { sq[q] = 0.0; mx[q] = 0.0; }
    if (i < n) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const double den = pap[q];
            const double al = den != 0.0 ? rz[q] / den : 0.0;
            const size_t t = (size_t)i * K + q;
            x[t] += al * p[t];
            const double rv = r[t] - al * ap[t];
            r[t] = rv;
            sq[q] = rv * rv;
            mx[q] = fabs(rv);
        }
    }
    block_partials<K>(sq, mx, partial);
}

// z as the preconditioner left it: FP64 iterate, or the FP32 iterate of the
// scaled system times the scale (max |r| per column, as in refinement)
template <int K, bool Z32>
__device__ __forceinline__ double cg_z(size_t t, int q, const double *z64, const float *z32,
                                       const double *zscale) {
    if constexpr (Z32) return (double)z32[t] * zscale[K + q];
    else return z64[t];
}

// partials of r . z
template <int K, bool Z32>
__global__ __launch_bounds__(kBlock) void k_cg_dot(int n, const double *__restrict__ r,
                                                   const double *__restrict__ z64, const float *__restrict__ z32,
                                                   const double *__restrict__ zscale, double *__restrict__ partial) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double v[K], zero[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { v[q] = 0.0; zero[q] = 0.0; }
    if (i < n)
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const size_t t = (size_t)i * K + q;
            v[q] = r[t] * cg_z<K, Z32>(t, q, z64, z32, zscale);
        }
    block_partials<K>(v, zero, partial);
}

// p = z + beta p with beta = rz_new / rz_old (0 when rz_old is 0; p = z when
// rz_old is null); the preconditioner's iterate is cleared for its next use.
template <int K, bool Z32>
__global__ __launch_bounds__(kBlock) void k_cg_direction(int n, const double *__restrict__ rz_new,
                                                         const double *__restrict__ rz_old,
                                                         double *__restrict__ z64, float *__restrict__ z32,
                                                         const double *__restrict__ zscale,
                                                         double *__restrict__ p) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * K) return;
    const int q = (int)(t % K);
    const double z = cg_z<K, Z32>((size_t)t, q, z64, z32, zscale);
    if (rz_old) {
        const double den = rz_old[q];
        const double beta = den != 0.0 ? rz_new[q] / den : 0.0;
        p[t] = z + beta * p[t];
    } else {
        p[t] = z;
    }
    if constexpr (Z32) z32[t] = 0.0f;
    else z64[t] = 0.0;
}

// --------------------------------------------------------------- transfers
// rc_a = sum_{i} R_ai r_i with R = P^T (gather; deterministic order)
template <int K, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(int nc, int lr, const int32_t *__restrict__ rs_off,
                                                     const int32_t *__restrict__ rs_idx,
                                                     const T *__restrict__ rw,
                                                     const T *__restrict__ r, T *__restrict__ rc,
                                                     T *__restrict__ xc, const int32_t *__restrict__ order) {
    constexpr int CH = 8;
    const int t = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int w0 = t >> 6, lane = t & 63, rps = 64 / lr;
    if (w0 * rps >= nc) return;   // whole wavefronts leave together
    const int s = order != nullptr ? order[w0] : w0;
    const int a = s * rps + lane / lr, j = lane & (lr - 1);
    const int o0 = rs_off[s] + lane, w = (rs_off[s + 1] - rs_off[s]) >> 6;
    T acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = T(0);
    for (int k0 = 0; k0 < w; k0 += CH) {   // all loads of a chunk in flight; rounds past w weigh 0
        int i[CH];
        T wt[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int at = o0 + 64 * min(k0 + u, w - 1);
            i[u] = rs_idx[at];
            wt[u] = k0 + u < w ? rw[at] : T(0);
        }
        T rv[CH][K];
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
            for (int q = 0; q < K; ++q) rv[u][q] = r[(size_t)i[u] * K + q];
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] += wt[u] * rv[u][q];
    }
    group_sum<K>(acc, lr);
    if (a < nc && j == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            rc[(size_t)a * K + q] = acc[q];
            if (xc) xc[(size_t)a * K + q] = T(0);
        }
    }
}

// x_i += sum_m P_im e_{c_im}
template <int K, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(int n, const int32_t *__restrict__ pc,
                                                        const T *__restrict__ pw,
                                                        const T *__restrict__ e,
                                                        T *__restrict__ x) {
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    T acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = T(0);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int c = pc[(size_t)m * n + i];
        const T w = pw[(size_t)m * n + i];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += w * e[(size_t)c * K + q];
    }
#pragma unroll
    for (int q = 0; q < K; ++q) x[(size_t)i * K + q] += acc[q];
}

// --------------------------------------------------------------- reductions
template <int K>
__global__ __launch_bounds__(kBlock) void k_colnorm_partial(const double *__restrict__ v, int n,
                                                            double *__restrict__ partial) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ double red[2 * K][kBlock / 64];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double a = i < n ? v[(size_t)i * K + q] : 0.0;
        const double s = wave_sum(a * a), m = wave_max(fabs(a));
        if (lane == 0) { red[q][wv] = s; red[K + q][wv] = m; }
    }
    __syncthreads();
    if (threadIdx.x < K) {
        const int q = threadIdx.x;
        double a = 0.0, m = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) { a += red[q][w]; m = fmax(m, red[K + q][w]); }
        partial[(size_t)blockIdx.x * 2 * K + q] = a;
        partial[(size_t)blockIdx.x * 2 * K + K + q] = m;
    }
}

// one block: out[q] = sum_b partial[b][q], out[K+q] = max_b partial[b][K+q]
// (each thread folds every 1024th block, then wavefront shuffles, then the
// 16 wavefronts in order: a fixed summation order, one barrier)
template <int K>
__global__ __launch_bounds__(1024) void k_reduce_partial(const double *__restrict__ partial, int nblk,
                                                         double *__restrict__ out, double *__restrict__ host_out,
                                                         double seq) {
    __shared__ double red[2 * K][16];
    __shared__ double fin[2 * K];
    double a[K], m[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { a[q] = 0.0; m[q] = 0.0; }
    for (int b = threadIdx.x; b < nblk; b += 1024) {
        const double *pb = partial + (size_t)b * 2 * K;
#pragma unroll
        for (int q = 0; q < K; ++q) { a[q] += pb[q]; m[q] = fmax(m[q], pb[K + q]); }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double sa = wave_sum(a[q]), sm = wave_max(m[q]);
        if (lane == 0) { red[q][wv] = sa; red[K + q][wv] = sm; }
    }
    __syncthreads();
    if (threadIdx.x < 2 * K) {
        const int j = threadIdx.x;
        double v = 0.0;
        for (int w = 0; w < 16; ++w) v = j < K ? v + red[j][w] : fmax(v, red[j][w]);
        fin[j] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < 2 * K; ++j) out[j] = fin[j];
        if (host_out) {   // the host reads the norms once it sees seq
            for (int j = 0; j < 2 * K; ++j) host_out[j] = fin[j];
            __threadfence_system();
            host_out[2 * K] = seq;
        }
    }
}

// ---------------------------------------------------------------- coarsest
// Right-looking dense Cholesky of a column-major n x n matrix (lower part
// used), one workgroup.  flag <- 1 if a pivot is not positive.
__global__ __launch_bounds__(1024) void k_cholesky(double *__restrict__ A, int n,
                                                   int *__restrict__ flag) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (threadIdx.x == 0) {
            const double d = A[(size_t)j * n + j];
            if (!(d > 0.0)) { bad = 1; *flag = 1; }
            else A[(size_t)j * n + j] = sqrt(d);
        }
        __syncthreads();
        if (bad) return;
        const double djj = A[(size_t)j * n + j];
        for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[(size_t)j * n + i] /= djj;
        __syncthreads();
        const int m = n - j - 1;
        const int total = m * m;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int i = j + 1 + t % m, c = j + 1 + t / m;
            if (i >= c) A[(size_t)c * n + i] -= A[(size_t)j * n + i] * A[(size_t)j * n + c];
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
        const int i = t % n, c = t / n;
        if (i < c) A[(size_t)c * n + i] = 0.0;
    }
}

// Blocked right-looking Cholesky A = G G^T (column-major n x n, lower
// triangle; upper triangle zeroed), one workgroup.  A panel of nb columns is
// factored in LDS (ld = rows of the panel), written back, and the trailing
// lower triangle receives the panel's rank-nb update in 2 x 2 register blocks.
__global__ __launch_bounds__(1024) void k_cholesky_blocked(double *__restrict__ A, int n, int nbmax,
                                                           int *__restrict__ flag) {
    extern __shared__ double pan[];
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += nbmax) {
        const int nb = min(nbmax, n - k0), m = n - k0;
        for (int t = tid; t < m * nb; t += nt) {
            const int i = t % m, c = t / m;
            pan[c * m + i] = A[(size_t)(k0 + c) * n + k0 + i];
        }
        __syncthreads();
        for (int j = 0; j < nb; ++j) {
            if (tid == 0) {
                const double d = pan[j * m + j];
                if (!(d > 0.0)) { bad = 1; *flag = 1; }
                else pan[j * m + j] = sqrt(d);
            }
            __syncthreads();
            if (bad) return;
            const double djj = pan[j * m + j];
            for (int i = j + 1 + tid; i < m; i += nt) pan[j * m + i] /= djj;
            __syncthreads();
            const int w = nb - j - 1;
            for (int t = tid; t < w * m; t += nt) {
                const int c = j + 1 + t / m, i = t % m;
                if (i >= c) pan[c * m + i] -= pan[j * m + i] * pan[j * m + c];
            }
            __syncthreads();
        }
        for (int t = tid; t < m * nb; t += nt) {
            const int i = t % m, c = t / m;
            if (i >= c) A[(size_t)(k0 + c) * n + k0 + i] = pan[c * m + i];
        }
        const int mt = m - nb;                       // trailing block rows/cols nb..m-1 of the panel frame
        const int nbk = (mt + 1) / 2;                // 2 x 2 blocks per side
        const int ntri = nbk * (nbk + 1) / 2;
        for (int b = tid; b < ntri; b += nt) {
            int bi = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
            while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
            while (bi * (bi + 1) / 2 > b) --bi;
            const int bc = b - bi * (bi + 1) / 2;
            const int i0 = nb + 2 * bi, c0 = nb + 2 * bc;
            const bool i1ok = i0 + 1 < m, c1ok = c0 + 1 < m;
            double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
            for (int q = 0; q < nb; ++q) {
                const double li0 = pan[q * m + i0], li1 = i1ok ? pan[q * m + i0 + 1] : 0.0;
                const double lc0 = pan[q * m + c0], lc1 = c1ok ? pan[q * m + c0 + 1] : 0.0;
                s00 += li0 * lc0; s01 += li0 * lc1; s10 += li1 * lc0; s11 += li1 * lc1;
            }
            double *col0 = A + (size_t)(k0 + c0) * n + k0, *col1 = col0 + n;
            col0[i0] -= s00;                                   // i0 >= c0 always
            if (i1ok) col0[i0 + 1] -= s10;
            if (c1ok && i0 >= c0 + 1) col1[i0] -= s01;
            if (c1ok && i1ok) col1[i0 + 1] -= s11;             // i0 + 1 >= c0 + 1
        }
        __syncthreads();
    }
    for (int t = tid; t < n * n; t += nt) {
        const int i = t % n, c = t / n;
        if (i < c) A[(size_t)c * n + i] = 0.0;
    }
}

// ------------------------------------------- blocked Cholesky on many CUs
// Right-looking A = G G^T (column-major, lower) in panels of kCholNb columns.
// Per panel, k_chol_panel factors the diagonal block in the registers of one
// wavefront per workgroup (row i in lane i, pivots and multipliers read from
// other lanes by v_readlane) and solves every row below it against that
// block (one thread per row); k_chol_update then updates the trailing lower
// triangle A22 -= L21 L21^T in 16 x 16 tiles, one wavefront per tile on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64, K = 4 per instruction).  A pivot
// <= 0 sets *flag and every later kernel returns at once.
constexpr int kCholNb = 32;
// coarsest levels up to this size are factored and inverted by the
// one-workgroup kernels (k_cholesky_blocked, k_tri_inverse_cols)
constexpr int kCoarseOneGroup = 96;
typedef double v4d_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)u, lane), hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __hiloint2double(hi, lo);
}

// Factor the b x b diagonal block at (k0, k0) in the registers of one
// wavefront: lane i holds row i (a[c] = A(k0 + i, k0 + c), c <= i; rows b..31
// are identity rows, so a ragged last block runs the same 32 steps).  Step j
// takes the pivot from lane j, scales column j and updates the columns right
// of it with L(c, j) read from lane c; nothing leaves the registers.  Leaves
// L11 row-major in T (zero above the diagonal, identity rows below b) and
// returns false on a pivot <= 0 (the same decision in every lane).
__device__ bool chol_block_regs(double *__restrict__ A, int n, int k0, int b, double *T) {
    const int lane = threadIdx.x & 63;
    double a[kCholNb];
#pragma unroll
    for (int c = 0; c < kCholNb; ++c)
    {   // in-bounds address for every lane, then a select (no branch)
        const double v = A[(size_t)(k0 + min(c, b - 1)) * n + k0 + min(lane, b - 1)];
        a[c] = (lane < b && c <= lane) ? v : (c == lane ? 1.0 : 0.0);
    }
    bool ok = true;
#pragma unroll
    for (int j = 0; j < kCholNb; ++j) {
        const double piv = readlane_f64(a[j], j);
        ok = ok && (piv > 0.0);
        const double d = sqrt(piv);
        a[j] = lane > j ? a[j] / d : (lane == j ? d : 0.0);
#pragma unroll
        for (int c = j + 1; c < kCholNb; ++c) a[c] -= a[j] * readlane_f64(a[j], c);
    }
    if (lane < kCholNb) {
#pragma unroll
        for (int c = 0; c < kCholNb; ++c) T[lane * kCholNb + c] = c <= lane ? a[c] : 0.0;
        if (blockIdx.x == 0 && lane < b) {   // the factored block back to A (lower part)
#pragma unroll
            for (int c = 0; c < kCholNb; ++c)
                if (c <= lane) A[(size_t)(k0 + c) * n + k0 + lane] = a[c];
        }
    }
    return ok;
}

// x L^T = a for one row held in registers (forward substitution against the
// row-major lower triangle T; rows of T past the block are identity rows, so
// x stays zero there): x_j = (a_j - sum_{p<j} L_jp x_p) / L_jj.  The same
// recurrence solves L x = w for one column of a right-hand side.
__device__ __forceinline__ void tri_solve_regs(double (&x)[kCholNb], const double *__restrict__ T) {
#pragma unroll
    for (int j = 0; j < kCholNb; ++j) {
        double s = x[j];
#pragma unroll
        for (int p = 0; p < j; ++p) s -= T[j * kCholNb + p] * x[p];
        x[j] = s / T[j * kCholNb + j];
        __builtin_amdgcn_sched_barrier(0);   // keep row j's loads of T from being hoisted: they would spill
    }
}

__global__ __launch_bounds__(256) void k_chol_panel(double *__restrict__ A, int n, int k0, int b,
                                                    int *__restrict__ flag) {
    __shared__ double T[kCholNb * kCholNb];
    __shared__ int good;
    if (*flag) return;
    // rows k0 + b .. n-1 of the panel: x L11^T = a, one thread per row.  Only
    // the last panel can be narrower than kCholNb, and it has no rows below.
    // Each thread's row is loaded before the diagonal block is factored (the
    // loads overlap the factorization; a thread past n loads row n-1 and
    // stores nothing).
    const int i = k0 + b + blockIdx.x * blockDim.x + threadIdx.x;
    const int ii = min(i, n - 1);
    double x[kCholNb];
    if (k0 + b < n) {
#pragma unroll
        for (int j = 0; j < kCholNb; ++j) x[j] = A[(size_t)(k0 + j) * n + ii];
    }
    if (threadIdx.x < 64) {
        const bool ok = chol_block_regs(A, n, k0, b, T);
        if (threadIdx.x == 0) good = ok ? 1 : 0;
    }
    __syncthreads();
    if (!good) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 1;
        return;
    }
    if (i >= n) return;
    tri_solve_regs(x, T);
#pragma unroll
    for (int j = 0; j < kCholNb; ++j) A[(size_t)(k0 + j) * n + i] = x[j];
}

// Lower-triangle tile index w -> (ti, tj), ti >= tj.
__device__ __forceinline__ void tri_tile(int w, int &ti, int &tj) {
    ti = (int)((sqrt(8.0 * w + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= w) ++ti;
    while (ti * (ti + 1) / 2 > w) --ti;
    tj = w - ti * (ti + 1) / 2;
}

// Trailing update of the lower triangle of rows / columns k0 + b..: one
// wavefront per 16 x 16 tile (more wavefronts in flight hide the operand
// loads better than 32 x 32 blocks per wavefront, measured).
__global__ __launch_bounds__(256) void k_chol_update(double *__restrict__ A, int n, int k0, int b, int ntile,
                                                     const int *__restrict__ flag) {
    if (*flag) return;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (w >= ntile) return;
    int ti, tj;
    tri_tile(w, ti, tj);
    const int r0 = k0 + b + 16 * ti, c0 = k0 + b + 16 * tj;
    const int lr = lane & 15, lk = lane >> 4;
    v4d_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int p = 0; p < b; p += 4) {
        const int kk = p + lk;
        const double a = (kk < b && r0 + lr < n) ? A[(size_t)(k0 + kk) * n + r0 + lr] : 0.0;
        const double bb = (kk < b && c0 + lr < n) ? A[(size_t)(k0 + kk) * n + c0 + lr] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
    }
    // lane holds D[lane / 16 + 4 q][lane % 16], q = 0..3 (the A operand: lane
    // holds A[lane % 16][lane / 16]; B: B[lane / 16][lane % 16])
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = r0 + lk + 4 * q, c = c0 + lr;
        if (r < n && c < n && r >= c) A[(size_t)c * n + r] -= acc[q];
    }
}

__global__ __launch_bounds__(256) void k_zero_upper(double *__restrict__ A, int n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int i = (int)(t % n), c = (int)(t / n);
    if (i < c) A[t] = 0.0;
}

// ----------------------------------- A_H^{-1} = G^{-T} G^{-1} on many CUs
// W = G^{-1} by a right-looking blocked forward substitution G W = I: per
// block row k (kCholNb rows), k_trinv_rows solves the diagonal block against
// those rows of the right-hand side (one thread per column), k_trinv_update
// subtracts G_ik W_k from every block row below (16 x 16 MFMA tiles).  Then
// k_inv_syrk forms the lower triangle of W^T W in 32 x 32 blocks (and mirrors
// it).
__global__ __launch_bounds__(256) void k_identity(double *__restrict__ W, int n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    W[t] = (t % n == t / n) ? 1.0 : 0.0;
}

// 256 columns of the block row per workgroup: the block (b rows x 256
// columns, each column's b values contiguous in W) is read and written
// coalesced through LDS, and each thread forward-substitutes one column in
// its registers against L_kk (row-major in LDS, identity rows past b).
__global__ __launch_bounds__(256) void k_trinv_rows(const double *__restrict__ G, double *__restrict__ W, int n,
                                                    int k0, int b) {
    __shared__ double T[kCholNb * kCholNb];
    __shared__ double X[256 * (kCholNb + 1)];   // column t at X[t * (kCholNb + 1)], padded against bank conflicts
    for (int t = threadIdx.x; t < kCholNb * kCholNb; t += blockDim.x) {
        const int i = t / kCholNb, j = t % kCholNb;
        T[t] = (i < b && j <= i) ? G[(size_t)(k0 + j) * n + k0 + i] : (i == j ? 1.0 : 0.0);
    }
    const int cbase = blockIdx.x * 256, ncol = min(256, k0 + b - cbase);
    for (int t = threadIdx.x; t < ncol * kCholNb; t += blockDim.x) {   // zero rows past b
        const int i = t % kCholNb, cc = t / kCholNb;
        X[cc * (kCholNb + 1) + i] = i < b ? W[(size_t)(cbase + cc) * n + k0 + i] : 0.0;
    }
    __syncthreads();
    if ((int)threadIdx.x < ncol) {
        double *xc = X + threadIdx.x * (kCholNb + 1);
        double x[kCholNb];
#pragma unroll
        for (int i = 0; i < kCholNb; ++i) x[i] = xc[i];
        tri_solve_regs(x, T);
#pragma unroll
        for (int i = 0; i < kCholNb; ++i) xc[i] = x[i];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ncol * b; t += blockDim.x) {
        const int i = t % b, cc = t / b;
        W[(size_t)(cbase + cc) * n + k0 + i] = X[cc * (kCholNb + 1) + i];
    }
}

// W[i][c] -= sum_p G[i][k0 + p] W[k0 + p][c], rows i >= k0 + b, columns
// c < k0 + b: one wavefront per 16 x 16 tile
__global__ __launch_bounds__(256) void k_trinv_update(const double *__restrict__ G, double *__restrict__ W, int n,
                                                      int k0, int b, int tcols, int ntile) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (w >= ntile) return;
    const int ti = w / tcols, tj = w % tcols;
    const int r0 = k0 + b + 16 * ti, c0 = 16 * tj;
    const int lr = lane & 15, lk = lane >> 4;
    v4d_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int p = 0; p < b; p += 4) {
        const int kk = p + lk;
        const double a = (kk < b && r0 + lr < n) ? G[(size_t)(k0 + kk) * n + r0 + lr] : 0.0;
        const double bb = (kk < b && c0 + lr < k0 + b) ? W[(size_t)(c0 + lr) * n + k0 + kk] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = r0 + lk + 4 * q, c = c0 + lr;
        if (r < n && c < k0 + b) W[(size_t)c * n + r] -= acc[q];
    }
}

// Ainv = W^T W: one wavefront per 32 x 32 block of the lower triangle (2 x 2
// MFMA tiles; the sum runs over rows m >= the block's first row, W being
// zero above its diagonal), each entry r >= c written with its mirror so
// that Ainv is exactly symmetric
__global__ __launch_bounds__(256) void k_inv_syrk(const double *__restrict__ W, double *__restrict__ Ainv, int n,
                                                  int ntile) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (w >= ntile) return;
    int ti, tj;
    tri_tile(w, ti, tj);
    const int i0 = 32 * ti, j0 = 32 * tj;
    const int lr = lane & 15, lk = lane >> 4;
    bool iok[2], jok[2];
    const double *wi[2], *wj[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = i0 + 16 * h + lr, c = j0 + 16 * h + lr;
        iok[h] = r < n;
        jok[h] = c < n;
        wi[h] = W + (size_t)min(r, n - 1) * n;
        wj[h] = W + (size_t)min(c, n - 1) * n;
    }
    v4d_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d_t{0.0, 0.0, 0.0, 0.0};
    int m = i0;
    for (; m + 8 <= n; m += 8) {   // two K-steps per round, loads first
        double a[2][2], bb[2][2];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                a[u][h] = iok[h] ? wi[h][m + 4 * u + lk] : 0.0;
                bb[u][h] = jok[h] ? wj[h][m + 4 * u + lk] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][i], bb[u][j], acc[i][j], 0, 0, 0);
    }
    for (; m < n; m += 4) {
        const int mm = m + lk;
        double a[2], bb[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            a[h] = (iok[h] && mm < n) ? wi[h][mm] : 0.0;
            bb[h] = (jok[h] && mm < n) ? wj[h][mm] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = i0 + 16 * i + lk + 4 * q, c = j0 + 16 * j + lr;   // sum_m W[m][r] W[m][c]
                if (r < n && c < n && r >= c) {
                    Ainv[(size_t)c * n + r] = acc[i][j][q];
                    Ainv[(size_t)r * n + c] = acc[i][j][q];
                }
            }
}

// W = G^{-1} one column per wavefront: forward substitution G w = e_c in
// column order (w_k /= G_kk, then w_i -= G_ik w_k below), w kept in LDS.
__global__ __launch_bounds__(256) void k_tri_inverse_cols(const double *__restrict__ G, int n,
                                                          double *__restrict__ W) {
    extern __shared__ double wb[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + wv;
    if (c >= n) return;
    double *w = wb + (size_t)wv * n;
    for (int i = lane; i < n; i += 64) w[i] = i == c ? 1.0 : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int k = c; k < n; ++k) {
        const double wk = w[k] / G[(size_t)k * n + k];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lane == 0) w[k] = wk;
        for (int i = k + 1 + lane; i < n; i += 64) w[i] -= G[(size_t)k * n + i] * wk;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    for (int i = lane; i < n; i += 64) W[(size_t)c * n + i] = i >= c ? w[i] : 0.0;
}

// W = G^{-1} for the lower-triangular Cholesky factor G (column-major), one
// workgroup, right-looking: start from W = I, then for each row j scale row j
// by 1/G_jj and eliminate it from the rows below (parallel over the
// (row, column) pairs of the trailing block).
__global__ __launch_bounds__(1024) void k_tri_inverse(const double *__restrict__ G, int n,
                                                      double *__restrict__ W) {
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) W[t] = (t % n == t / n) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double inv = 1.0 / G[(size_t)j * n + j];
        for (int c = threadIdx.x; c <= j; c += blockDim.x) W[(size_t)c * n + j] *= inv;
        __syncthreads();
        const int rows = n - j - 1, cols = j + 1;
        for (int t = threadIdx.x; t < rows * cols; t += blockDim.x) {
            const int i = j + 1 + t % rows, c = t / rows;
            W[(size_t)c * n + i] -= G[(size_t)j * n + i] * W[(size_t)c * n + j];
        }
        __syncthreads();
    }
}

// A^{-1} = W^T W (symmetric), entry (i, j) = sum_{m >= max(i,j)} W_mi W_mj.
__global__ __launch_bounds__(kBlock) void k_inverse_product(const double *__restrict__ W, int n,
                                                            double *__restrict__ Ainv) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int i = (int)(t % n), j = (int)(t / n);
    double s = 0.0;
    for (int m = max(i, j); m < n; ++m) s += W[(size_t)i * n + m] * W[(size_t)j * n + m];   // W_mi W_mj
    Ainv[(size_t)j * n + i] = s;
}

// x = A_H^{-1} b (the coarsest direct solve), one wavefront per row, FP64
// accumulation; A_H^{-1} is exactly symmetric (each entry is the same sum of
// the same products for (i, j) and (j, i)), so row i is read contiguously.
template <int K, typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_coarse_apply(const double *__restrict__ Ainv, int n,
                                                         const Tin *__restrict__ b,
                                                         Tout *__restrict__ x) {
    constexpr int CH = 4;
    const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= n) return;   // whole wavefronts leave together
    const double *row = Ainv + (size_t)i * n;
    double acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0;
    for (int j0 = lane; j0 < n; j0 += 64 * CH) {
        double a[CH], bv[CH][K];
#pragma unroll
        for (int u = 0; u < CH; ++u) {   // all loads of a chunk in flight; columns past n weigh 0
            const int j = min(j0 + 64 * u, n - 1);
            a[u] = j0 + 64 * u < n ? row[j] : 0.0;
#pragma unroll
            for (int q = 0; q < K; ++q) bv[u][q] = (double)b[(size_t)j * K + q];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] += a[u] * bv[u][q];
    }
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = wave_sum(acc[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) x[(size_t)i * K + q] = (Tout)acc[q];
    }
}

// ------------------------------------------------------------ team V-cycle
// A team runs Alg. "V-cycle" over a range of levels with barriers between its
// dependent phases (relaxation colors, residual, restriction, coarsest solve,
// prolongation).  A team is one workgroup (barrier = __syncthreads), or
// several workgroups of one batched mesh synchronised through a counter with
// agent-scope release/acquire.  Every wait is bounded: a wait that times out
// raises the team's abort flag, after which no member waits any more, so the
// kernel always drains (results are then invalid and the host reports it).
// Rows are handled by groups of G lanes (G = L.grp) and every lane keeps four
// independent gathers in flight.
struct Team {
    int tid, nthreads;      // thread index within the team, team size
    int rank, nblk;         // workgroup index within the team, team workgroups
    unsigned *ctr;          // barrier counter (nblk > 1)
    int *abort;             // raised when a wait times out
    unsigned target;        // arrivals expected at the next barrier
    double *partial;        // nblk * 8 doubles for team reductions
    int local = 0;          // 1: every workgroup of the team sits on one XCD (one L2)
};

__device__ __forceinline__ Team single_team() {
    return Team{(int)threadIdx.x, (int)blockDim.x, 0, 1, nullptr, nullptr, 0u, nullptr, 0};
}

// Index of the XCD (accelerator complex die) this wavefront runs on.
__device__ __forceinline__ unsigned xcc_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xfu;   // HW_REG_XCC_ID, bits 3:0
}

// Barrier of a team whose workgroups share one L2 (one XCD).  Every wave
// waits until its stores are acknowledged by the L2; thread 0 then adds its
// arrival with an atomic and polls the counter with atomic read-modify-writes
// that leave it unchanged (a compare-and-swap that never matches): atomics
// all see the same counter, while plain loads of it were measured to return
// stale values for up to a second.  Neither needs the L2 write-back that the
// scope of the whole device costs.  After the wait it invalidates the
// compute unit's L1 with the device-scope form of the invalidate, so that
// later loads read the other workgroups' stores from the shared L2: the
// workgroup-scope form was measured to leave stale lines (wrong solves with
// 256- and 512-thread workgroups), the device-scope one costs no measurable
// time here.  The wait is bounded (abort flag).
__device__ __forceinline__ unsigned team_count(unsigned *ctr) {
    unsigned seen = 0xffffffffu;
    __hip_atomic_compare_exchange_strong(ctr, &seen, 0xffffffffu, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return seen;
}
__device__ __forceinline__ void team_sync_local(Team &T) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    T.target += (unsigned)T.nblk;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(T.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        unsigned spins = 0;
        while (team_count(T.ctr) < T.target) {
            if (__hip_atomic_load(T.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (++spins > (1u << 22)) {
                __hip_atomic_store(T.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ void team_sync(Team &T) {
    if (T.local) { team_sync_local(T); return; }
    __syncthreads();
    if (T.nblk > 1) {
        T.target += (unsigned)T.nblk;
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(T.ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            unsigned spins = 0;
            while (__hip_atomic_load(T.ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < T.target) {
                if (__hip_atomic_load(T.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1u << 22)) {
                    __hip_atomic_store(T.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __syncthreads();
    }
}

// team-wide sum or max of K doubles; every team thread gets the result
template <int K>
__device__ __forceinline__ void team_reduce(Team &T, double (&v)[K], bool take_max) {
    __shared__ double red[4 * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = take_max ? wave_max(v[q]) : wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) red[q * nw + wv] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double a = 0.0;
        for (int w = 0; w < nw; ++w) a = take_max ? fmax(a, red[q * nw + w]) : a + red[q * nw + w];
        v[q] = a;
    }
    __syncthreads();
    if (T.nblk > 1) {
        if (threadIdx.x == 0)
#pragma unroll
            for (int q = 0; q < K; ++q) T.partial[T.rank * 8 + q] = v[q];
        team_sync(T);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double a = 0.0;
            for (int r = 0; r < T.nblk; ++r)
                a = take_max ? fmax(a, T.partial[r * 8 + q]) : a + T.partial[r * 8 + q];
            v[q] = a;
        }
        team_sync(T);   // the partial slots may be reused afterwards
    }
}

// off-diagonal sum of row r (valid) over its lane group; all lanes call it.
// The row's first slot comes from a per-row table (one load beside its
// length), the lane's entries are taken four at a time with all loads in
// flight, and its last (fewer than four) entries as one more such chunk whose
// loads are clamped to the row's last entry and whose products are added only
// for entries that exist: one round trip for the row's place, then two per
// chunk.  Products are added in entry order.
template <int K, typename T>
__device__ __forceinline__ void wg_row_sum(const TailLevel<T> &L, int r, bool valid, int j, int G,
                                           const T *__restrict__ x, T (&acc)[K]) {
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = T(0);
    if (valid) {
        const int base = gld(L.row_base, r);
        const int len = gld(L.rowlen, r);
        int e = j;
        for (; e + 3 * G < len; e += 4 * G) {   // four independent gathers in flight
            int c[4];
            T a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ee = e + u * G;
                const int slot = base + (ee / L.lpr) * 64 + (ee % L.lpr);
                c[u] = gld(L.cols, slot);
                a[u] = gld(L.vals, slot);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < K; ++q) acc[q] += a[u] * x[(size_t)c[u] * K + q];
        }
        if (e < len) {
            int c[4];
            T a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ee = min(e + u * G, len - 1);
                const int slot = base + (ee / L.lpr) * 64 + (ee % L.lpr);
                c[u] = gld(L.cols, slot);
                a[u] = gld(L.vals, slot);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e + u * G < len)
#pragma unroll
                    for (int q = 0; q < K; ++q) acc[q] += a[u] * x[(size_t)c[u] * K + q];
        }
    }
    group_sum<K>(acc, G);
}

template <int K, typename T>
__device__ __forceinline__ void wg_relax(Team &tm, const TailLevel<T> &L, int sweeps) {
    const int G = L.grp;
    const int j = tm.tid & (G - 1), g = tm.tid / G, per = tm.nthreads / G;
    for (int sw = 0; sw < sweeps; ++sw)
        for (int c = 0; c < L.ncolors; ++c) {
            const int r0 = gld(L.color_row, c), r1 = gld(L.color_row, c + 1);
            for (int rb = r0; rb < r1; rb += per) {
                const int r = rb + g;
                const bool valid = r < r1;
                T d = T(1), bq[K];   // loaded beside the row's place, ahead of the sum
#pragma unroll
                for (int q = 0; q < K; ++q) bq[q] = T(0);
                if (valid && j == 0) {
                    d = gld(L.diag, r);
#pragma unroll
                    for (int q = 0; q < K; ++q) bq[q] = gld(L.b, (size_t)r * K + q);
                }
                T acc[K];
                wg_row_sum<K, T>(L, r, valid, j, G, L.x, acc);
                if (valid && j == 0) {
#pragma unroll
                    for (int q = 0; q < K; ++q) gst(L.x, (size_t)r * K + q, (bq[q] - acc[q]) / d);
                }
            }
            team_sync(tm);
        }
}

// r = b - A x on one level; optional per-thread column sums / maxima (FP64)
template <int K, typename T>
__device__ __forceinline__ void wg_residual(Team &tm, const TailLevel<T> &L, double (*sq)[K] = nullptr,
                            double (*mx)[K] = nullptr) {
    const int G = L.grp;
    const int j = tm.tid & (G - 1), g = tm.tid / G, per = tm.nthreads / G;
    for (int rb = 0; rb < L.n; rb += per) {
        const int r = rb + g;
        const bool valid = r < L.n;
        T d = T(1), bq[K], xo[K];   // loaded beside the row's place, ahead of the sum
#pragma unroll
        for (int q = 0; q < K; ++q) { bq[q] = T(0); xo[q] = T(0); }
        if (valid && j == 0) {
            d = gld(L.diag, r);
#pragma unroll
            for (int q = 0; q < K; ++q) { bq[q] = gld(L.b, (size_t)r * K + q); xo[q] = gld(L.x, (size_t)r * K + q); }
        }
        T acc[K];
        wg_row_sum<K, T>(L, r, valid, j, G, L.x, acc);
        if (valid && j == 0) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const T rv = bq[q] - (acc[q] + d * xo[q]);
                gst(L.r, (size_t)r * K + q, rv);
                if (sq) { (*sq)[q] += (double)rv * (double)rv; (*mx)[q] = fmax((*mx)[q], fabs((double)rv)); }
            }
        }
    }
}

template <int K, typename T>
__device__ __forceinline__ void wg_vcycle(Team &tm, const TailLevel<T> *__restrict__ lv, int first, int nlev,
                          int mu_pre, int mu_post, const double *__restrict__ Ainv) {
    const int nt = tm.nthreads;
    const int last = nlev - 1;   // coarsest
    for (int l = first; l < last; ++l) {
        const TailLevel<T> L = lv[l];
        if (l > first) {
            for (int t = tm.tid; t < L.n * K; t += nt) gst(L.x, t, T(0));
            team_sync(tm);
        }
        wg_relax<K, T>(tm, L, mu_pre);
        wg_residual<K, T>(tm, L);
        team_sync(tm);
        // restriction into the next level's b (4 lanes per coarse row)
        const TailLevel<T> C = lv[l + 1];
        {
            const int j = tm.tid & 3, per = nt / 4;
            for (int ab = 0; ab < C.n; ab += per) {
                const int a = ab + tm.tid / 4;
                T acc[K];
#pragma unroll
                for (int q = 0; q < K; ++q) acc[q] = T(0);
                if (a < C.n) {
                    for (int p = gld(L.rptr, a) + j; p < gld(L.rptr, a + 1); p += 4) {
                        const int i = gld(L.ridx, p);
                        const T w = gld(L.rw, p);
#pragma unroll
                        for (int q = 0; q < K; ++q) acc[q] += w * gld(L.r, (size_t)i * K + q);
                    }
                }
                group_sum<K>(acc, 4);
                if (a < C.n && j == 0) {
#pragma unroll
                    for (int q = 0; q < K; ++q) gst(C.b, (size_t)a * K + q, acc[q]);
                }
            }
        }
        team_sync(tm);
    }
    {   // coarsest: x = A^{-1} b in FP64, 4 lanes per row
        const TailLevel<T> C = lv[last];
        const int j = tm.tid & 3, per = nt / 4;
        for (int ib = 0; ib < C.n; ib += per) {
            const int i = ib + tm.tid / 4;
            double acc[K];
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] = 0.0;
            if (i < C.n) {
                int jj = j;
                for (; jj + 12 < C.n; jj += 16) {
                    double a[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) a[u] = gld(Ainv, (size_t)(jj + 4 * u) * C.n + i);
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int q = 0; q < K; ++q) acc[q] += a[u] * (double)gld(C.b, (size_t)(jj + 4 * u) * K + q);
                }
                for (; jj < C.n; jj += 4) {
                    const double a = gld(Ainv, (size_t)jj * C.n + i);
#pragma unroll
                    for (int q = 0; q < K; ++q) acc[q] += a * (double)gld(C.b, (size_t)jj * K + q);
                }
            }
            group_sum<K>(acc, 4);
            if (i < C.n && j == 0) {
#pragma unroll
                for (int q = 0; q < K; ++q) gst(C.x, (size_t)i * K + q, (T)acc[q]);
            }
        }
        team_sync(tm);
    }
    for (int l = last - 1; l >= first; --l) {
        const TailLevel<T> L = lv[l];
        const TailLevel<T> C = lv[l + 1];
        for (int i = tm.tid; i < L.n; i += nt) {
            T acc[K];
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] = T(0);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const int c = gld(L.pc, (size_t)m * L.n + i);
                const T w = gld(L.pw, (size_t)m * L.n + i);
#pragma unroll
                for (int q = 0; q < K; ++q) acc[q] += w * gld(C.x, (size_t)c * K + q);
            }
#pragma unroll
            for (int q = 0; q < K; ++q) gst(L.x, (size_t)i * K + q, gld(L.x, (size_t)i * K + q) + acc[q]);
        }
        team_sync(tm);
        wg_relax<K, T>(tm, L, mu_post);
    }
}

// ----------------------------------------------- one-XCD team V-cycle
// Alg. "V-cycle" from level `first` down to the coarsest and back by m
// workgroups that share one XCD (one L2), meeting at L2-local team barriers
// instead of kernel boundaries.  The grid has 8 m workgroups; they are handed
// to the 8 XCDs in turn, so every XCD receives m of them.  The first
// workgroup to start claims its XCD for the team (cb[0] = xcc + 1), the
// workgroups of that XCD take ranks 0..m-1 from cb[1], all others return.
// cb[32] is the barrier counter (a cache line of its own: it lives in that
// XCD's L2 while cb[0..1] are updated at device scope); cb[0..63] are zero
// before the launch.  A team that
// does not come together (a barrier wait that times out) raises flag[0].
template <int K, typename T>
__global__ __launch_bounds__(1024) void k_team_vcycle(const TailLevel<T> *__restrict__ lv, int first, int nlev,
                                                      int mu_pre, int mu_post, const double *__restrict__ Ainv,
                                                      unsigned *__restrict__ cb, int *__restrict__ flag, int m) {
    __shared__ int s_rank;
    if (threadIdx.x == 0) {
        const unsigned mine = xcc_id() + 1u;
        unsigned expect = 0u;
        __hip_atomic_compare_exchange_strong(cb, &expect, mine, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const unsigned owner = expect == 0u ? mine : expect;   // expect holds the winner when the exchange failed
        int rank = -1;
        if (owner == mine) {
            rank = (int)__hip_atomic_fetch_add(cb + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (rank >= m) rank = -1;
        }
        s_rank = rank;
    }
    __syncthreads();
    if (s_rank < 0) return;
    Team tm;
    tm.rank = s_rank;
    tm.nblk = m;
    tm.tid = tm.rank * (int)blockDim.x + (int)threadIdx.x;
    tm.nthreads = m * (int)blockDim.x;
    tm.ctr = cb + 32;
    tm.abort = flag;
    tm.target = 0u;
    tm.partial = nullptr;
    tm.local = 1;
    wg_vcycle<K, T>(tm, lv, first, nlev, mu_pre, mu_post, Ainv);
}

// ------------------------------------------------------ LDS-resident tail
// One workgroup runs Alg. "V-cycle" over the coarse end of the hierarchy
// with the iterate x of every tail level (and b of the coarsest) in LDS, rows
// padded to KP values.  Each relaxation pass issues all its independent loads
// (records, diagonal, b) at once and gathers x from LDS, so a color costs one
// memory round trip (mostly L2 hits) plus one workgroup barrier.  Pointers
// read from the level descriptors are marked global explicitly (the compiler
// cannot infer it) so loads need not wait on LDS traffic, and every load of a
// chunk is unconditional (clamped index, masked value) so all are in flight.

template <typename T, int K, int KP>
__device__ __forceinline__ void lds_get(const T *xs, int c, T (&v)[K]) {
    if constexpr (KP == 4 && sizeof(T) == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(xs + (size_t)c * 4);
        const T t4[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] = t4[q];
    } else if constexpr (KP == 4 && sizeof(T) == 8) {
        const double2 a = *reinterpret_cast<const double2 *>(xs + (size_t)c * 4);
        const double2 b = *reinterpret_cast<const double2 *>(xs + (size_t)c * 4 + 2);
        const T t4[4] = {a.x, a.y, b.x, b.y};
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] = t4[q];
    } else {
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] = xs[(size_t)c * KP + q];
    }
}

// acc += sum over this thread's records (rounds k < kmax, 64 apart) in
// chunks of CH rounds; rounds past kmax re-read the last record with weight 0,
// so nothing in a chunk is conditional
// A lane's two records of a pair: one 16-byte load in FP32 (one compute
// unit streams 16-byte loads from L2 about twice as fast as 8-byte ones),
// two in FP64.
typedef int vint4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void pair_load(const TailRec<float> *p, size_t i, int (&c)[2], float (&v)[2]) {
    const vint4 a = gld(reinterpret_cast<const vint4 *>(p + i), 0);
    c[0] = a.x; v[0] = __int_as_float(a.y); c[1] = a.z; v[1] = __int_as_float(a.w);
}
__device__ __forceinline__ void pair_load(const TailRec<double> *p, size_t i, int (&c)[2], double (&v)[2]) {
    const vint4 a = gld(reinterpret_cast<const vint4 *>(p + i), 0);
    const vint4 b = gld(reinterpret_cast<const vint4 *>(p + i + 1), 0);
    c[0] = a.x; v[0] = __hiloint2double(a.w, a.z); c[1] = b.x; v[1] = __hiloint2double(b.w, b.z);
}

// acc += this lane's records of pairs [p0, p0 + CH) (pairs past np re-read the
// last one with weight 0), all loads issued before any is used
template <int CH, int K, int KP, typename T>
__device__ __forceinline__ void tail_gather_ch(const TailRec<T> *rp, int p0, int np, const T *xs,
                                               T (&acc)[K]) {
    int c[CH][2];
    T v[CH][2];
#pragma unroll
    for (int u = 0; u < CH; ++u) pair_load(rp, (size_t)min(p0 + u, np - 1) * 128, c[u], v[u]);
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const T w = p0 + u < np ? v[u][h] : T(0);
            T xv[K];
            lds_get<T, K, KP>(xs, c[u][h], xv);
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] += w * xv[q];
        }
}
// full chunks of 4 pairs, then one chunk of 1, 2 or 4 pairs for the rest
template <int K, int KP, typename T>
__device__ __forceinline__ void tail_gather(const TailRec<T> *rp, int np, const T *xs, T (&acc)[K]) {
    int p0 = 0;
    for (; p0 + 4 <= np; p0 += 4) tail_gather_ch<4, K, KP, T>(rp, p0, np, xs, acc);
    const int rem = np - p0;
    if (rem <= 0) return;
    if (rem == 1) tail_gather_ch<1, K, KP, T>(rp, p0, np, xs, acc);
    else if (rem == 2) tail_gather_ch<2, K, KP, T>(rp, p0, np, xs, acc);
    else tail_gather_ch<4, K, KP, T>(rp, p0, np, xs, acc);
}

// one pass row: diagonal, b and the off-diagonal sum over the lane group
// (the wavefront's record offset and rounds come from the LDS table)
template <int K, int KP, typename T>
__device__ __forceinline__ void tail_row(const LdsLevel<T> &L, const int2 *wv, int tid, int row, int G,
                                         const T *xs, T &d, T (&bq)[K], T (&acc)[K], int vs, int vc) {
    const int2 W = wv[tid >> 6];
    const int off = __builtin_amdgcn_readfirstlane(W.x), kmax = __builtin_amdgcn_readfirstlane(W.y);
    d = gld(L.diag, row);
#pragma unroll
    for (int q = 0; q < K; ++q) { bq[q] = gld(L.b, (size_t)row * vs + vc + q); acc[q] = T(0); }
    tail_gather<K, KP, T>(L.rec + off + 2 * (tid & 63), kmax, xs, acc);
    group_sum<K>(acc, G);
}

// Multicolor Gauss-Seidel on one tail level (App. A): passes in color order
// (descending: colors last to first), a barrier after every color.
template <int K, int KP, typename T>
__device__ void tail_relax(const LdsLevel<T> &L, const int4 *sp, const int2 *swv, T *xs, int sweeps,
                           bool descending, int vs, int vc) {
    const int tid = threadIdx.x, lg = L.lg_grp, G = 1 << lg;
    const int g = tid >> lg, j = tid & (G - 1);
    for (int sw = 0; sw < sweeps; ++sw)
        for (int pp = 0; pp < L.npass; ++pp) {
            const int p = descending ? L.npass - 1 - pp : pp;
            const int4 P = sp[p];
            const int nta = P.y << lg;
            if (tid < nta) {
                const int row = P.x + g;
                T d, bq[K], acc[K];
                tail_row<K, KP, T>(L, swv + P.w, tid, row, G, xs, d, bq, acc, vs, vc);
                if (j == 0)
#pragma unroll
                    for (int q = 0; q < K; ++q) xs[(size_t)row * KP + q] = (bq[q] - acc[q]) / d;
            }
            // a color ends after its last pass, or, going down, its first one
            if (descending ? (p == 0 || (sp[p - 1].z >> 16)) : (P.z >> 16)) __syncthreads();
        }
}

// r = b - A x on one tail level (r in global memory); no barrier inside
template <int K, int KP, typename T>
__device__ void tail_residual(const LdsLevel<T> &L, const int4 *sp, const int2 *swv, const T *xs, int vs, int vc) {
    const int tid = threadIdx.x, lg = L.lg_grp, G = 1 << lg;
    const int g = tid >> lg, j = tid & (G - 1);
    for (int p = 0; p < L.npass; ++p) {
        const int4 P = sp[p];
        const int nta = P.y << lg;
        if (tid < nta) {
            const int row = P.x + g;
            T d, bq[K], acc[K];
            tail_row<K, KP, T>(L, swv + P.w, tid, row, G, xs, d, bq, acc, vs, vc);
            if (j == 0) {
                T xv[K];
                lds_get<T, K, KP>(xs, row, xv);
#pragma unroll
                for (int q = 0; q < K; ++q) gst(L.r, (size_t)row * vs + vc + q, bq[q] - (acc[q] + d * xv[q]));
            }
        }
    }
}

// b_{l+1} = R r (R = P^T as ELL); into LDS (bl) for the coarsest level, else
// into the next level's global b, whose x is then cleared in LDS
template <int K, int KP, typename T>
__device__ void tail_restrict(const LdsLevel<T> &L, T *bc_global, T *bl, T *xc, int vs, int vc) {
    constexpr int CH = 8;
    const int tid = threadIdx.x, nt = blockDim.x, nc = L.nc, rk = L.rk;
    for (int a = tid; a < nc; a += nt) {
        T acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = T(0);
        for (int k0 = 0; k0 < rk; k0 += CH) {
            int c[CH];
            T w[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const size_t at = (size_t)min(k0 + u, rk - 1) * nc + a;
                c[u] = gld(L.ridx, at);
                w[u] = k0 + u < rk ? gld(L.rw, at) : T(0);
            }
            T rv[CH][K];
#pragma unroll
            for (int u = 0; u < CH; ++u)
#pragma unroll
                for (int q = 0; q < K; ++q) rv[u][q] = gld((const T *)L.r, (size_t)c[u] * vs + vc + q);
#pragma unroll
            for (int u = 0; u < CH; ++u)
#pragma unroll
                for (int q = 0; q < K; ++q) acc[q] += w[u] * rv[u][q];
        }
        if (bl) {
#pragma unroll
            for (int q = 0; q < K; ++q) bl[(size_t)a * KP + q] = acc[q];
        } else {
#pragma unroll
            for (int q = 0; q < K; ++q) gst(bc_global, (size_t)a * vs + vc + q, acc[q]);
        }
    }
    if (!bl)
        for (int t = tid; t < nc * KP; t += nt) xc[t] = T(0);
}

// coarsest: x = A_H^{-1} b in FP64 (A_H^{-1} column-major), 4 lanes per row
template <int K, int KP, typename T>
__device__ void tail_coarse(int n, const double *__restrict__ Ainv, const T *bl, T *xl) {
    constexpr int CH = 8;
    const int tid = threadIdx.x, nt = blockDim.x, j = tid & 3;
    for (int ib = 0; ib < n; ib += nt / 4) {
        const int i = ib + tid / 4;
        const int ic = min(i, n - 1);
        double acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = 0.0;
        for (int j0 = j; j0 < n; j0 += 4 * CH) {
            double a[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) a[u] = Ainv[(size_t)min(j0 + 4 * u, n - 1) * n + ic];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int jj = j0 + 4 * u;
                if (jj < n) {
                    T bv[K];
                    lds_get<T, K, KP>(bl, jj, bv);
#pragma unroll
                    for (int q = 0; q < K; ++q) acc[q] += a[u] * (double)bv[q];
                }
            }
        }
        group_sum<K>(acc, 4);
        if (i < n && j == 0)
#pragma unroll
            for (int q = 0; q < K; ++q) xl[(size_t)i * KP + q] = (T)acc[q];
    }
}

// x_l += P_l x_{l+1}
template <int K, int KP, typename T>
__device__ void tail_prolong(const LdsLevel<T> &L, T *xs, const T *xc) {
    const int tid = threadIdx.x, nt = blockDim.x, n = L.n;
    for (int i = tid; i < n; i += nt) {
        T acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = T(0);
        int c[3];
        T w[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) { c[m] = gld(L.pc, (size_t)m * n + i); w[m] = gld(L.pw, (size_t)m * n + i); }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            T xv[K];
            lds_get<T, K, KP>(xc, c[m], xv);
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] += w[m] * xv[q];
        }
#pragma unroll
        for (int q = 0; q < K; ++q) xs[(size_t)i * KP + q] += acc[q];
    }
}

template <int K, typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail_lds(const LdsLevel<T> *__restrict__ lv,
                                                           const int4 *__restrict__ passes,
                                                           const int2 *__restrict__ waves, int first,
                                                           int nlev, int mu_pre, int mu_post,
                                                           const double *__restrict__ Ainv, int post_desc,
                                                           int vs) {
    constexpr int KP = K == 3 ? 4 : K;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x, last = nlev - 1;
    // global vectors are n x vs; this workgroup owns columns [vc, vc + K)
    const int vc = blockIdx.x * K;
    const int pbeg = lv[first].pass0, pend = lv[last].pass0;
    const int wbeg = lv[first].wave0, wend = lv[last].wave0;
    int4 *sp = reinterpret_cast<int4 *>(smem);
    int2 *swv = reinterpret_cast<int2 *>(smem + (size_t)(pend - pbeg) * sizeof(int4));
    for (int i = tid; i < pend - pbeg; i += nt) {
        int4 P = passes[pbeg + i];
        P.w -= wbeg;   // wavefront index relative to the LDS copy
        sp[i] = P;
    }
    for (int i = tid; i < wend - wbeg; i += nt) swv[i] = waves[wbeg + i];
    const size_t tables = ((size_t)(pend - pbeg) * 16 + (size_t)(wend - wbeg) * 8 + 15) / 16 * 16;
    T *xall = reinterpret_cast<T *>(smem + tables);
    const int base = lv[first].nsum;
    T *bl = xall + (size_t)(lv[last].nsum + lv[last].n - base) * KP;
    {
        const int n0 = lv[first].n;
        const T *xg = lv[first].x;
        for (int t = tid; t < n0 * K; t += nt) xall[(size_t)(t / K) * KP + t % K] = gld(xg, (size_t)(t / K) * vs + vc + t % K);
    }
    __syncthreads();
    for (int l = first; l < last; ++l) {
        const LdsLevel<T> L = lv[l];
        T *xs = xall + (size_t)(L.nsum - base) * KP;
        T *xc = xall + (size_t)(L.nsum + L.n - base) * KP;
        tail_relax<K, KP, T>(L, sp + (L.pass0 - pbeg), swv, xs, mu_pre, false, vs, vc);
        tail_residual<K, KP, T>(L, sp + (L.pass0 - pbeg), swv, xs, vs, vc);
        __syncthreads();
        tail_restrict<K, KP, T>(L, lv[l + 1].b, l + 1 == last ? bl : nullptr, xc, vs, vc);
        __syncthreads();
    }
    tail_coarse<K, KP, T>(lv[last].n, Ainv, bl, xall + (size_t)(lv[last].nsum - base) * KP);
    __syncthreads();
    for (int l = last - 1; l >= first; --l) {
        const LdsLevel<T> L = lv[l];
        T *xs = xall + (size_t)(L.nsum - base) * KP;
        tail_prolong<K, KP, T>(L, xs, xall + (size_t)(L.nsum + L.n - base) * KP);
        __syncthreads();
        tail_relax<K, KP, T>(L, sp + (L.pass0 - pbeg), swv, xs, mu_post, post_desc != 0, vs, vc);
    }
    {
        const int n0 = lv[first].n;
        T *xg = lv[first].x;
        for (int t = tid; t < n0 * K; t += nt) gst(xg, (size_t)(t / K) * vs + vc + t % K, xall[(size_t)(t / K) * KP + t % K]);
    }
}

// One step of the tail on level l alone, with the device code of k_tail_lds
// and its thread-to-row mapping (so its results equal that kernel's, pass
// for pass): the level's iterate is loaded into LDS from lv[l].x (and the
// next level's from lv[l + 1].x), the step runs, and what it changed is
// stored back.  op: kTailStepRelax `sweeps` sweeps (desc: colors
// descending), kTailStepResidual into lv[l].r, kTailStepRestrict into
// lv[l + 1].b, kTailStepProlong x_l += P_l x_{l+1}, kTailStepCoarse
// x_l = A_H^{-1} b_l on the coarsest level.
template <int K, typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail_step(const LdsLevel<T> *__restrict__ lv,
                                                            const int4 *__restrict__ passes,
                                                            const int2 *__restrict__ waves, int l, int nlev,
                                                            int op, int sweeps, int desc,
                                                            const double *__restrict__ Ainv, int vs) {
    constexpr int KP = K == 3 ? 4 : K;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x, last = nlev - 1;
    const int vc = blockIdx.x * K;
    const LdsLevel<T> L = lv[l];
    const int np = l < last ? L.npass : 0;
    const int wbeg = L.wave0, nw = l < last ? lv[l + 1].wave0 - wbeg : 0;
    int4 *sp = reinterpret_cast<int4 *>(smem);
    int2 *swv = reinterpret_cast<int2 *>(smem + (size_t)np * sizeof(int4));
    for (int i = tid; i < np; i += nt) {
        int4 P = passes[L.pass0 + i];
        P.w -= wbeg;
        sp[i] = P;
    }
    for (int i = tid; i < nw; i += nt) swv[i] = waves[wbeg + i];
    const size_t tables = ((size_t)np * 16 + (size_t)nw * 8 + 15) / 16 * 16;
    T *xs = reinterpret_cast<T *>(smem + tables);
    const int nc = l < last ? lv[l + 1].n : 0;
    T *xc = xs + (size_t)L.n * KP;
    const bool coarse_next = l + 1 == last;
    // load the iterate of this level (the coarsest solve reads b instead)
    const T *src = op == kTailStepCoarse ? L.b : L.x;
    for (int t = tid; t < L.n * K; t += nt) xs[(size_t)(t / K) * KP + t % K] = gld(src, (size_t)(t / K) * vs + vc + t % K);
    if (op == kTailStepProlong)
        for (int t = tid; t < nc * K; t += nt)
            xc[(size_t)(t / K) * KP + t % K] = gld((const T *)lv[l + 1].x, (size_t)(t / K) * vs + vc + t % K);
    __syncthreads();
    if (op == kTailStepRelax) {
        tail_relax<K, KP, T>(L, sp, swv, xs, sweeps, desc != 0, vs, vc);
    } else if (op == kTailStepResidual) {
        tail_residual<K, KP, T>(L, sp, swv, xs, vs, vc);
        return;
    } else if (op == kTailStepRestrict) {
        tail_restrict<K, KP, T>(L, lv[l + 1].b, coarse_next ? xc : nullptr, xc, vs, vc);
        if (!coarse_next) return;
        __syncthreads();
        for (int t = tid; t < nc * K; t += nt) gst(lv[l + 1].b, (size_t)(t / K) * vs + vc + t % K, xc[(size_t)(t / K) * KP + t % K]);
        return;
    } else if (op == kTailStepProlong) {
        tail_prolong<K, KP, T>(L, xs, xc);
    } else {
        tail_coarse<K, KP, T>(L.n, Ainv, xs, xc);
        __syncthreads();
        for (int t = tid; t < L.n * K; t += nt) gst(L.x, (size_t)(t / K) * vs + vc + t % K, xc[(size_t)(t / K) * KP + t % K]);
        return;
    }
    __syncthreads();
    for (int t = tid; t < L.n * K; t += nt) gst(L.x, (size_t)(t / K) * vs + vc + t % K, xs[(size_t)(t / K) * KP + t % K]);
}

__global__ void k_gather_records(const int32_t *__restrict__ src, const int32_t *__restrict__ cols,
                                 int64_t n, const double *__restrict__ vals,
                                 const float *__restrict__ vals32, TailRec<double> *__restrict__ rec64,
                                 TailRec<float> *__restrict__ rec32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t s = src[i], c = cols[i];
    rec64[i] = TailRec<double>{c, 0, s >= 0 ? vals[s] : 0.0};
    rec32[i] = TailRec<float>{c, s >= 0 ? vals32[s] : 0.0f};
}


// ---------------------------------------------------------- batched solve
// A team of workgroups per mesh runs Alg. "Galerkin Surface Multigrid
// Solver" to convergence: FP64 level-0 residual and norms, FP32 V-cycle on
// r / max|r|, FP64 update, with the convergence test on the device.  Meshes
// never wait for each other; converged meshes' teams exit.
template <int K>
__device__ __forceinline__ void batch_mesh(Team &tm, const BatchMesh &M) {
    const TailLevel<double> L0 = M.l0;
    const int n = L0.n, nt = tm.nthreads;
    // b (caller order) -> level-0 color-major order; x = 0; r = b
    for (int t = tm.tid; t < n * K; t += nt) {
        const int r = t / K, q = t % K;
        const double v = gld(M.b_user, (size_t)gld(M.perm0, r) * K + q);
        gst(L0.b, t, v);
        gst(L0.r, t, v);
        gst(L0.x, t, 0.0);
    }
    double bn[K], sq[K], mx[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { sq[q] = 0.0; mx[q] = 0.0; }
    for (int t = tm.tid; t < n * K; t += nt) {
        const double v = gld(M.b_user, (size_t)gld(M.perm0, t / K) * K + t % K);
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (t % K == q) { sq[q] += v * v; mx[q] = fmax(mx[q], fabs(v)); }
    }
    team_reduce<K>(tm, sq, false);
    team_reduce<K>(tm, mx, true);
    double rho[K];
#pragma unroll
    for (int q = 0; q < K; ++q) { bn[q] = sqrt(sq[q]); rho[q] = bn[q] > 0.0 ? 1.0 : 0.0; }
    const TailLevel<float> F0 = M.lv32[0];
    int cycles = 0;
    for (;;) {
        double worst = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) worst = fmax(worst, rho[q]);
        if (!(worst > M.rtol) || cycles >= M.max_cycles) break;
        if (M.precision == 0) {   // plain FP64 V-cycle on (b, x) of level 0
            wg_vcycle<K, double>(tm, M.lv64, 0, M.nlev, M.mu_pre, M.mu_post, M.Ainv);
        } else {
            // r32 = r / max|r| ; x32 = 0
            for (int t = tm.tid; t < n * K; t += nt) {
                const int q = t % K;
                double s = 0.0;
#pragma unroll
                for (int qq = 0; qq < K; ++qq) if (qq == q) s = mx[qq];
                gst(F0.b, t, (float)(s > 0.0 ? gld(L0.r, t) / s : 0.0));
                gst(F0.x, t, 0.0f);
            }
            team_sync(tm);
            wg_vcycle<K, float>(tm, M.lv32, 0, M.nlev, M.mu_pre, M.mu_post, M.Ainv);
            for (int t = tm.tid; t < n * K; t += nt) {
                const int q = t % K;
                double s = 0.0;
#pragma unroll
                for (int qq = 0; qq < K; ++qq) if (qq == q) s = mx[qq];
                gst(L0.x, t, gld(L0.x, t) + s * (double)gld(F0.x, t));
            }
            team_sync(tm);
        }
#pragma unroll
        for (int q = 0; q < K; ++q) { sq[q] = 0.0; mx[q] = 0.0; }
        wg_residual<K, double>(tm, L0, &sq, &mx);
        team_reduce<K>(tm, sq, false);
        team_reduce<K>(tm, mx, true);
        ++cycles;
#pragma unroll
        for (int q = 0; q < K; ++q) rho[q] = bn[q] > 0.0 ? sqrt(sq[q]) / bn[q] : sqrt(sq[q]);
        bool finite = true;
#pragma unroll
        for (int q = 0; q < K; ++q) finite = finite && isfinite(rho[q]);
        if (!finite) break;
    }
    for (int t = tm.tid; t < n * K; t += nt) {
        const int r = t / K, q = t % K;
        gst(M.x_user, (size_t)gld(M.perm0, r) * K + q, gld(L0.x, t));
    }
    if (tm.tid == 0) {
        gst(M.out, 0, (double)cycles);
#pragma unroll
        for (int q = 0; q < K; ++q) gst(M.out, 1 + q, rho[q]);
    }
}

// block b works for mesh team_mesh[b] as member team_rank[b] of team_size[mesh];
// one instantiation per workgroup size, so smaller workgroups get the larger
// register budget instead of spilling.  Everything below the kernel is
// inlined: an outlined call takes the Team by reference, which puts it in
// scratch memory and turns every use of its fields into a scratch load
// (measured: 1,624 scratch loads in the 1024-thread kernel, 29 inlined;
// 208 -> 200 ms per 64-mesh batch)
template <int BS>
__global__ __launch_bounds__(BS) void k_batch_solve(const BatchMesh *__restrict__ meshes,
                                                      const int32_t *__restrict__ team_mesh,
                                                      const int32_t *__restrict__ team_rank,
                                                      unsigned *__restrict__ ctrs,
                                                      int *__restrict__ aborts,
                                                      double *__restrict__ partials) {
    const int m = team_mesh[blockIdx.x];
    if (m < 0) return;   // an idle slot of the XCD-packed grid
    const BatchMesh M = meshes[m];
    Team tm;
    tm.rank = team_rank[blockIdx.x];
    tm.nblk = M.team;
    tm.tid = tm.rank * (int)blockDim.x + (int)threadIdx.x;
    tm.nthreads = tm.nblk * (int)blockDim.x;
    tm.ctr = ctrs + (size_t)m * kBatchCtrStride;
    tm.abort = aborts + m;
    tm.target = 0u;
    tm.partial = partials + (size_t)m * 8 * 64;
    tm.local = M.local;
    // the team's L2-local barriers need every member on one XCD: the first
    // member to arrive records its XCD (device-scope compare-and-swap on a
    // word the launch cleared), the others check theirs against it
    if (M.local && threadIdx.x == 0) {
        unsigned expected = 0u;
        const unsigned mine = xcc_id() + 1u;
        unsigned *slot = tm.ctr + 1;
        if (!__hip_atomic_compare_exchange_strong(slot, &expected, mine, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) &&
            expected != mine)
            __hip_atomic_store(tm.abort, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    switch (M.k) {
    case 1: batch_mesh<1>(tm, M); break;
    case 2: batch_mesh<2>(tm, M); break;
    case 3: batch_mesh<3>(tm, M); break;
    default: batch_mesh<4>(tm, M); break;
    }
}

// ------------------------------------------------------- hierarchy values
__global__ __launch_bounds__(kBlock) void k_scatter_values(const double *__restrict__ src,
                                                           const int32_t *__restrict__ store,
                                                           int64_t nnz, double *__restrict__ vals,
                                                           double *__restrict__ diag,
                                                           int *__restrict__ flag) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nnz) return;
    const double v = src[p];
    if (!isfinite(v)) *flag = 1;
    const int32_t s = store[p];
    if (s >= 0) vals[s] = v;
    else diag[-1 - s] = v;
}

// T = A P, G lanes per permuted fine row (the owners of its T row): lane g
// takes the row's off-diagonal entries e = g, g + G, ... (lane 0 also the
// diagonal term first) and accumulates them in its own LDS slots (slot k of
// thread i at k * bs + i) in that fixed order; the row's G partial rows are
// then added in lane order and written out contiguously, so the result does
// not depend on timing.
template <int G>
__global__ __launch_bounds__(64) void k_galerkin_t(
    int n, const int32_t *__restrict__ tptr, const int32_t *__restrict__ plan1ptr,
    const uint16_t *__restrict__ plan1, const int32_t *__restrict__ row_slice,
    const int32_t *__restrict__ slice_row0, const int32_t *__restrict__ slice_off, int lpr,
    const int32_t *__restrict__ rowlen, const int32_t *__restrict__ cols,
    const double *__restrict__ vals, const double *__restrict__ diag,
    const double *__restrict__ pw, double *__restrict__ Tb) {
    extern __shared__ double acc_t[];
    const int bs = blockDim.x, rows = bs / G;
    const int jr = (int)threadIdx.x / G, g = (int)threadIdx.x % G;
    const int r = blockIdx.x * rows + jr;
    const bool act = r < n;
    double *acc = acc_t + threadIdx.x;
    const int t0 = act ? tptr[r] : 0, len = act ? tptr[r + 1] - t0 : 0;
    for (int k = 0; k < len; ++k) acc[k * bs] = 0.0;
    if (act) {
        const uint16_t *pl = plan1 + plan1ptr[r];
        if (g == 0) {
            const double d = diag[r];
#pragma unroll
            for (int m = 0; m < 3; ++m) acc[pl[m] * bs] += d * pw[(size_t)m * n + r];
        }
        const int s = row_slice[r];
        const int base = slice_off[s] + (r - slice_row0[s]) * lpr;
        const int rl = rowlen[r];
#pragma unroll 2
        for (int e = g; e < rl; e += G) {
            const int slot = base + (e / lpr) * 64 + (e % lpr);
            const int c = cols[slot];
            const double a = vals[slot];
#pragma unroll
            for (int m = 0; m < 3; ++m) acc[pl[3 * (e + 1) + m] * bs] += a * pw[(size_t)m * n + c];
        }
    }
    __syncthreads();
    for (int k = g; k < len; k += G) {
        double v = 0.0;
#pragma unroll
        for (int h = 0; h < G; ++h) v += acc_t[k * bs + jr * G + h];
        Tb[t0 + k] = v;
    }
}

// A_{l+1} = P^T T, G lanes per permuted coarse row: lane g takes the row's R
// entries p = g, g + G, ... (each contributing w T_rb for every entry of T row
// r) into its own LDS slots, in (R entry, T entry) order; the G partial rows
// are then added in lane order and each slot stored to its position in level
// l+1.
template <int G>
__global__ __launch_bounds__(64) void k_galerkin_c(
    int nc, const int32_t *__restrict__ plan2ptr, const uint16_t *__restrict__ plan2,
    const int32_t *__restrict__ rptr, const int32_t *__restrict__ ridx,
    const double *__restrict__ rw, const int32_t *__restrict__ tptr,
    const double *__restrict__ Tb, const int32_t *__restrict__ optr,
    const int32_t *__restrict__ opos, double *__restrict__ vals, double *__restrict__ diag) {
    extern __shared__ double acc_c[];
    const int bs = blockDim.x, rows = bs / G;
    const int jr = (int)threadIdx.x / G, g = (int)threadIdx.x % G;
    const int a = blockIdx.x * rows + jr;
    const bool act = a < nc;
    double *acc = acc_c + threadIdx.x;
    const int o0 = act ? optr[a] : 0, len = act ? optr[a + 1] - o0 : 0;
    for (int k = 0; k < len; ++k) acc[k * bs] = 0.0;
    if (act) {
        int idx = plan2ptr[a];   // the plan lists the row's (p, t) pairs in order
        const int p0 = rptr[a], p1 = rptr[a + 1];
        for (int p = p0; p < p1; ++p) {
            const int r = ridx[p];
            const int tb = tptr[r], te = tptr[r + 1];
            if ((p - p0) % G == g) {
                const double w = rw[p];
#pragma unroll 4
                for (int t = tb; t < te; ++t) acc[plan2[idx + (t - tb)] * bs] += w * Tb[t];
            }
            idx += te - tb;
        }
    }
    __syncthreads();
    for (int k = g; k < len; k += G) {
        double v = 0.0;
#pragma unroll
        for (int h = 0; h < G; ++h) v += acc_c[k * bs + jr * G + h];
        const int32_t pos = opos[o0 + k];
        if (pos >= 0) vals[pos] = v;
        else diag[-1 - pos] = v;
    }
}

// ------------------------------------------------------------ elementwise
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *__restrict__ p, T v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ __launch_bounds__(kBlock) void k_to_f32(const double *__restrict__ s, float *__restrict__ d,
                                                   int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}
template <typename Ts, typename Td>
__global__ __launch_bounds__(kBlock) void k_gather_rows(const int32_t *__restrict__ perm,
                                                        const Ts *__restrict__ src,
                                                        Td *__restrict__ dst, int n, int k) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * k) return;
    const int r = (int)(t / k), q = (int)(t % k);
    dst[t] = (Td)src[(size_t)perm[r] * k + q];
}
template <typename Ts, typename Td>
__global__ __launch_bounds__(kBlock) void k_scatter_rows(const int32_t *__restrict__ perm,
                                                         const Ts *__restrict__ src,
                                                         Td *__restrict__ dst, int n, int k) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * k) return;
    const int r = (int)(t / k), q = (int)(t % k);
    dst[(size_t)perm[r] * k + q] = (Td)src[t];
}
__global__ __launch_bounds__(kBlock) void k_check_finite(const double *__restrict__ v, int64_t n,
                                                         int *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && !isfinite(v[i])) *flag = 1;
}
// r32 = r64 / sigma_q with sigma_q = max |r_q| (1 if the column is zero)
__global__ __launch_bounds__(kBlock) void k_ir_down(const double *__restrict__ r64,
                                                    const double *__restrict__ norms,
                                                    float *__restrict__ r32, int n, int k) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * k) return;
    const int q = (int)(t % k);
    const double s = norms[k + q];
    r32[t] = (float)(s > 0.0 ? r64[t] / s : 0.0);
}
__global__ __launch_bounds__(kBlock) void k_ir_up(float *__restrict__ d32,
                                                  const double *__restrict__ norms,
                                                  double *__restrict__ x64, int n, int k) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n * k) return;
    const int q = (int)(t % k);
    const double s = norms[k + q];
    x64[t] += (s > 0.0 ? s : 0.0) * (double)d32[t];
    d32[t] = 0.0f;
}

// ----------------------------------------------------------- assembly (K6)
// Row v of A = diag(s m) + t L_w, with L_ij = -1/2 sum cot(opposite angles)
// (times w_e), L_ii = -sum_j L_ij, m_v = sum of incident face areas / 3.
// One thread owns row v; contributions are gathered from v's faces.
constexpr int kAsmSlots = 16;   // row entries accumulated in LDS by k_assemble (longer rows: in place)
__global__ __launch_bounds__(kBlock) void k_assemble(MeshView M, const double *__restrict__ V,
                                                     double t, const double *__restrict__ s,
                                                     const float *__restrict__ ew,
                                                     double *__restrict__ a_vals,
                                                     double *__restrict__ l_vals,
                                                     double *__restrict__ mass) {
    // the row is accumulated in the thread's own LDS slots (slot e at
    // e * kBlock), or in place in a_vals when it is longer than kAsmSlots;
    // either way the same additions in the same order
    __shared__ double racc[kAsmSlots * kBlock];
    const int v = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (v >= M.n) return;
    const int p0 = M.rowptr[v], p1 = M.rowptr[v + 1];
    const bool in_lds = p1 - p0 <= kAsmSlots;
    double *ra = racc + threadIdx.x;
    auto row = [&](int p) -> double & { return in_lds ? ra[(p - p0) * kBlock] : a_vals[p]; };
    for (int p = p0; p < p1; ++p) row(p) = 0.0;
    double m = 0.0;
    for (int q = M.vf_ptr[v]; q < M.vf_ptr[v + 1]; ++q) {
        const int f = M.vf_face[q];
        int c0 = 0;
        while (M.faces[3 * f + c0] != v) ++c0;
        const int a = M.faces[3 * f + (c0 + 1) % 3], b = M.faces[3 * f + (c0 + 2) % 3];
        const double vx = V[3 * v], vy = V[3 * v + 1], vz = V[3 * v + 2];
        const double ax = V[3 * a], ay = V[3 * a + 1], az = V[3 * a + 2];
        const double bx = V[3 * b], by = V[3 * b + 1], bz = V[3 * b + 2];
        // angle at b (opposite edge v-a): vectors b->v, b->a
        double ux = vx - bx, uy = vy - by, uz = vz - bz, wx = ax - bx, wy = ay - by, wz = az - bz;
        double cx = uy * wz - uz * wy, cy = uz * wx - ux * wz, cz = ux * wy - uy * wx;
        const double cn = sqrt(cx * cx + cy * cy + cz * cz);
        const double cot_b = (ux * wx + uy * wy + uz * wz) / cn;
        // angle at a (opposite edge v-b): vectors a->v, a->b
        ux = vx - ax; uy = vy - ay; uz = vz - az; wx = bx - ax; wy = by - ay; wz = bz - az;
        cx = uy * wz - uz * wy; cy = uz * wx - ux * wz; cz = ux * wy - uy * wx;
        const double cot_a = (ux * wx + uy * wy + uz * wz) / sqrt(cx * cx + cy * cy + cz * cz);
        const int sa = M.slot_a[q], sb = M.slot_b[q];
        const double wa = ew ? (double)ew[M.edge_of_entry[sa]] : 1.0;
        const double wb = ew ? (double)ew[M.edge_of_entry[sb]] : 1.0;
        row(sa) += -0.5 * cot_b * wa;
        row(sb) += -0.5 * cot_a * wb;
        m += cn / 6.0;   // area / 3 = |cross| / 6
    }
    double off = 0.0;
    const int dp = M.diag_pos[v];
    for (int p = p0; p < p1; ++p) {
        if (p == dp) continue;
        const double lv = row(p);
        off += lv;
        if (l_vals) l_vals[p] = lv;
        a_vals[p] = t * lv;
    }
    if (l_vals) l_vals[dp] = -off;
    if (mass) mass[v] = m;
    a_vals[dp] = t * (-off) + (s ? s[v] : 1.0) * m;
}

// per-block partial of sum_i lam_i (L u)_i, stored as (sum, 0) pairs
__global__ __launch_bounds__(kBlock) void k_spmv_dot(const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ cols,
                                                     const double *__restrict__ vals,
                                                     const double *__restrict__ lam,
                                                     const double *__restrict__ u, int n,
                                                     double *__restrict__ partial) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        double acc = 0.0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) acc += vals[p] * u[cols[p]];
        v = lam[i] * acc;
    }
    __shared__ double red[kBlock / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) a += red[w];
        partial[2 * (size_t)blockIdx.x] = a;
        partial[2 * (size_t)blockIdx.x + 1] = 0.0;
    }
}
__global__ __launch_bounds__(kBlock) void k_mass_grad(const double *__restrict__ lam,
                                                      const double *__restrict__ m,
                                                      const double *__restrict__ u,
                                                      double *__restrict__ out, int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = -lam[i] * m[i] * u[i];
}

inline int nblocks(int64_t n, int per = kBlock) { return (int)((n + per - 1) / per); }

}  // namespace

// ============================================================== launchers
#define SMG_K_SWITCH(k, CALL) \
    switch (k) {              \
    case 1: { constexpr int KK = 1; CALL; break; } \
    case 2: { constexpr int KK = 2; CALL; break; } \
    case 3: { constexpr int KK = 3; CALL; break; } \
    case 4: { constexpr int KK = 4; CALL; break; } \
    default: return hipErrorInvalidValue; }

template <typename T>
hipError_t launch_gs_color(const SellView<T> &A, const ColorSpan &c, const T *b, T *x, int k,
                           hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    const int s_begin = c.s_begin, s_end = c.s_end;
    const int ns = s_end - s_begin;
    if (ns <= 0) return hipSuccess;
    const int g = nblocks(ns, kGsBlock / 64);
    if (c.w > 0) {
        if (ev0) {
            SMG_K_SWITCH(k, (hipExtLaunchKernelGGL(k_gs_color_w<KK, T>, dim3(g), dim3(kGsBlock), 0, st, ev0, ev1, 0,
                                                   ns, c.row0, c.row_end, c.off0, c.w, A.lpr, A.cols, A.vals,
                                                   A.diag, b, x)));
        } else {
            SMG_K_SWITCH(k, (k_gs_color_w<KK, T><<<g, kGsBlock, 0, st>>>(ns, c.row0, c.row_end, c.off0, c.w, A.lpr,
                                                                       A.cols, A.vals, A.diag, b, x)));
        }
        return hipGetLastError();
    }
    if (ev0) {
        SMG_K_SWITCH(k, (hipExtLaunchKernelGGL(k_gs_color<KK, T>, dim3(g), dim3(kGsBlock), 0, st, ev0, ev1, 0,
                                               s_begin, s_end, A.lpr, A.slice_row0, A.slice_off, A.cols,
                                               A.vals, A.diag, b, x)));
    } else {
        SMG_K_SWITCH(k, (k_gs_color<KK, T><<<g, kGsBlock, 0, st>>>(s_begin, s_end, A.lpr, A.slice_row0, A.slice_off,
                                                                 A.cols, A.vals, A.diag, b, x)));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi(const SellView<T> &A, int nslices, const T *b, const T *x, T *xo, const double *omega,
                         int k, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (nslices <= 0) return hipSuccess;
    const int g = nblocks(nslices, kBlock / 64);
    if (ev0) {
        SMG_K_SWITCH(k, (hipExtLaunchKernelGGL(k_jacobi<KK, T>, dim3(g), dim3(kBlock), 0, st, ev0, ev1, 0,
                                               nslices, A.lpr, A.slice_row0, A.slice_off, A.cols, A.vals,
                                               A.diag, b, x, xo, omega)));
    } else {
        SMG_K_SWITCH(k, (k_jacobi<KK, T><<<g, kBlock, 0, st>>>(nslices, A.lpr, A.slice_row0, A.slice_off, A.cols,
                                                               A.vals, A.diag, b, x, xo, omega)));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi_first(int n, int k, const T *diag, const T *b, T *xo, const double *omega, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nk = (int64_t)n * k;
    k_jacobi_first<T><<<nblocks(nk), kBlock, 0, st>>>(nk, k, diag, b, xo, omega);
    return hipGetLastError();
}
template hipError_t launch_jacobi_first<double>(int, int, const double *, const double *, double *, const double *,
                                                hipStream_t);
template hipError_t launch_jacobi_first<float>(int, int, const float *, const float *, float *, const double *,
                                               hipStream_t);

hipError_t launch_dirichlet_reduce(int nu, const int32_t *uidx, const int32_t *rowptr, const int32_t *cols,
                                   const double *vals, const uint8_t *known, const double *x, const double *b, int k,
                                   const int32_t *uptr, double *uvals, double *rhs, hipStream_t st) {
    if (nu <= 0) return hipSuccess;
    SMG_K_SWITCH(k, (k_dirichlet_reduce<KK><<<nblocks(nu), kBlock, 0, st>>>(nu, uidx, rowptr, cols, vals, known, x, b,
                                                                         uptr, uvals, rhs)));
    return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double *x, double b, const double *y, double *out,
                        hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_axpby<<<nblocks(n), kBlock, 0, st>>>(n, a, x, b, y, out);
    return hipGetLastError();
}

hipError_t launch_jacobi_factor(const SellView<double> &A, int n, int nslices, const int32_t *perm, double *v,
                                double *u, double *partial, double *sums, double *omega_l, hipStream_t st) {
    if (n <= 0 || nslices <= 0) return hipSuccess;
    const int g = nblocks(nslices, kBlock / 64);
    k_power_start<<<nblocks(n), kBlock, 0, st>>>(n, perm, v);
    for (int i = 0; i < kJacobiPowerSteps; ++i) {
        k_power_step<false><<<g, kBlock, 0, st>>>(nslices, A.lpr, A.slice_row0, A.slice_off, A.cols, A.vals, A.diag,
                                                  v, u, nullptr);
        double *t = v; v = u; u = t;
    }
    k_power_step<true><<<g, kBlock, 0, st>>>(nslices, A.lpr, A.slice_row0, A.slice_off, A.cols, A.vals, A.diag,
                                             v, nullptr, partial);
    k_reduce_partial<2><<<1, 1024, 0, st>>>(partial, g, sums, nullptr, 0.0);
    k_power_omega<<<1, 64, 0, st>>>(sums, omega_l);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(const SellView<T> &A, int nslices, const T *b, const T *x, T *r,
                           int k, double *partial, int *nblk, hipStream_t st, hipEvent_t ev0,
                           hipEvent_t ev1) {
    const int ns = nslices;
    const int g = nblocks(ns, kBlock / 64);
    *nblk = g;
    if (ns <= 0) return hipSuccess;
    if (ev0) {
        if (partial) {
            SMG_K_SWITCH(k, (hipExtLaunchKernelGGL(k_residual<KK, T, true>, dim3(g), dim3(kBlock), 0, st, ev0, ev1, 0,
                                                   ns, A.lpr, A.slice_row0, A.slice_off, A.cols, A.vals, A.diag,
                                                   b, x, r, partial, A.order)));
        } else {
            SMG_K_SWITCH(k, (hipExtLaunchKernelGGL(k_residual<KK, T, false>, dim3(g), dim3(kBlock), 0, st, ev0, ev1, 0,
                                                   ns, A.lpr, A.slice_row0, A.slice_off, A.cols, A.vals, A.diag,
                                                   b, x, r, (double *)nullptr, A.order)));
        }
    } else if (partial) {
        SMG_K_SWITCH(k, (k_residual<KK, T, true><<<g, kBlock, 0, st>>>(ns, A.lpr, A.slice_row0, A.slice_off, A.cols,
                                                                       A.vals, A.diag, b, x, r, partial, A.order)));
    } else {
        SMG_K_SWITCH(k, (k_residual<KK, T, false><<<g, kBlock, 0, st>>>(ns, A.lpr, A.slice_row0, A.slice_off, A.cols,
                                                                        A.vals, A.diag, b, x, r, nullptr, A.order)));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const TransferView &P, const T *rw, const T *r, T *rc, int k,
                           hipStream_t st, T *xc) {
    if (P.nc <= 0) return hipSuccess;
    const int lr = P.rs_lanes, rps = 64 / lr;
    const int64_t threads = (int64_t)((P.nc + rps - 1) / rps) * 64;
    SMG_K_SWITCH(k, (k_restrict<KK, T><<<nblocks(threads), kBlock, 0, st>>>(P.nc, lr, P.rs_off, P.rs_idx, rw, r,
                                                                            rc, xc, P.rs_order)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const TransferView &P, const T *pw, const T *e, T *x, int k,
                              hipStream_t st) {
    if (P.n <= 0) return hipSuccess;
    SMG_K_SWITCH(k, (k_prolong_add<KK, T><<<nblocks(P.n), kBlock, 0, st>>>(P.n, P.pc, pw, e, x)));
    return hipGetLastError();
}

hipError_t launch_colnorm_partial(const double *v, int n, int k, double *partial, int *nblk,
                                  hipStream_t st) {
    const int g = nblocks(n);
    *nblk = g;
    if (n <= 0) return hipSuccess;
    SMG_K_SWITCH(k, (k_colnorm_partial<KK><<<g, kBlock, 0, st>>>(v, n, partial)));
    return hipGetLastError();
}

hipError_t launch_reduce_partial(const double *partial, int nblk, int k, double *out,
                                 hipStream_t st, double *host_out, double seq) {
    SMG_K_SWITCH(k, (k_reduce_partial<KK><<<1, 1024, 0, st>>>(partial, nblk, out, host_out, seq)));
    return hipGetLastError();
}

hipError_t launch_cholesky(double *A, int n, int *flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n > kCoarseOneGroup) {   // many compute units, the trailing updates on the FP64 matrix cores
        for (int k0 = 0; k0 < n; k0 += kCholNb) {
            const int b = min(kCholNb, n - k0), m = n - k0 - b;
            k_chol_panel<<<max(1, (m + 255) / 256), 256, 0, st>>>(A, n, k0, b, flag);
            if (m > 0) {
                const int T = (m + 15) / 16, ntile = T * (T + 1) / 2;
                k_chol_update<<<(ntile + 3) / 4, 256, 0, st>>>(A, n, k0, b, ntile, flag);
            }
        }
        k_zero_upper<<<(int)(((int64_t)n * n + 255) / 256), 256, 0, st>>>(A, n);
        return hipGetLastError();
    }
    int nb = 16;   // panel width: the panel (n x nb doubles) must fit 128 KB of LDS
    while (nb > 1 && (size_t)n * nb * sizeof(double) > 128 * 1024) nb >>= 1;
    const size_t lds = (size_t)n * nb * sizeof(double);
    if (lds > 128 * 1024) {   // very large coarsest level: unblocked, in global memory
        k_cholesky<<<1, 1024, 0, st>>>(A, n, flag);
        return hipGetLastError();
    }
    hipError_t e = hipFuncSetAttribute((const void *)k_cholesky_blocked, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_cholesky_blocked<<<1, 1024, lds, st>>>(A, n, nb, flag);
    return hipGetLastError();
}

template <typename Tin, typename Tout>
hipError_t launch_coarse_solve(const double *Ainv, int n, const Tin *b, Tout *x, int k,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    SMG_K_SWITCH(k, (k_coarse_apply<KK, Tin, Tout><<<nblocks(n, kBlock / 64), kBlock, 0, st>>>(Ainv, n, b, x)));
    return hipGetLastError();
}

hipError_t launch_coarse_inverse(const double *G, int n, double *W, double *Ainv, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n > kCoarseOneGroup) {   // blocked, the updates and W^T W on the FP64 matrix cores
        k_identity<<<(int)(((int64_t)n * n + 255) / 256), 256, 0, st>>>(W, n);
        for (int k0 = 0; k0 < n; k0 += kCholNb) {
            const int b = min(kCholNb, n - k0), m = n - k0 - b;
            k_trinv_rows<<<(k0 + b + 255) / 256, 256, 0, st>>>(G, W, n, k0, b);
            if (m > 0) {
                const int tr = (m + 15) / 16, tc = (k0 + b + 15) / 16, ntile = tr * tc;
                k_trinv_update<<<(ntile + 3) / 4, 256, 0, st>>>(G, W, n, k0, b, tc, ntile);
            }
        }
        const int T = (n + 31) / 32, ntile = T * (T + 1) / 2;
        k_inv_syrk<<<(ntile + 3) / 4, 256, 0, st>>>(W, Ainv, n, ntile);
        return hipGetLastError();
    }
    const size_t lds = (size_t)4 * n * sizeof(double);
    if (lds <= 128 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_tri_inverse_cols, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        k_tri_inverse_cols<<<(n + 3) / 4, 256, lds, st>>>(G, n, W);
    } else {
        k_tri_inverse<<<1, 1024, 0, st>>>(G, n, W);
    }
    k_inverse_product<<<nblocks((int64_t)n * n), kBlock, 0, st>>>(W, n, Ainv);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_lds(const LdsLevel<T> *lv, const int32_t *passes, const int32_t *waves,
                           int first, int nlev, int mu_pre, int mu_post, const double *Ainv, int k,
                           size_t lds_bytes, hipStream_t st, bool post_desc, bool per_column) {
    if (per_column) {   // one workgroup per right-hand side, all in parallel
        k_tail_lds<1, T><<<k, kTailThreads, lds_bytes, st>>>(
            lv, reinterpret_cast<const int4 *>(passes), reinterpret_cast<const int2 *>(waves), first, nlev, mu_pre,
            mu_post, Ainv, post_desc ? 1 : 0, k);
        return hipGetLastError();
    }
    SMG_K_SWITCH(k, (k_tail_lds<KK, T><<<1, kTailThreads, lds_bytes, st>>>(
                        lv, reinterpret_cast<const int4 *>(passes), reinterpret_cast<const int2 *>(waves),
                        first, nlev, mu_pre, mu_post, Ainv, post_desc ? 1 : 0, k)));
    return hipGetLastError();
}

hipError_t launch_cg_spmv(const SellView<double> &A, int nslices, const double *p, double *ap, int k,
                          double *partial, int *nblk, hipStream_t st) {
    const int g = nblocks(nslices, kBlock / 64);
    *nblk = g;
    if (nslices <= 0) return hipSuccess;
    SMG_K_SWITCH(k, (k_cg_spmv<KK><<<g, kBlock, 0, st>>>(nslices, A.lpr, A.slice_row0, A.slice_off, A.cols,
                                                         A.vals, A.diag, p, ap, partial, A.order)));
    return hipGetLastError();
}

hipError_t launch_cg_update(int n, const double *rz, const double *pap, const double *p, const double *ap,
                            double *x, double *r, int k, double *partial, int *nblk, hipStream_t st) {
    const int g = nblocks(n);
    *nblk = g;
    if (n <= 0) return hipSuccess;
    SMG_K_SWITCH(k, (k_cg_update<KK><<<g, kBlock, 0, st>>>(n, rz, pap, p, ap, x, r, partial)));
    return hipGetLastError();
}

hipError_t launch_cg_dot(int n, const double *r, const double *z64, const float *z32, const double *zscale,
                         int k, double *partial, int *nblk, hipStream_t st) {
    const int g = nblocks(n);
    *nblk = g;
    if (n <= 0) return hipSuccess;
    if (z32) {
        SMG_K_SWITCH(k, (k_cg_dot<KK, true><<<g, kBlock, 0, st>>>(n, r, z64, z32, zscale, partial)));
    } else {
        SMG_K_SWITCH(k, (k_cg_dot<KK, false><<<g, kBlock, 0, st>>>(n, r, z64, z32, zscale, partial)));
    }
    return hipGetLastError();
}

hipError_t launch_cg_direction(int n, const double *rz_new, const double *rz_old, double *z64, float *z32,
                               const double *zscale, double *p, int k, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int g = nblocks((int64_t)n * k);
    if (z32) {
        SMG_K_SWITCH(k, (k_cg_direction<KK, true><<<g, kBlock, 0, st>>>(n, rz_new, rz_old, z64, z32, zscale, p)));
    } else {
        SMG_K_SWITCH(k, (k_cg_direction<KK, false><<<g, kBlock, 0, st>>>(n, rz_new, rz_old, z64, z32, zscale, p)));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_step(const LdsLevel<T> *lv, const int32_t *passes, const int32_t *waves, int l, int nlev,
                            int op, int sweeps, bool desc, const double *Ainv, int k, size_t lds_bytes,
                            hipStream_t st) {
    // one workgroup per right-hand side, as k_tail_lds runs them
    const void *f = (const void *)k_tail_step<1, T>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    k_tail_step<1, T><<<k, kTailThreads, lds_bytes, st>>>(lv, reinterpret_cast<const int4 *>(passes),
                                                         reinterpret_cast<const int2 *>(waves), l, nlev, op,
                                                         sweeps, desc ? 1 : 0, Ainv, k);
    return hipGetLastError();
}
template hipError_t launch_tail_step<double>(const LdsLevel<double> *, const int32_t *, const int32_t *, int, int,
                                             int, int, bool, const double *, int, size_t, hipStream_t);
template hipError_t launch_tail_step<float>(const LdsLevel<float> *, const int32_t *, const int32_t *, int, int,
                                            int, int, bool, const double *, int, size_t, hipStream_t);

// Dynamic LDS above the default limit must be granted per kernel once.
template <typename T>
hipError_t tail_lds_allow(size_t bytes) {
    hipError_t e = hipSuccess;
    for (const void *f : {(const void *)k_tail_lds<1, T>, (const void *)k_tail_lds<2, T>,
                          (const void *)k_tail_lds<3, T>, (const void *)k_tail_lds<4, T>})
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return e;
}
template hipError_t tail_lds_allow<double>(size_t);
template hipError_t tail_lds_allow<float>(size_t);

hipError_t launch_gather_records(const int32_t *src, const int32_t *cols, int64_t n,
                                 const double *vals, const float *vals32, TailRec<double> *rec64,
                                 TailRec<float> *rec32, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_gather_records<<<nblocks(n), kBlock, 0, st>>>(src, cols, n, vals, vals32, rec64, rec32);
    return hipGetLastError();
}

hipError_t launch_batch_solve(const BatchMesh *meshes, const int32_t *team_mesh,
                              const int32_t *team_rank, int nblocks_total, int threads,
                              unsigned *ctrs, int *aborts, double *partials, int count,
                              hipStream_t st) {
    if (nblocks_total <= 0) return hipSuccess;
    if (threads != 256 && threads != 512 && threads != 1024) return hipErrorInvalidValue;
    k_fill<unsigned><<<nblocks((int64_t)count * kBatchCtrStride), kBlock, 0, st>>>(ctrs, 0u,
                                                                                  (int64_t)count * kBatchCtrStride);
    k_fill<int><<<nblocks(count), kBlock, 0, st>>>(aborts, 0, count);
    if (threads == 256) k_batch_solve<256><<<nblocks_total, 256, 0, st>>>(meshes, team_mesh, team_rank, ctrs, aborts, partials);
    else if (threads == 512) k_batch_solve<512><<<nblocks_total, 512, 0, st>>>(meshes, team_mesh, team_rank, ctrs, aborts, partials);
    else k_batch_solve<1024><<<nblocks_total, 1024, 0, st>>>(meshes, team_mesh, team_rank, ctrs, aborts, partials);
    return hipGetLastError();
}

// Launch-latency probes with the grid of a relaxation launch (64-thread
// workgroups, xcd_block order): an empty kernel, and one whose every thread
// loads an index, then the value it points to, and stores it (the dependent
// chain of a relaxation: matrix entry, then neighbour gather, then store).
__global__ __launch_bounds__(kGsBlock) void k_floor_empty() {}
__global__ __launch_bounds__(kGsBlock) void k_floor_chain(const int32_t *__restrict__ idx,
                                                          const float *__restrict__ v, float *__restrict__ out,
                                                          int n) {
    const int t = xcd_block(blockIdx.x, gridDim.x) * kGsBlock + threadIdx.x;
    if (t >= n) return;
    out[t] = v[idx[t]];
}
hipError_t launch_floor(int kind, int nblk, const int32_t *idx, const float *v, float *out, int n, hipStream_t st) {
    if (kind == 0) k_floor_empty<<<nblk, kGsBlock, 0, st>>>();
    else k_floor_chain<<<nblk, kGsBlock, 0, st>>>(idx, v, out, n);
    return hipGetLastError();
}

// one wavefront sleeping for a fixed count (~3.4 us per iteration): holds a
// stream while the host queues work behind it
__global__ __launch_bounds__(64) void k_delay(int iters) {
    for (int i = 0; i < iters; ++i) __builtin_amdgcn_s_sleep(127);
}
hipError_t launch_delay(int iters, hipStream_t st) {
    k_delay<<<1, 64, 0, st>>>(iters);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_team_vcycle(const TailLevel<T> *lv, int first, int nlev, int mu_pre, int mu_post,
                              const double *Ainv, unsigned *cb, int *flag, int m, int k, hipStream_t st) {
    k_fill<unsigned><<<1, kBlock, 0, st>>>(cb, 0u, 64);   // election, ranks, barrier counter
    SMG_K_SWITCH(k, (k_team_vcycle<KK, T><<<8 * m, 1024, 0, st>>>(lv, first, nlev, mu_pre, mu_post, Ainv, cb,
                                                                    flag, m)));
    return hipGetLastError();
}
template hipError_t launch_team_vcycle<float>(const TailLevel<float> *, int, int, int, int, const double *,
                                              unsigned *, int *, int, int, hipStream_t);
template hipError_t launch_team_vcycle<double>(const TailLevel<double> *, int, int, int, int, const double *,
                                               unsigned *, int *, int, int, hipStream_t);

int batch_blocks_per_cu(int threads) {
    int occ = 0;
    hipError_t e = hipErrorInvalidValue;
    if (threads == 256) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_solve<256>, 256, 0);
    else if (threads == 512) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_solve<512>, 512, 0);
    else if (threads == 1024) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_solve<1024>, 1024, 0);
    return e == hipSuccess ? occ : 0;
}

hipError_t launch_scatter_values(const double *src, const int32_t *store, int64_t nnz,
                                 double *vals, double *diag, int *flag, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    k_scatter_values<<<nblocks(nnz), kBlock, 0, st>>>(src, store, nnz, vals, diag, flag);
    return hipGetLastError();
}

// threads per block so that every thread has `slots` doubles of LDS
// Lanes per output row of the Galerkin kernels on levels below kGalerkinLanesBelow
// rows, whose products are latency-bound; larger levels keep one thread per
// row (measured: 4 lanes made the 250k-row product 33% slower, the small ones
// 15-40% faster).
constexpr int kGalerkinLanes = 4;
constexpr int kGalerkinLanesBelow = 32768;
static int galerkin_block(int slots) {
    int bs = 64;
    while (bs > 1 && (size_t)bs * slots * sizeof(double) > 160 * 1024) bs >>= 1;
    return bs;
}

hipError_t launch_galerkin_t(int n, int tmax, const int32_t *tptr, const int32_t *plan1ptr,
                             const uint16_t *plan1, const int32_t *row_slice,
                             const int32_t *slice_row0, const int32_t *slice_off, int lpr,
                             const int32_t *rowlen, const int32_t *cols, const double *vals,
                             const double *diag, const double *pw, double *Tbuf, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int slots = tmax > 0 ? tmax : 1, bs = galerkin_block(slots);
    const size_t lds = (size_t)bs * slots * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)k_galerkin_t<kGalerkinLanes>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_galerkin_t<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (bs >= kGalerkinLanes && n < kGalerkinLanesBelow) {
        const int rows = bs / kGalerkinLanes;
        k_galerkin_t<kGalerkinLanes><<<(n + rows - 1) / rows, bs, lds, st>>>(
            n, tptr, plan1ptr, plan1, row_slice, slice_row0, slice_off, lpr, rowlen, cols, vals, diag, pw, Tbuf);
    } else {
        k_galerkin_t<1><<<(n + bs - 1) / bs, bs, lds, st>>>(n, tptr, plan1ptr, plan1, row_slice, slice_row0,
                                                            slice_off, lpr, rowlen, cols, vals, diag, pw, Tbuf);
    }
    return hipGetLastError();
}

hipError_t launch_galerkin_c(int nc, int cmax, const int32_t *plan2ptr, const uint16_t *plan2,
                             const int32_t *rptr, const int32_t *ridx, const double *rw,
                             const int32_t *tptr, const double *Tbuf, const int32_t *optr,
                             const int32_t *opos, double *vals, double *diag, hipStream_t st) {
    if (nc <= 0) return hipSuccess;
    const int slots = cmax > 0 ? cmax : 1, bs = galerkin_block(slots);
    const size_t lds = (size_t)bs * slots * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)k_galerkin_c<kGalerkinLanes>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_galerkin_c<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (bs >= kGalerkinLanes && nc < kGalerkinLanesBelow) {
        const int rows = bs / kGalerkinLanes;
        k_galerkin_c<kGalerkinLanes><<<(nc + rows - 1) / rows, bs, lds, st>>>(nc, plan2ptr, plan2, rptr, ridx, rw,
                                                                              tptr, Tbuf, optr, opos, vals, diag);
    } else {
        k_galerkin_c<1><<<(nc + bs - 1) / bs, bs, lds, st>>>(nc, plan2ptr, plan2, rptr, ridx, rw, tptr, Tbuf,
                                                             optr, opos, vals, diag);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T *p, T v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_fill<T><<<nblocks(n), kBlock, 0, st>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_to_f32<<<nblocks(n), kBlock, 0, st>>>(src, dst, n);
    return hipGetLastError();
}

template <typename Ts, typename Td>
hipError_t launch_gather_rows(const int32_t *perm, const Ts *src, Td *dst, int n, int k, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_gather_rows<Ts, Td><<<nblocks((int64_t)n * k), kBlock, 0, st>>>(perm, src, dst, n, k);
    return hipGetLastError();
}
template hipError_t launch_gather_rows<double, double>(const int32_t *, const double *, double *, int, int,
                                                       hipStream_t);
template hipError_t launch_gather_rows<double, float>(const int32_t *, const double *, float *, int, int,
                                                      hipStream_t);

template <typename Ts, typename Td>
hipError_t launch_scatter_rows(const int32_t *perm, const Ts *src, Td *dst, int n, int k, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_scatter_rows<Ts, Td><<<nblocks((int64_t)n * k), kBlock, 0, st>>>(perm, src, dst, n, k);
    return hipGetLastError();
}
template hipError_t launch_scatter_rows<double, double>(const int32_t *, const double *, double *, int, int,
                                                        hipStream_t);
template hipError_t launch_scatter_rows<float, double>(const int32_t *, const float *, double *, int, int,
                                                       hipStream_t);

hipError_t launch_check_finite(const double *v, int64_t n, int *flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_check_finite<<<nblocks(n), kBlock, 0, st>>>(v, n, flag);
    return hipGetLastError();
}

hipError_t launch_ir_down(const double *r64, const double *norms, float *r32, int n, int k,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_ir_down<<<nblocks((int64_t)n * k), kBlock, 0, st>>>(r64, norms, r32, n, k);
    return hipGetLastError();
}

hipError_t launch_ir_up(float *d32, const double *norms, double *x64, int n, int k,
                        hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_ir_up<<<nblocks((int64_t)n * k), kBlock, 0, st>>>(d32, norms, x64, n, k);
    return hipGetLastError();
}

hipError_t launch_assemble(const MeshView &M, const double *V, double t, const double *mass_scale,
                           const float *edge_w, double *a_vals, double *l_vals, double *mass,
                           hipStream_t st) {
    if (M.n <= 0) return hipSuccess;
    k_assemble<<<nblocks(M.n), kBlock, 0, st>>>(M, V, t, mass_scale, edge_w, a_vals, l_vals, mass);
    return hipGetLastError();
}

hipError_t launch_spmv_dot(const int32_t *rowptr, const int32_t *cols, const double *vals,
                           const double *lam, const double *u, int n, double *partial,
                           int *nblk, hipStream_t st) {
    const int g = nblocks(n);
    *nblk = g;
    if (n <= 0) return hipSuccess;
    k_spmv_dot<<<g, kBlock, 0, st>>>(rowptr, cols, vals, lam, u, n, partial);
    return hipGetLastError();
}

hipError_t launch_mass_grad(const double *lam, const double *m, const double *u, double *out,
                            int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_mass_grad<<<nblocks(n), kBlock, 0, st>>>(lam, m, u, out, n);
    return hipGetLastError();
}

template hipError_t launch_gs_color<double>(const SellView<double> &, const ColorSpan &, const double *,
                                            double *, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_gs_color<float>(const SellView<float> &, const ColorSpan &, const float *,
                                           float *, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_jacobi<double>(const SellView<double> &, int, const double *, const double *,
                                          double *, const double *, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_jacobi<float>(const SellView<float> &, int, const float *, const float *, float *,
                                         const double *, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_residual<double>(const SellView<double> &, int, const double *,
                                            const double *, double *, int, double *, int *,
                                            hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_residual<float>(const SellView<float> &, int, const float *,
                                           const float *, float *, int, double *, int *,
                                           hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_restrict<double>(const TransferView &, const double *, const double *,
                                            double *, int, hipStream_t, double *);
template hipError_t launch_restrict<float>(const TransferView &, const float *, const float *,
                                           float *, int, hipStream_t, float *);
template hipError_t launch_prolong_add<double>(const TransferView &, const double *,
                                               const double *, double *, int, hipStream_t);
template hipError_t launch_prolong_add<float>(const TransferView &, const float *, const float *,
                                              float *, int, hipStream_t);
template hipError_t launch_coarse_solve<double, double>(const double *, int, const double *,
                                                        double *, int, hipStream_t);
template hipError_t launch_coarse_solve<float, float>(const double *, int, const float *, float *,
                                                      int, hipStream_t);
template hipError_t launch_tail_lds<double>(const LdsLevel<double> *, const int32_t *, const int32_t *,
                                            int, int, int, int, const double *, int, size_t, hipStream_t, bool,
                                            bool);
template hipError_t launch_tail_lds<float>(const LdsLevel<float> *, const int32_t *, const int32_t *,
                                           int, int, int, int, const double *, int, size_t, hipStream_t, bool,
                                           bool);
template hipError_t launch_fill<double>(double *, double, int64_t, hipStream_t);
template hipError_t launch_fill<float>(float *, float, int64_t, hipStream_t);
template hipError_t launch_fill<int>(int *, int, int64_t, hipStream_t);
template hipError_t launch_fill<unsigned>(unsigned *, unsigned, int64_t, hipStream_t);

}  // namespace smg
