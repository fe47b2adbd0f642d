// PCA of the rows of X to p dimensions, the preprocessing the paper applies
// before its k-NN stage (pca_dim; sections "Reproducibility" and "Scaling
// Behavior"), in FP64 from the stored values:
//
//  1. mean:     column sums over fixed row chunks, then summed in chunk order;
//  2. Gram:     C = (X - mu)^T (X - mu) / (n - 1) on v_mfma_f64_16x16x4_f64,
//               upper-triangle 64x64 tiles, one partial per 4096-row chunk
//               (rows staged in LDS as FP32, centred as they become
//               operands), partials summed in chunk order: no atomics, so
//               the result does not depend on scheduling;
//  3. subspace: m = min(d, 80, max(2p, p + 16)) columns V (seeded, hashed
//               values) iterate V <- orth(C V) (C V on
//               v_mfma_f64_16x16x4_f64), orthonormalised by one shifted
//               Cholesky-QR pass every q products (q from the basis'
//               estimated conditioning, 1..8) and by shifted + two plain
//               passes after the last (Cholesky-QR3); then
//               Rayleigh-Ritz: H = V^T C V, whose eigenpairs come from cyclic
//               Jacobi rotations (one workgroup, round-robin pairing), and
//               the p largest Ritz pairs are kept; each eigenvector's entry
//               of largest magnitude is made positive;
//  4. project:  Z = (X - mu) V_p, rounded to FP32.
// When m = d the Ritz pairs are the exact eigenpairs of C.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "knn_common.hpp"

namespace knn {

constexpr int kPcaMaxP = 64;      // components
constexpr int kPcaMaxM = 80;      // subspace width (an m x m double matrix fits in LDS)
static_assert(kPcaMaxM % 16 == 0, "LDS kernels stride columns by 16");
constexpr int kPcaChunk = 4096;   // rows per Gram partial
constexpr int kPcaSumChunk = 512; // rows per column-sum partial
constexpr int kPcaMaxQ = 8;       // products C V between orthonormalisations, at most
constexpr int kPcaTile = 64;      // Gram tile edge

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ mean

// part[c][t] = sum of column t over rows [c * kPcaSumChunk, ...), in row order
// (thread t of a 256-wide column block walks the chunk's rows).
template <int DT>
__global__ __launch_bounds__(256) void pca_colsum_kernel(const void* __restrict__ X, int64_t n, int64_t ld, int d,
                                                         double* __restrict__ part)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (t >= d) return;
    const int64_t r0 = c * kPcaSumChunk, r1 = r0 + kPcaSumChunk < n ? r0 + kPcaSumChunk : n;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += (double)elem<DT>::ld(X, r * ld + t);
    part[c * d + t] = s;
}

__global__ __launch_bounds__(256) void pca_mean_kernel(const double* __restrict__ part, int nch, int d, int64_t n,
                                                       double* __restrict__ mu)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= d) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[(int64_t)c * d + t];
    mu[t] = s / (double)n;
}

// ------------------------------------------------------------------ Gram

// Tile (ta, tb), ta <= tb, of chunk c: G[a][b] over the chunk's rows for
// columns a in [64 ta, +64), b in [64 tb, +64).  Rows are staged 64 at a
// time (FP32, both column slices).  Wave w owns tile rows 16w .. 16w+15 and
// all 64 tile columns: four 16x16 f64 accumulators.  v_mfma_f64_16x16x4:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator item
// i of lane l is D[l / 16 + 4 i][l % 16] (rows interleaved by 4).
template <int DT>
__global__ __launch_bounds__(256) void pca_gram_kernel(const void* __restrict__ X, int64_t n, int64_t ld, int d,
                                                       const double* __restrict__ mu, const int2* __restrict__ tiles,
                                                       double* __restrict__ part)
{
    __shared__ float sa[64][kPcaTile + 1];
    __shared__ float sb[64][kPcaTile + 1];
    __shared__ double sma[kPcaTile], smb[kPcaTile];
    const int2 tt = tiles[blockIdx.x];
    const int64_t c = blockIdx.y;
    const int a0 = tt.x * kPcaTile, b0 = tt.y * kPcaTile;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t r0 = c * kPcaChunk, r1 = r0 + kPcaChunk < n ? r0 + kPcaChunk : n;
    if (tid < kPcaTile) {
        sma[tid] = a0 + tid < d ? mu[a0 + tid] : 0.0;
        smb[tid] = b0 + tid < d ? mu[b0 + tid] : 0.0;
    }
    // staging: thread (rq, cc) holds rows rq, rq + 4, ..., rq + 60 of column
    // cc of both slices; the next 64 rows are loaded while this step's
    // MFMAs run (zeros past d and past the chunk)
    const int cc = tid & 63, rq = tid >> 6;
    const bool acol = a0 + cc < d, bcol = b0 + cc < d;
    float pa[16], pb[16];
    auto fetch = [&](int64_t rs) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int64_t row = rs + rq + 4 * u;
            const bool ok = row < r1;
            pa[u] = ok && acol ? elem<DT>::ld(X, row * ld + a0 + cc) : 0.0f;
            pb[u] = ok && bcol ? elem<DT>::ld(X, row * ld + b0 + cc) : 0.0f;
        }
    };
    fetch(r0);
    f64x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int ia = 16 * w + (lane & 15);
    for (int64_t rs = r0; rs < r1; rs += 64) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            sa[rq + 4 * u][cc] = pa[u];
            sb[rq + 4 * u][cc] = pb[u];
        }
        __syncthreads();
        if (rs + 64 < r1) fetch(rs + 64);
        const int nr = (int)(r1 - rs < 64 ? r1 - rs : 64);
#pragma unroll 4
        for (int k0 = 0; k0 < 64; k0 += 4) {
            const int kk = k0 + (lane >> 4);
            const bool kv = kk < nr;
            // centred operands; padded rows and columns contribute 0
            const float xa = sa[kk][ia];
            const double av = kv ? (double)xa - sma[ia] : 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int jb = 16 * j + (lane & 15);
                const float xb = sb[kk][jb];
                const double bv = kv ? (double)xb - smb[jb] : 0.0;
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[j], 0, 0, 0);
            }
        }
    }
    // partial tile, full 64 x 64 block of the chunk's d x d matrix
    double* out = part + c * (int64_t)d * d;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ra = a0 + 16 * w + (lane >> 4) + 4 * i, cb = b0 + 16 * j + (lane & 15);
            if (ra < d && cb < d) out[(int64_t)ra * d + cb] = acc[j][i];
        }
    }
}

// C[a][b] = sum of the chunk partials (chunk order) / (n - 1) for a <= b
// (inside the upper tiles computed), mirrored to C[b][a].
__global__ __launch_bounds__(256) void pca_gram_reduce_kernel(const double* __restrict__ part, int nch, int d,
                                                              int64_t n, double* __restrict__ C)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)d * d) return;
    const int a = (int)(e / d), b = (int)(e % d);
    if (a > b) return;   // the lower triangle is mirrored from the upper one
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[(int64_t)c * d * d + e];
    s /= (double)(n - 1);
    C[(int64_t)a * d + b] = s;
    C[(int64_t)b * d + a] = s;
}

// ------------------------------------------------------------------ subspace

// V (m columns of length d, column-major) from hashed values in [-1, 1).
__global__ __launch_bounds__(256) void pca_init_kernel(int d, int m, uint64_t seed, double* __restrict__ V)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)d * m) return;
    V[e] = 2.0 * ((double)(hash4(seed, 11, (uint64_t)e, 0) >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

// V = the first m columns of the d x d identity (column-major).
__global__ __launch_bounds__(256) void pca_identity_kernel(int d, int m, double* __restrict__ V)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)d * m) return;
    V[e] = (e / d == e % d) ? 1.0 : 0.0;
}

// W = C V on v_mfma_f64_16x16x4_f64, one workgroup per 16 x 16 block of W
// (rows a of C, columns j of V).  K runs in blocks of 16, block b taken by
// wave b % 4 (four blocks per round, loads first): lane l (r = l % 16, g = l / 16) holds C[a0 + r][k0 + 4g ..
// +3] and V[j0 + r][k0 + 4g .. +3], and step s multiplies the k = k0 + 4g +
// s slice, so every k enters once; entries past d or m are zero.  The four
// waves' sums are added in wave order.  Accumulator item i of lane l is
// W[j0 + r][a0 + g + 4i].
__global__ __launch_bounds__(256) void pca_cv_kernel(const double* __restrict__ C, const double* __restrict__ V, int d,
                                                     int m, double* __restrict__ W)
{
    __shared__ double part[3][64][4];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, r = l & 15, g = l >> 4;
    const int a0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
    const bool aok = a0 + r < d, jok = j0 + r < m;
    const double* crow = C + (int64_t)(aok ? a0 + r : 0) * d;
    const double* vcol = V + (int64_t)(jok ? j0 + r : 0) * d;
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
    // four of the wave's K blocks per round, all their loads issued first
    for (int kb = 16 * wv; kb < d; kb += 256) {
        double ca[4][4], vb[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = kb + 64 * b + 4 * g + s;
                ca[b][s] = aok && k < d ? crow[k] : 0.0;
                vb[b][s] = jok && k < d ? vcol[k] : 0.0;
            }
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[b][s], vb[b][s], acc, 0, 0, 0);
    }
    if (wv > 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) part[wv - 1][l][i] = acc[i];
    }
    __syncthreads();
    if (wv == 0 && jok) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double v = ((acc[i] + part[0][l][i]) + part[1][l][i]) + part[2][l][i];
            const int a = a0 + g + 4 * i;
            if (a < d) W[(int64_t)(j0 + r) * d + a] = v;
        }
    }
}

// S[i][j] = <W_i, W_j> over d (i <= j; mirrored), one workgroup per pair,
// a fixed-order tree over the 256 thread sums.
__global__ __launch_bounds__(256) void pca_gram_small_kernel(const double* __restrict__ W, const double* __restrict__ U,
                                                             int d, int m, double* __restrict__ S)
{
    __shared__ double red[256];
    const int i = blockIdx.x, j = blockIdx.y;
    if (U == W && i > j) return;
    const double* wi = U + (int64_t)i * d;
    const double* wj = W + (int64_t)j * d;
    double s = 0.0;
    for (int a = threadIdx.x; a < d; a += 256) s = fma(wi[a], wj[a], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        S[i * m + j] = red[0];
        if (U == W) S[j * m + i] = red[0];
    }
}

// One Cholesky-QR pass: V = W R^{-1}, where S = W^T W = R^T R (R upper
// triangular).  Every workgroup factors S (its entries in registers, 25 per
// thread), the same operations in each, so all hold the same factor; then
// it forms 64 rows of W R^{-1} for its eight columns.  The factor comes from
// symmetric elimination on [S | I] (one barrier per step, the pivot row
// passed through LDS): step k subtracts
// S[k][i] / S[k][k] times row k from each row i > k, on the trailing upper
// triangle of S and on the unit lower triangular M beside it, so that at
// the end M S = D L^T with S = L D L^T (L unit lower triangular, D the
// pivots) and M = L^{-1}.  Then R = D^{1/2} L^T and R^{-1}[i][j] = M[j][i] /
// sqrt(D[j]): no triangular solve is needed.  M's strict lower triangle sits
// in the lower half of S, which the upper-triangle elimination never reads.  With shift_rel > 0 the factored matrix is
// S + s I, s = shift_rel * trace(S) (shifted Cholesky-QR: V spans the same
// space as W, but is only near-orthonormal, and no pivot can fail however
// badly W is conditioned).  A non-positive pivot (W of lower rank than m,
// unshifted) is replaced by 1 and flagged, which keeps the factor finite.
// The pivots D[k] (as used) go to `pivots`: their spread estimates W's
// conditioning.
constexpr int kPcaCols = 8;

__global__ __launch_bounds__(256) void pca_cholqr_kernel(const double* __restrict__ Sg, const double* __restrict__ W,
                                                         int d, int m, double* __restrict__ V,
                                                         unsigned* __restrict__ bad, double* __restrict__ pivots,
                                                         double shift_rel)
{
    __shared__ double S[kPcaMaxM * kPcaMaxM];   // the result: upper R-scaled rows, strict lower M
    __shared__ double rowk[2][kPcaMaxM];         // the step's pivot row (double-buffered)
    __shared__ double rinv[kPcaMaxM];
    __shared__ double diag[kPcaMaxM];
    __shared__ double shift_;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    // thread (ty, tx) owns entries (ty + 16u, tx + 16q), u, q < NJ, held in
    // registers through the whole elimination; only the pivot row of each
    // step goes through LDS (one barrier per step)
    constexpr int NJ = kPcaMaxM / 16;
    double x[NJ][NJ];
#pragma unroll
    for (int u = 0; u < NJ; ++u)
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const int i = ty + 16 * u, j = tx + 16 * q;
            x[u][q] = i < m && j < m && j >= i ? Sg[i * m + j] : 0.0;
        }
    if (shift_rel > 0.0) {
        // S + s I with s = shift_rel * trace(S): the same span, positive
        // pivots however badly W is conditioned
        if (ty == tx) {
#pragma unroll
            for (int u = 0; u < NJ; ++u) diag[ty + 16 * u] = x[u][u];
        }
        __syncthreads();
        if (tid == 0) {
            double tr = 0.0;
            for (int k = 0; k < m; ++k) tr += diag[k];
            shift_ = shift_rel * tr;
        }
        __syncthreads();
        if (ty == tx) {
#pragma unroll
            for (int u = 0; u < NJ; ++u)
                if (ty + 16 * u < m) x[u][u] += shift_;
        }
    }
    if (ty == 0) {
#pragma unroll
        for (int q = 0; q < NJ; ++q) rowk[0][tx + 16 * q] = x[0][q];
    }
    for (int k = 0; k < m; ++k) {
        __syncthreads();
        const double* rk = rowk[k & 1];
        double pk = rk[k];
        if (!(pk > 0.0)) {
            if (tid == 0 && blockIdx.x == 0 && blockIdx.y == 0) atomicOr(bad, 1u);
            pk = 1.0;
        }
        const double ip = 1.0 / pk;
        double rkq[NJ], fu[NJ];
#pragma unroll
        for (int q = 0; q < NJ; ++q) rkq[q] = rk[tx + 16 * q];
#pragma unroll
        for (int u = 0; u < NJ; ++u) fu[u] = rk[ty + 16 * u] * ip;
#pragma unroll
        for (int u = 0; u < NJ; ++u)
#pragma unroll
            for (int q = 0; q < NJ; ++q) {
                const int i = ty + 16 * u, j = tx + 16 * q;
                // rows below k: the upper triangle (j >= i) and M (j < k) take
                // row k's entry; M's column k takes its unit diagonal; k < j < i
                // stays 0
                const double nv = (j >= i || j < k) ? fma(-fu[u], rkq[q], x[u][q])
                                                    : (j == k ? x[u][q] - fu[u] : x[u][q]);
                x[u][q] = i > k ? nv : x[u][q];
            }
        if (tid == 0) {
            rinv[k] = 1.0 / sqrt(pk);
            if (blockIdx.x == 0 && blockIdx.y == 0) pivots[k] = pk;
        }
        // row k + 1 is final now: its owners publish it for the next step
        const int k1 = k + 1;
        if (k1 < m && ty == (k1 & 15)) {
#pragma unroll
            for (int u = 0; u < NJ; ++u)
                if (u == (k1 >> 4)) {
#pragma unroll
                    for (int q = 0; q < NJ; ++q) rowk[k1 & 1][tx + 16 * q] = x[u][q];
                }
        }
    }
#pragma unroll
    for (int u = 0; u < NJ; ++u)
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
            const int i = ty + 16 * u, j = tx + 16 * q;
            if (i < m && j < m) S[i * m + j] = x[u][q];
        }
    __syncthreads();
    // V = W R^{-1} for rows a0 .. a0 + 63 and the workgroup's eight columns:
    // wave g sums the products over its quarter of the index range i (so
    // each thread issues a quarter of the row loads), and the four partial
    // sums are added in wave order
    const int r = tid & 63, g = tid >> 6;
    const int a = blockIdx.x * 64 + r;
    const int j0 = blockIdx.y * kPcaCols;
    const int jmax = j0 + kPcaCols < m ? j0 + kPcaCols : m;
    const int ilen = (jmax + 3) / 4, ib = g * ilen, ie = ib + ilen < jmax ? ib + ilen : jmax;
    double sp[kPcaCols];
#pragma unroll
    for (int q = 0; q < kPcaCols; ++q) sp[q] = 0.0;
    if (a < d) {
        for (int i0 = ib; i0 < ie; i0 += 8) {
            double wv[8];   // eight rows of W in flight at once
#pragma unroll
            for (int u = 0; u < 8; ++u) wv[u] = i0 + u < ie ? W[(int64_t)(i0 + u) * d + a] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u;
#pragma unroll
                for (int q = 0; q < kPcaCols; ++q) {
                    const int j = j0 + q;
                    if (i < ie && j < m && i <= j) sp[q] = i == j ? sp[q] + wv[u] : fma(wv[u], S[j * m + i], sp[q]);
                }
            }
        }
    }
    __shared__ double part[3][64][kPcaCols];
    if (g > 0) {
#pragma unroll
        for (int q = 0; q < kPcaCols; ++q) part[g - 1][r][q] = sp[q];
    }
    __syncthreads();
    if (g == 0 && a < d) {
#pragma unroll
        for (int q = 0; q < kPcaCols; ++q)
            if (j0 + q < m)
                V[(int64_t)(j0 + q) * d + a] = (((sp[q] + part[0][r][q]) + part[1][r][q]) + part[2][r][q]) * rinv[j0 + q];
    }
}

// Cyclic Jacobi on the symmetric m x m matrix H (row-major; H and the
// rotations E held in LDS, copied back at the end), one workgroup: each sweep runs m - 1 rounds of the round-robin tournament
// (m even; an odd m plays a bye), every round rotating its m/2 disjoint
// pairs (p, q) so that H[p][q] becomes 0: rows then columns, with E
// accumulating the rotations (E starts as the identity).  Sweeps stop when
// the off-diagonal mass (sum of squares) falls below 1e-26 of the total
// (off-diagonal entries below 1e-13 of the norm), or after 40.
__global__ __launch_bounds__(256) void pca_jacobi_kernel(double* __restrict__ Hg, double* __restrict__ Eg, int m)
{
    __shared__ double H[kPcaMaxM * kPcaMaxM];
    __shared__ double E[kPcaMaxM * kPcaMaxM];
    __shared__ double cs[kPcaMaxM / 2], sn[kPcaMaxM / 2];
    __shared__ int pp[kPcaMaxM / 2], qq[kPcaMaxM / 2];
    __shared__ double red[256];
    const int tid = threadIdx.x;
    // V^T (C V) is symmetric up to rounding: take its symmetric part
    for (int e = tid; e < m * m; e += 256) H[e] = 0.5 * (Hg[e] + Hg[(e % m) * m + e / m]);
    const int mm = m + (m & 1);   // players, with a bye for odd m
    for (int e = tid; e < m * m; e += 256) E[e] = (e / m == e % m) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        __syncthreads();
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < m * m; e += 256) {
            const double h = H[e];
            tot += h * h;
            if (e / m != e % m) off += h * h;
        }
        red[tid] = off;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        off = red[0];
        __syncthreads();
        red[tid] = tot;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        tot = red[0];
        __syncthreads();
        if (!(off > 1e-26 * tot)) break;
        for (int round = 0; round < mm - 1; ++round) {
            // pairs of this round: player 0 fixed, the others rotate
            for (int t = tid; t < mm / 2; t += 256) {
                int a = t == 0 ? 0 : 1 + (round + t - 1) % (mm - 1);
                int b = 1 + (round + mm - 2 - t) % (mm - 1);
                if (a > b) {
                    const int x = a;
                    a = b;
                    b = x;
                }
                pp[t] = a;
                qq[t] = b;
                double c = 1.0, s = 0.0;
                if (b < m) {
                    const double apq = H[a * m + b];
                    if (apq != 0.0) {
                        const double theta = (H[b * m + b] - H[a * m + a]) / (2.0 * apq);
                        const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        s = tt * c;
                    }
                }
                cs[t] = c;
                sn[t] = s;
            }
            __syncthreads();
            // rows: H[p][*], H[q][*] <- c H[p] - s H[q], s H[p] + c H[q]
            // (pair t by threads with tid / 16 = t mod 16, entries by tid % 16)
            constexpr int NJ = kPcaMaxM / 16;
            for (int t = tid >> 4; t < mm / 2; t += 16) {
                const int p = pp[t], q = qq[t];
                if (q >= m) continue;
                const double c = cs[t], s = sn[t];
                double hp[NJ], hq[NJ];
#pragma unroll
                for (int u = 0; u < NJ; ++u) {
                    const int col = (tid & 15) + 16 * u;
                    hp[u] = col < m ? H[p * m + col] : 0.0;
                    hq[u] = col < m ? H[q * m + col] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < NJ; ++u) {
                    const int col = (tid & 15) + 16 * u;
                    if (col < m) {
                        H[p * m + col] = c * hp[u] - s * hq[u];
                        H[q * m + col] = s * hp[u] + c * hq[u];
                    }
                }
            }
            __syncthreads();
            // columns, and the accumulated rotations E <- E J
            for (int t = tid >> 4; t < mm / 2; t += 16) {
                const int p = pp[t], q = qq[t];
                if (q >= m) continue;
                const double c = cs[t], s = sn[t];
                double hp[NJ], hq[NJ], ep[NJ], eq[NJ];
#pragma unroll
                for (int u = 0; u < NJ; ++u) {
                    const int row = (tid & 15) + 16 * u;
                    const bool ok = row < m;
                    hp[u] = ok ? H[row * m + p] : 0.0;
                    hq[u] = ok ? H[row * m + q] : 0.0;
                    ep[u] = ok ? E[row * m + p] : 0.0;
                    eq[u] = ok ? E[row * m + q] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < NJ; ++u) {
                    const int row = (tid & 15) + 16 * u;
                    if (row < m) {
                        H[row * m + p] = c * hp[u] - s * hq[u];
                        H[row * m + q] = s * hp[u] + c * hq[u];
                        E[row * m + p] = c * ep[u] - s * eq[u];
                        E[row * m + q] = s * ep[u] + c * eq[u];
                    }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += 256) {
        Hg[e] = H[e];
        Eg[e] = E[e];
    }
}

// The p largest Ritz pairs: eigenvalues from diag(H) sorted descending
// (ties by index), vectors U_j = V e_j (e_j a column of E), each sign-fixed
// so that its entry of largest magnitude (the first such) is positive.
// Workgroup j forms component j; U is d x p row-major, lam has p entries.
__global__ __launch_bounds__(256) void pca_ritz_kernel(const double* __restrict__ H, const double* __restrict__ E,
                                                       const double* __restrict__ V, int d, int m, int p,
                                                       double* __restrict__ U, double* __restrict__ lam)
{
    __shared__ double ecol[kPcaMaxM];
    __shared__ double red[256];
    __shared__ int redi[256];
    __shared__ int col_;
    const int tid = threadIdx.x, j = blockIdx.x;
    if (tid < m) {
        const double x = H[tid * m + tid];
        int rank = 0;
        for (int q = 0; q < m; ++q) {
            const double y = H[q * m + q];
            rank += (y > x || (y == x && q < tid)) ? 1 : 0;
        }
        if (rank == j) col_ = tid;
    }
    __syncthreads();
    const int col = col_;
    if (tid < m) ecol[tid] = E[tid * m + col];
    __syncthreads();
    double best = -1.0;
    int bi = 0;
    for (int a = tid; a < d; a += 256) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s = fma(V[(int64_t)i * d + a], ecol[i], s);
        if (fabs(s) > best) {
            best = fabs(s);
            bi = a;
        }
        U[(int64_t)a * p + j] = s;
    }
    red[tid] = best;
    redi[tid] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o && (red[tid + o] > red[tid] || (red[tid + o] == red[tid] && redi[tid + o] < redi[tid]))) {
            red[tid] = red[tid + o];
            redi[tid] = redi[tid + o];
        }
        __syncthreads();
    }
    const double sg = U[(int64_t)redi[0] * p + j] < 0.0 ? -1.0 : 1.0;
    if (tid == 0) lam[j] = H[col * m + col];
    for (int a = tid; a < d; a += 256) U[(int64_t)a * p + j] *= sg;
}

// Z[r][j] = sum_t (x_rt - mu_t) U[t][j] on v_mfma_f64_16x16x4_f64, rounded
// to FP32: wave w of workgroup b takes rows 16 (4b + w) .. +15 and every
// 16-column block of U (p <= 64: up to four accumulators), so each row of X
// is read once.  K runs as in pca_cv_kernel (lane l holds coordinates
// k0 + 4 (l / 16) .. +3 of row l % 16, step s takes the k0 + 4g + s slice).
template <int DT>
__global__ __launch_bounds__(256) void pca_project_kernel(const void* __restrict__ X, int64_t n, int64_t ld, int d,
                                                          const double* __restrict__ mu, const double* __restrict__ U,
                                                          int p, float* __restrict__ Z)
{
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, r = l & 15, g = l >> 4;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
    if (row0 >= n) return;   // the whole wave
    const int64_t row = row0 + r;
    const bool rok = row < n;
    const int nt = (p + 15) / 16;
    f64x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    // two K blocks per round, the row's loads issued first
    for (int kb = 0; kb < d; kb += 32) {
        float xr[2][4];
        double mk[2][4];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = kb + 16 * b + 4 * g + s;
                xr[b][s] = rok && k < d ? elem<DT>::ld(X, row * ld + k) : 0.0f;
                mk[b][s] = k < d ? mu[k] : 0.0;
            }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < nt) {
                const int jj = 16 * t + r;
                double ub[2][4];
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int k = kb + 16 * b + 4 * g + s;
                        ub[b][s] = k < d && jj < p ? U[(int64_t)k * p + jj] : 0.0;
                    }
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const double xa = rok ? (double)xr[b][s] - mk[b][s] : 0.0;
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, ub[b][s], acc[t], 0, 0, 0);
                    }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t < nt) {
            const int jj = 16 * t + r;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t rr = row0 + g + 4 * i;
                if (rr < n && jj < p) Z[rr * p + jj] = (float)acc[t][i];
            }
        }
    }
}

template <typename F>
static void pca_by_dtype(int dt, F&& f)
{
    if (dt == KNN_F32) f(std::integral_constant<int, KNN_F32>());
    else if (dt == KNN_BF16) f(std::integral_constant<int, KNN_BF16>());
    else f(std::integral_constant<int, KNN_F16>());
}

}  // namespace knn

using namespace knn;

extern "C" knn_status knn_pca(knn_matrix X, int32_t p, int32_t iters, float* Z, double* components,
                              double* eigenvalues, double* mean, void* stream)
{
    try {
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if (!Z) return fail(KNN_EINVAL, "Z is null");
        if (X.n < 2) return fail(KNN_EINVAL, "X.n must be >= 2");
        if (p < 1 || p > X.d) return fail(KNN_EINVAL, "p must satisfy 1 <= p <= d");
        if (p > kPcaMaxP) return fail(KNN_ENOTSUP, "p above 64 is not supported");
        if (iters < 0) return fail(KNN_EINVAL, "iters must be >= 0");
        const int d = X.d;
        if (d > 16384) return fail(KNN_ENOTSUP, "d above 16384 is not supported by the PCA");
        int m = 2 * p > p + 16 ? 2 * p : p + 16;
        if (m > kPcaMaxM) m = kPcaMaxM;
        if (m > d) m = d;
        const int T = m == d ? 0 : (iters > 0 ? iters : 200);
        const int64_t n = X.n;
        const int nch = (int)ceil_div(n, kPcaChunk);
        const int nsum = (int)ceil_div(n, kPcaSumChunk);
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        double *part, *mu, *C, *V, *W, *U2, *piv, *S, *H, *E, *U, *lam;
        unsigned* bad;
        const int nt = (int)ceil_div(d, kPcaTile);
        int2* tiles;
        if ((r = ws.alloc(&part, (size_t)std::max<int64_t>((int64_t)nch * d * d, (int64_t)nsum * d))) != KNN_OK)
            return r;
        if ((r = ws.alloc(&mu, (size_t)d)) != KNN_OK) return r;
        if ((r = ws.alloc(&C, (size_t)d * d)) != KNN_OK) return r;
        if ((r = ws.alloc(&V, (size_t)d * m)) != KNN_OK) return r;
        if ((r = ws.alloc(&W, (size_t)d * m)) != KNN_OK) return r;
        if ((r = ws.alloc(&U2, (size_t)d * m)) != KNN_OK) return r;
        if ((r = ws.alloc(&piv, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&S, (size_t)m * m)) != KNN_OK) return r;
        if ((r = ws.alloc(&H, (size_t)m * m)) != KNN_OK) return r;
        if ((r = ws.alloc(&E, (size_t)m * m)) != KNN_OK) return r;
        if ((r = ws.alloc(&U, (size_t)d * p)) != KNN_OK) return r;
        if ((r = ws.alloc(&lam, (size_t)p)) != KNN_OK) return r;
        if ((r = ws.alloc(&bad, 1)) != KNN_OK) return r;
        if ((r = ws.alloc(&tiles, (size_t)nt * (nt + 1) / 2)) != KNN_OK) return r;
        // upper-triangle tile list
        std::vector<int2> tl;
        for (int a = 0; a < nt; ++a)
            for (int b = a; b < nt; ++b) tl.push_back(make_int2(a, b));
        KNN_HIP(hipMemcpyAsync(tiles, tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice, st));
        KNN_HIP(hipMemsetAsync(bad, 0, 4, st));
        pca_by_dtype(X.dtype, [&](auto dt) {
            pca_colsum_kernel<decltype(dt)::value><<<dim3((unsigned)ceil_div(d, 256), (unsigned)nsum), 256, 0, st>>>(
                X.data, n, X.ld, d, part);
        });
        pca_mean_kernel<<<(unsigned)ceil_div(d, 256), 256, 0, st>>>(part, nsum, d, n, mu);
        pca_by_dtype(X.dtype, [&](auto dt) {
            pca_gram_kernel<decltype(dt)::value><<<dim3((unsigned)tl.size(), (unsigned)nch), 256, 0, st>>>(
                X.data, n, X.ld, d, mu, tiles, part);
        });
        pca_gram_reduce_kernel<<<(unsigned)ceil_div((int64_t)d * d, 256), 256, 0, st>>>(part, nch, d, n, C);
        KNN_HIP(hipGetLastError());
        // subspace iteration (skipped when the subspace is all of R^d)
        if (m == d) {
            // V = I: the Rayleigh-Ritz matrix is C itself
            pca_identity_kernel<<<(unsigned)ceil_div((int64_t)d * m, 256), 256, 0, st>>>(d, m, V);
        } else {
            pca_init_kernel<<<(unsigned)ceil_div((int64_t)d * m, 256), 256, 0, st>>>(d, m, 0x5CA1AB1Eull, W);
        }
        const dim3 gcols((unsigned)ceil_div(d, 64), (unsigned)ceil_div(m, kPcaCols));
        const dim3 gcv((unsigned)ceil_div(d, 16), (unsigned)ceil_div(m, 16));
        // shift of the shifted passes: 11 (m d + m (m + 1)) u relative to
        // trace(S) >= |W|_2^2, the bound under which a shifted Cholesky-QR
        // is guaranteed to succeed in double precision (Fukaya, Kannan,
        // Nakatsukasa, Yamamoto and Yanagisawa, 2020)
        const double shift = 11.0 * ((double)m * d + (double)m * (m + 1)) * 1.1102230246251565e-16;
        auto cholqr = [&](const double* in, double* out, double sh) {
            pca_gram_small_kernel<<<dim3((unsigned)m, (unsigned)m), 256, 0, st>>>(in, in, d, m, S);
            pca_cholqr_kernel<<<gcols, 256, 0, st>>>(S, in, d, m, out, bad, piv, sh);
        };
        if (m < d) {
            // Subspace iteration needs orthonormalisation only often enough
            // to keep the basis well conditioned: W = C^q V for q products,
            // then one shifted Cholesky-QR pass (the span is that of
            // orthonormalising after every product).  q is chosen so that the
            // basis' condition number, estimated from the spread of the last
            // pass's pivots (kappa(C^q V) ~ sqrt(max D / min D), so kappa(C V)
            // ~ that to the power 1/q), stays below about 1e4 over the q
            // products (larger targets lost the weak directions of the pixel
            // set's block in a CPU emulation).  After the last product a
            // shifted pass and two plain ones (Cholesky-QR3) make the basis
            // orthonormal to rounding for Rayleigh-Ritz.
            std::vector<double> hp((size_t)m);
            cholqr(W, V, shift);
            int q = 1, since = kPcaMaxQ;   // products since q was last re-estimated
            for (int it = 0; it < T;) {
                const int qq = std::min(q, T - it);
                const double* src = V;
                for (int r = 0; r < qq; ++r) {
                    double* dst = (r & 1) ? U2 : W;
                    pca_cv_kernel<<<gcv, 256, 0, st>>>(C, src, d, m, dst);
                    src = dst;
                }
                it += qq;
                since += qq;
                cholqr(src, V, shift);
                // re-estimated about every kPcaMaxQ products (each estimate
                // waits for the pass's pivots)
                if (it < T && since >= kPcaMaxQ) {
                    since = 0;
                    KNN_HIP(hipMemcpyAsync(hp.data(), piv, (size_t)m * 8, hipMemcpyDeviceToHost, st));
                    KNN_HIP(hipStreamSynchronize(st));
                    double lo = hp[0], hi = hp[0];
                    for (int k = 1; k < m; ++k) {
                        lo = std::min(lo, hp[k]);
                        hi = std::max(hi, hp[k]);
                    }
                    // kappa(C V) estimate (the pass saw C^qq V), and the
                    // products that keep kappa^q <= 1e4
                    const double kap = lo > 0.0 ? std::pow(hi / lo, 0.5 / qq) : 1e300;
                    q = kap <= 1.0 + 1e-12 ? kPcaMaxQ : (int)std::floor(4.0 / std::log10(kap));
                    q = std::max(1, std::min(q, kPcaMaxQ));
                }
            }
            cholqr(V, W, shift);
            cholqr(W, V, 0.0);
            cholqr(V, W, 0.0);
            std::swap(V, W);
            KNN_HIP(hipGetLastError());
        }
        // Rayleigh-Ritz: H = V^T C V
        pca_cv_kernel<<<gcv, 256, 0, st>>>(C, V, d, m, W);
        pca_gram_small_kernel<<<dim3((unsigned)m, (unsigned)m), 256, 0, st>>>(W, V, d, m, H);
        pca_jacobi_kernel<<<1, 256, 0, st>>>(H, E, m);
        pca_ritz_kernel<<<(unsigned)p, 256, 0, st>>>(H, E, V, d, m, p, U, lam);
        pca_by_dtype(X.dtype, [&](auto dt) {
            pca_project_kernel<decltype(dt)::value><<<(unsigned)ceil_div(n, 64), 256, 0, st>>>(
                X.data, n, X.ld, d, mu, U, p, Z);
        });
        KNN_HIP(hipGetLastError());
        if (components) KNN_HIP(hipMemcpyAsync(components, U, (size_t)d * p * 8, hipMemcpyDeviceToDevice, st));
        if (eigenvalues) KNN_HIP(hipMemcpyAsync(eigenvalues, lam, (size_t)p * 8, hipMemcpyDeviceToDevice, st));
        if (mean) KNN_HIP(hipMemcpyAsync(mean, mu, (size_t)d * 8, hipMemcpyDeviceToDevice, st));
        unsigned hb = 0;
        KNN_HIP(hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipStreamSynchronize(st));
        if (hb) return fail(KNN_EINVAL, "X has rank below the subspace width (a zero pivot in Cholesky-QR)");
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}
