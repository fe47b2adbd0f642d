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
//               values) iterate V <- orth(C V), orthonormalised by
//               Cholesky-QR (twice: the second pass restores the
//               orthogonality the first loses to conditioning); then
//               Rayleigh-Ritz: H = V^T C V, whose eigenpairs come from cyclic
//               Jacobi rotations (one workgroup, round-robin pairing), and
//               the p largest Ritz pairs are kept; each eigenvector's entry
//               of largest magnitude is made positive;
//  4. project:  Z = (X - mu) V_p, rounded to FP32.
// When m = d the Ritz pairs are the exact eigenpairs of C.
#include <math.h>

#include <vector>

#include "knn_common.hpp"

namespace knn {

constexpr int kPcaMaxP = 64;      // components
constexpr int kPcaMaxM = 80;      // subspace width (an m x m double matrix fits in LDS)
constexpr int kPcaChunk = 4096;   // rows per Gram partial
constexpr int kPcaTile = 64;      // Gram tile edge

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ mean

// part[c][t] = sum of column t over rows [c * kPcaChunk, ...), in row order
// (thread t of a 256-wide column block walks the chunk's rows).
template <int DT>
__global__ __launch_bounds__(256) void pca_colsum_kernel(const void* __restrict__ X, int64_t n, int64_t ld, int d,
                                                         double* __restrict__ part)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (t >= d) return;
    const int64_t r0 = c * kPcaChunk, r1 = r0 + kPcaChunk < n ? r0 + kPcaChunk : n;
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
    f64x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int64_t rs = r0; rs < r1; rs += 64) {
        __syncthreads();
        // stage 64 rows x 64 columns of each slice (zeros past d and past the chunk)
        for (int e = tid; e < 64 * kPcaTile; e += 256) {
            const int rr = e / kPcaTile, cc = e % kPcaTile;
            const int64_t row = rs + rr;
            const bool ok = row < r1;
            sa[rr][cc] = ok && a0 + cc < d ? elem<DT>::ld(X, row * ld + a0 + cc) : 0.0f;
            sb[rr][cc] = ok && b0 + cc < d ? elem<DT>::ld(X, row * ld + b0 + cc) : 0.0f;
        }
        __syncthreads();
        const int nr = (int)(r1 - rs < 64 ? r1 - rs : 64);
        for (int k0 = 0; k0 < nr; k0 += 4) {
            const int kk = k0 + (lane >> 4);
            const bool kv = kk < nr;
            const int ia = 16 * w + (lane & 15);
            // centred operands; padded rows and columns contribute 0
            const double av = kv && a0 + ia < d ? (double)sa[kk][ia] - sma[ia] : 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int jb = 16 * j + (lane & 15);
                const double bv = kv && b0 + jb < d ? (double)sb[kk][jb] - smb[jb] : 0.0;
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

// W[j][a] = sum_b C[b][a] V[j][b] (C symmetric: lanes over a read rows of C,
// coalesced), eight columns j per thread so that each C element loaded
// serves eight products.
constexpr int kPcaCols = 8;

__global__ __launch_bounds__(256) void pca_cv_kernel(const double* __restrict__ C, const double* __restrict__ V,
                                                     int d, int m, double* __restrict__ W)
{
    const int a = blockIdx.x * 256 + threadIdx.x;
    const int j0 = blockIdx.y * kPcaCols;
    if (a >= d) return;
    double s[kPcaCols];
#pragma unroll
    for (int q = 0; q < kPcaCols; ++q) s[q] = 0.0;
    for (int b = 0; b < d; ++b) {
        const double c = C[(int64_t)b * d + a];
#pragma unroll
        for (int q = 0; q < kPcaCols; ++q)
            if (j0 + q < m) s[q] = fma(c, V[(int64_t)(j0 + q) * d + b], s[q]);
    }
#pragma unroll
    for (int q = 0; q < kPcaCols; ++q)
        if (j0 + q < m) W[(int64_t)(j0 + q) * d + a] = s[q];
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

// Cholesky factor S = R^T R (R upper triangular) of the m x m Gram matrix
// in LDS, one workgroup, column by column, then its inverse Ri = R^{-1}
// (upper triangular, one column per thread by back substitution); Ri goes
// to global memory.  A non-positive pivot (a rank-deficient W) is replaced
// by 1 and flagged, which keeps the factor finite.
__global__ __launch_bounds__(256) void pca_chol_inv_kernel(const double* __restrict__ Sg, int m,
                                                           double* __restrict__ Ri, unsigned* __restrict__ bad)
{
    __shared__ double S[kPcaMaxM * kPcaMaxM];
    const int tid = threadIdx.x;
    for (int e = tid; e < m * m; e += 256) S[e] = Sg[e];
    for (int k = 0; k < m; ++k) {
        __syncthreads();
        double piv = S[k * m + k];
        if (!(piv > 0.0)) {
            if (tid == 0) atomicOr(bad, 1u);
            piv = 1.0;
        }
        const double r = sqrt(piv);
        __syncthreads();
        for (int j = k + 1 + tid; j < m; j += 256) S[k * m + j] /= r;
        if (tid == 0) S[k * m + k] = r;
        __syncthreads();
        const int w = m - k - 1;
        for (int e = tid; e < w * w; e += 256) {
            const int i = k + 1 + e / w, j = k + 1 + e % w;
            if (i <= j) S[i * m + j] -= S[k * m + i] * S[k * m + j];
        }
    }
    __syncthreads();
    // column j of R^{-1}: R x = e_j, rows j, j-1, ..., 0
    for (int j = tid; j < m; j += 256) {
        for (int i = m - 1; i > j; --i) Ri[i * m + j] = 0.0;
        Ri[j * m + j] = 1.0 / S[j * m + j];
        for (int i = j - 1; i >= 0; --i) {
            double t = 0.0;
            for (int l = i + 1; l <= j; ++l) t = fma(S[i * m + l], Ri[l * m + j], t);
            Ri[i * m + j] = -t / S[i * m + i];
        }
    }
}

// V[j][a] = sum_{i <= j} W[i][a] Ri[i][j] (= W R^{-1}, eight columns per
// thread).
__global__ __launch_bounds__(256) void pca_apply_kernel(const double* __restrict__ W, const double* __restrict__ Ri,
                                                        int d, int m, double* __restrict__ V)
{
    const int a = blockIdx.x * 256 + threadIdx.x;
    const int j0 = blockIdx.y * kPcaCols;
    if (a >= d) return;
    double s[kPcaCols];
#pragma unroll
    for (int q = 0; q < kPcaCols; ++q) s[q] = 0.0;
    const int jmax = j0 + kPcaCols < m ? j0 + kPcaCols : m;
    for (int i = 0; i < jmax; ++i) {
        const double w = W[(int64_t)i * d + a];
#pragma unroll
        for (int q = 0; q < kPcaCols; ++q)
            if (j0 + q < m && i <= j0 + q) s[q] = fma(w, Ri[i * m + j0 + q], s[q]);
    }
#pragma unroll
    for (int q = 0; q < kPcaCols; ++q)
        if (j0 + q < m) V[(int64_t)(j0 + q) * d + a] = s[q];
}

// Cyclic Jacobi on the symmetric m x m matrix H (row-major, copied into LDS
// and back), one workgroup: each sweep runs m - 1 rounds of the round-robin tournament
// (m even; an odd m plays a bye), every round rotating its m/2 disjoint
// pairs (p, q) so that H[p][q] becomes 0: rows then columns, with E
// accumulating the rotations (E starts as the identity).  Sweeps stop when
// the off-diagonal mass falls below 1e-30 of the total, or after 40.
__global__ __launch_bounds__(256) void pca_jacobi_kernel(double* __restrict__ Hg, double* __restrict__ E, int m)
{
    __shared__ double H[kPcaMaxM * kPcaMaxM];
    __shared__ double cs[kPcaMaxM / 2], sn[kPcaMaxM / 2];
    __shared__ int pp[kPcaMaxM / 2], qq[kPcaMaxM / 2];
    __shared__ double red[256];
    const int tid = threadIdx.x;
    for (int e = tid; e < m * m; e += 256) H[e] = Hg[e];
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
        if (!(off > 1e-30 * tot)) break;
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
            for (int e = tid; e < (mm / 2) * m; e += 256) {
                const int t = e / m, col = e % m, p = pp[t], q = qq[t];
                if (q >= m) continue;
                const double hp = H[p * m + col], hq = H[q * m + col];
                H[p * m + col] = cs[t] * hp - sn[t] * hq;
                H[q * m + col] = sn[t] * hp + cs[t] * hq;
            }
            __syncthreads();
            // columns, and the accumulated rotations E <- E J
            for (int e = tid; e < (mm / 2) * m; e += 256) {
                const int t = e / m, row = e % m, p = pp[t], q = qq[t];
                if (q >= m) continue;
                const double hp = H[row * m + p], hq = H[row * m + q];
                H[row * m + p] = cs[t] * hp - sn[t] * hq;
                H[row * m + q] = sn[t] * hp + cs[t] * hq;
                const double ep = E[row * m + p], eq = E[row * m + q];
                E[row * m + p] = cs[t] * ep - sn[t] * eq;
                E[row * m + q] = sn[t] * ep + cs[t] * eq;
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += 256) Hg[e] = H[e];
}

// The p largest Ritz pairs: eigenvalues from diag(H) sorted descending
// (ties by index), vectors U_j = V e_j (e_j a column of E), each sign-fixed
// so its entry of largest magnitude (the first such) is positive.  One
// workgroup; U (d x p row-major) and lam (p).
__global__ __launch_bounds__(256) void pca_ritz_kernel(const double* __restrict__ H, const double* __restrict__ E,
                                                       const double* __restrict__ V, int d, int m, int p,
                                                       double* __restrict__ U, double* __restrict__ lam)
{
    __shared__ int order[kPcaMaxM];
    __shared__ double sgn[kPcaMaxP];
    __shared__ double red[256];
    __shared__ int redi[256];
    const int tid = threadIdx.x;
    if (tid < m) {
        const double x = H[tid * m + tid];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double y = H[j * m + j];
            rank += (y > x || (y == x && j < tid)) ? 1 : 0;
        }
        order[rank] = tid;
    }
    __syncthreads();
    for (int j = 0; j < p; ++j) {
        const int col = order[j];
        // entry of largest magnitude of V E[:, col]
        double best = -1.0;
        int bi = 0;
        for (int a = tid; a < d; a += 256) {
            double s = 0.0;
            for (int i = 0; i < m; ++i) s = fma(V[(int64_t)i * d + a], E[i * m + col], s);
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
        if (tid == 0) {
            sgn[j] = U[(int64_t)redi[0] * p + j] < 0.0 ? -1.0 : 1.0;
            lam[j] = H[col * m + col];
        }
        __syncthreads();
    }
    for (int e = tid; e < d * p; e += 256) U[e] *= sgn[e % p];
}

// Z[r][j] = sum_t (x_rt - mu_t) U[t][j], in double, rounded to FP32.  One
// thread per (row, component); U and mu are read through the cache.
template <int DT>
__global__ __launch_bounds__(256) void pca_project_kernel(const void* __restrict__ X, int64_t n, int64_t ld, int d,
                                                          const double* __restrict__ mu, const double* __restrict__ U,
                                                          int p, float* __restrict__ Z)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * p) return;
    const int64_t r = e / p;
    const int j = (int)(e % p);
    double s = 0.0;
    for (int t = 0; t < d; ++t) s = fma((double)elem<DT>::ld(X, r * ld + t) - mu[t], U[(int64_t)t * p + j], s);
    Z[e] = (float)s;
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
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        double *part, *mu, *C, *V, *W, *S, *H, *E, *U, *lam;
        unsigned* bad;
        const int nt = (int)ceil_div(d, kPcaTile);
        int2* tiles;
        if ((r = ws.alloc(&part, (size_t)nch * std::max<int64_t>((int64_t)d * d, d))) != KNN_OK) return r;
        if ((r = ws.alloc(&mu, (size_t)d)) != KNN_OK) return r;
        if ((r = ws.alloc(&C, (size_t)d * d)) != KNN_OK) return r;
        if ((r = ws.alloc(&V, (size_t)d * m)) != KNN_OK) return r;
        if ((r = ws.alloc(&W, (size_t)d * m)) != KNN_OK) return r;
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
            pca_colsum_kernel<decltype(dt)::value><<<dim3((unsigned)ceil_div(d, 256), (unsigned)nch), 256, 0, st>>>(
                X.data, n, X.ld, d, part);
        });
        pca_mean_kernel<<<(unsigned)ceil_div(d, 256), 256, 0, st>>>(part, nch, d, n, mu);
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
        const dim3 gcols((unsigned)ceil_div(d, 256), (unsigned)ceil_div(m, kPcaCols));
        auto orthonormalise = [&](double* src, double* dst) -> knn_status {
            // two Cholesky-QR passes: src -> dst -> (src as scratch) -> dst
            double* in = src;
            for (int pass = 0; pass < 2; ++pass) {
                pca_gram_small_kernel<<<dim3((unsigned)m, (unsigned)m), 256, 0, st>>>(in, in, d, m, S);
                pca_chol_inv_kernel<<<1, 256, 0, st>>>(S, m, E, bad);
                double* out = pass == 0 ? dst : src;
                pca_apply_kernel<<<gcols, 256, 0, st>>>(in, E, d, m, out);
                in = out;
            }
            if (in != dst) KNN_HIP(hipMemcpyAsync(dst, in, (size_t)d * m * 8, hipMemcpyDeviceToDevice, st));
            KNN_HIP(hipGetLastError());
            return KNN_OK;
        };
        if (m < d) {
            if ((r = orthonormalise(W, V)) != KNN_OK) return r;
            for (int it = 0; it < T; ++it) {
                pca_cv_kernel<<<gcols, 256, 0, st>>>(C, V, d, m, W);
                if ((r = orthonormalise(W, V)) != KNN_OK) return r;
            }
        }
        // Rayleigh-Ritz: H = V^T C V
        pca_cv_kernel<<<dim3((unsigned)ceil_div(d, 256), (unsigned)ceil_div(m, kPcaCols)), 256, 0, st>>>(C, V, d, m,
                                                                                                      W);
        pca_gram_small_kernel<<<dim3((unsigned)m, (unsigned)m), 256, 0, st>>>(W, V, d, m, H);
        pca_jacobi_kernel<<<1, 256, 0, st>>>(H, E, m);
        pca_ritz_kernel<<<1, 256, 0, st>>>(H, E, V, d, m, p, U, lam);
        pca_by_dtype(X.dtype, [&](auto dt) {
            pca_project_kernel<decltype(dt)::value><<<(unsigned)ceil_div(n * p, 256), 256, 0, st>>>(
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
