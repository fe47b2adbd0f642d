// UMAP membership strengths of a k-NN graph and their fuzzy union
// (McInnes, Healy & Melville 2018): the graph the UMAP-family methods of the
// paper build from the shared k-NN stage (sections "Architecture" and
// "Method Implementations").
//
// For row i with neighbour distances d_1..d_k:
//   rho_i   = the smallest positive d_r (0 if there is none);
//   sigma_i solves sum_r exp(-max(0, d_r - rho_i) / sigma_i) = log2(k); the
//           sum falls from k (sigma -> inf) to c_i = #{r : d_r <= rho_i}
//           (sigma -> 0), so there is a root iff c_i < log2(k), else
//           sigma_i = 0 and the weights take the limit (1 where d_r <= rho_i,
//           0 elsewhere);
//   w_ir    = exp(-max(0, d_r - rho_i) / sigma_i);
// and the symmetric graph W = A + A^T - A o A^T with A[i][idx_ir] = w_ir.
//
// 1. rows:   one thread per row.  sigma is bracketed and bisected in FP32
//            (v_exp_f32), then polished by Newton steps on the sum in
//            double, whose root it converges to quadratically from the FP32
//            estimate; the weights are evaluated in double and rounded once.
//            Each edge (i -> j) emits two entries: (row i, col j) and
//            (row j, col i), both carrying w_ij, identified by their entry
//            number 2e and 2e + 1.
// 2. sort:   the entries are sorted by (row, col) with two stable LSD radix
//            sorts (by column, then by row) on 32-bit keys with the entry
//            number as payload; deterministic whatever the thread order.
// 3. emit:   runs of equal (row, col) fold their values by the probabilistic
//            union v <- v + x - v x (two entries: a + b - ab) in double; a
//            scan over the run heads gives each unique entry its CSR slot,
//            and the row boundaries give row_ptr.
#include <math.h>

#include "knn_common.hpp"

namespace knn {

knn_status radix_sort_bits(uint32_t*& k0, uint32_t*& v0, uint32_t*& k1, uint32_t*& v1, int64_t n,
                           uint32_t* counts, hipStream_t st, int bits, int S);
size_t radix_counts_words(int64_t n);

constexpr int kFzMaxK = KNN_MAX_K;

// ------------------------------------------------------------------ rows

// FP32 sum of exp(-x_r / s) (s > 0), as exp2 of -x_r * (log2(e) / s).
__device__ inline float fz_sum32(const float (&x)[kFzMaxK], int k, float s)
{
    const float c = 1.4426950408889634f / s;
    float t = 0.0f;
#pragma unroll
    for (int r = 0; r < kFzMaxK; ++r)
        if (r < k) t += exp2f(-x[r] * c);
    return t;
}

__global__ __launch_bounds__(256) void fuzzy_rows_kernel(
    const int32_t* __restrict__ idx, const float* __restrict__ dist, int64_t n, int k,
    float* __restrict__ rho_out, float* __restrict__ sigma_out, float* __restrict__ w_out,
    uint32_t* __restrict__ colkey, uint32_t* __restrict__ rowkey, uint32_t* __restrict__ eid,
    unsigned* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float d[kFzMaxK];
    double p = 0.0;
#pragma unroll
    for (int r = 0; r < kFzMaxK; ++r) {
        d[r] = r < k ? dist[i * k + r] : 0.0f;
        if (r < k && d[r] > 0.0f && (p == 0.0 || (double)d[r] < p)) p = (double)d[r];
    }
    // x_r = max(0, d_r - rho) in double (exact for FP32 inputs), kept as
    // FP32 for the bracket search
    float x[kFzMaxK];
    int cnt = 0;
    float xmax = 0.0f;
#pragma unroll
    for (int r = 0; r < kFzMaxK; ++r) {
        const double xd = (double)d[r] - p;
        x[r] = xd > 0.0 ? (float)xd : 0.0f;
        if (r < k && !(xd > 0.0)) ++cnt;
        if (r < k) xmax = fmaxf(xmax, x[r]);
    }
    const double target = log2((double)k);
    double sig = 0.0;
    if ((double)cnt < target) {
        const float t32 = (float)target;
        float lo = 0.0f, hi = xmax;
        while (fz_sum32(x, k, hi) < t32) hi *= 2.0f;
        for (int it = 0; it < 40; ++it) {
            const float mid = 0.5f * (lo + hi);
            if (!(mid > lo && mid < hi)) break;
            if (fz_sum32(x, k, mid) < t32) lo = mid;
            else hi = mid;
        }
        // Newton on f(s) = sum exp(-x_r / s) - log2(k), f'(s) = sum
        // exp(-x_r / s) x_r / s^2, in double from the FP32 bracket
        double s = 0.5 * ((double)lo + (double)hi);
        for (int it = 0; it < 4; ++it) {
            double f = -target, g = 0.0;
#pragma unroll
            for (int r = 0; r < kFzMaxK; ++r) {
                if (r < k) {
                    const double xr = fmax((double)d[r] - p, 0.0);
                    const double e = exp(-xr / s);
                    f += e;
                    g += e * xr;
                }
            }
            g /= s * s;
            if (!(g > 0.0)) break;
            const double ns = s - f / g;
            if (!(ns > 0.0) || !isfinite(ns)) break;
            s = ns;
        }
        sig = s;
    }
    if (rho_out) rho_out[i] = (float)p;
    if (sigma_out) sigma_out[i] = (float)sig;
    bool ok = true;
#pragma unroll
    for (int r = 0; r < kFzMaxK; ++r) {
        if (r < k) {
            const double xr = fmax((double)d[r] - p, 0.0);
            const float w = sig > 0.0 ? (float)exp(-xr / sig) : (xr == 0.0 ? 1.0f : 0.0f);
            const int64_t e = i * k + r;
            w_out[e] = w;
            const int32_t j = idx[e];
            const bool valid = j >= 0 && (int64_t)j < n && (int64_t)j != i;
            ok = ok && valid;
            // entry 2e: (i, j); entry 2e + 1: (j, i); invalid edges sort last (row n)
            colkey[2 * e] = valid ? (uint32_t)j : 0u;
            rowkey[2 * e] = valid ? (uint32_t)i : (uint32_t)n;
            colkey[2 * e + 1] = valid ? (uint32_t)i : 0u;
            rowkey[2 * e + 1] = valid ? (uint32_t)j : (uint32_t)n;
            eid[2 * e] = (uint32_t)(2 * e);
            eid[2 * e + 1] = (uint32_t)(2 * e + 1);
        }
    }
    if (!ok) atomicOr(bad, 1u);
}

// keys of the second sort: the row of each entry in column order
__global__ __launch_bounds__(256) void fuzzy_gather_kernel(const uint32_t* __restrict__ ids,
                                                          const uint32_t* __restrict__ rowkey, int64_t m,
                                                          uint32_t* __restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) out[p] = rowkey[ids[p]];
}

// ------------------------------------------------------------------ emit

constexpr int kFzThreads = 256, kFzItems = 8, kFzTile = kFzThreads * kFzItems;

// (row, col) of sorted entry p; entries of invalid edges have row n
__device__ inline void fz_entry(const uint32_t* ids, const int32_t* idx, int k, int64_t n, int64_t p,
                                uint32_t& row, uint32_t& col)
{
    const uint32_t id = ids[p];
    const int64_t e = id >> 1;
    const int64_t i = e / k;
    const int32_t j = idx[e];
    const bool valid = j >= 0 && (int64_t)j < n && (int64_t)j != i;
    if (!valid) {
        row = (uint32_t)n;
        col = 0;
    } else if (id & 1u) {
        row = (uint32_t)j;
        col = (uint32_t)i;
    } else {
        row = (uint32_t)i;
        col = (uint32_t)j;
    }
}

__device__ inline bool fz_head(const uint32_t* ids, const int32_t* idx, int k, int64_t n, int64_t p,
                               uint32_t& row, uint32_t& col)
{
    fz_entry(ids, idx, k, n, p, row, col);
    if ((int64_t)row >= n) return false;
    if (p == 0) return true;
    uint32_t r0, c0;
    fz_entry(ids, idx, k, n, p - 1, r0, c0);
    return r0 != row || c0 != col;
}

// Heads per tile of kFzTile sorted entries.
__global__ __launch_bounds__(kFzThreads) void fuzzy_count_kernel(const uint32_t* __restrict__ ids,
                                                                 const int32_t* __restrict__ idx, int k,
                                                                 int64_t n, int64_t m,
                                                                 uint32_t* __restrict__ tile_cnt)
{
    __shared__ uint32_t s[kFzThreads / 64];
    uint32_t c = 0;
    for (int it = 0; it < kFzItems; ++it) {
        const int64_t p = (int64_t)blockIdx.x * kFzTile + it * kFzThreads + threadIdx.x;
        uint32_t r, cl;
        if (p < m && fz_head(ids, idx, k, n, p, r, cl)) ++c;
    }
    for (int o = 32; o > 0; o >>= 1) c += shfl_u32(c, (threadIdx.x & 63) ^ o);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// Exclusive scan of the tile counts by one block (in order, with a carry);
// tile_cnt[ntile] receives the total.
__global__ __launch_bounds__(256) void fuzzy_scan_kernel(uint32_t* __restrict__ tile_cnt, int64_t ntile)
{
    __shared__ uint32_t s[256];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < ntile; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t x = b < ntile ? tile_cnt[b] : 0u;
        __syncthreads();
        s[threadIdx.x] = x;
        __syncthreads();
        for (int w = 1; w < 256; w <<= 1) {
            const uint32_t y = (int)threadIdx.x >= w ? s[threadIdx.x - w] : 0u;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (b < ntile) tile_cnt[b] = carry + s[threadIdx.x] - x;
        carry += s[255];
    }
    if (threadIdx.x == 0) tile_cnt[ntile] = carry;
}

// Each head folds its run into one CSR entry at (tile offset + heads before
// it in the tile) and fills row_ptr for the rows from the previous entry's
// row (exclusive) up to its own; the last valid entry fills the rest.
__global__ __launch_bounds__(kFzThreads) void fuzzy_emit_kernel(
    const uint32_t* __restrict__ ids, const int32_t* __restrict__ idx, const float* __restrict__ w, int k,
    int64_t n, int64_t m, const uint32_t* __restrict__ tile_off, int64_t* __restrict__ row_ptr,
    int32_t* __restrict__ col_out, float* __restrict__ val_out)
{
    __shared__ uint32_t s[kFzThreads];
    uint32_t run = tile_off[blockIdx.x];
    const int64_t nnz = tile_off[gridDim.x];
    for (int it = 0; it < kFzItems; ++it) {
        const int64_t p = (int64_t)blockIdx.x * kFzTile + it * kFzThreads + threadIdx.x;
        uint32_t row = 0, col = 0;
        const bool head = p < m && fz_head(ids, idx, k, n, p, row, col);
        __syncthreads();
        s[threadIdx.x] = head ? 1u : 0u;
        __syncthreads();
        for (int o = 1; o < kFzThreads; o <<= 1) {
            const uint32_t y = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        const uint32_t incl = s[threadIdx.x], total = s[kFzThreads - 1];
        if (head) {
            const int64_t o = (int64_t)run + incl - 1;
            double v = 0.0;
            int64_t q = p;
            for (;;) {
                const double x = (double)w[ids[q] >> 1];
                v = v + x - v * x;
                ++q;
                if (q >= m) break;
                uint32_t r2, c2;
                fz_entry(ids, idx, k, n, q, r2, c2);
                if (r2 != row || c2 != col) break;
            }
            col_out[o] = (int32_t)col;
            val_out[o] = (float)v;
            // rows after the previous entry's row, up to this one, start here
            int64_t prev = -1;
            if (p > 0) {
                uint32_t r0, c0;
                fz_entry(ids, idx, k, n, p - 1, r0, c0);
                prev = (int64_t)r0;
            }
            for (int64_t rr = prev + 1; rr <= (int64_t)row; ++rr) row_ptr[rr] = o;
            // the last valid entry closes the remaining rows
            bool last = q >= m;
            if (!last) {
                uint32_t r2, c2;
                fz_entry(ids, idx, k, n, q, r2, c2);
                last = (int64_t)r2 >= n;
            }
            if (last)
                for (int64_t rr = (int64_t)row + 1; rr <= n; ++rr) row_ptr[rr] = nnz;
        }
        run += total;
    }
}

__global__ __launch_bounds__(256) void fill_i64_kernel(int64_t* __restrict__ p, int64_t m, int64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int bits_for(int64_t v)   // bits to hold values 0..v
{
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) <= v) ++b;
    return b;
}

}  // namespace knn

using namespace knn;

extern "C" knn_status knn_fuzzy_graph(const int32_t* knn_idx, const float* knn_dist, int64_t n, int32_t k,
                                      float* rho, float* sigma, float* weights, int64_t* row_ptr,
                                      int32_t* col, float* val, int64_t* nnz, void* stream)
{
    try {
        if (!knn_idx || !knn_dist || !row_ptr || !col || !val || !nnz) return fail(KNN_EINVAL, "null argument");
        if (n < 2 || n >= (int64_t)0x7FFFFFFF) return fail(KNN_EINVAL, "n must satisfy 2 <= n < 2^31 - 1");
        if (k < 1 || (int64_t)k > n - 1) return fail(KNN_EINVAL, "k must satisfy 1 <= k <= n-1");
        if (k > kFzMaxK) return fail(KNN_ENOTSUP, "k above 32 is not supported by the fuzzy graph");
        const int64_t m = 2 * n * (int64_t)k;
        if (m >= ((int64_t)1 << 32)) return fail(KNN_ENOTSUP, "2 n k must be below 2^32");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        knn_status r;
        uint32_t *ck, *rk, *id, *k1, *v1, *counts, *tiles;
        unsigned* bad;
        float* w = weights;
        const int64_t ntile = ceil_div(m, kFzTile);
        if ((r = ws.alloc(&ck, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&rk, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&id, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&k1, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&v1, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&counts, radix_counts_words(m))) != KNN_OK) return r;
        if ((r = ws.alloc(&tiles, (size_t)ntile + 1)) != KNN_OK) return r;
        if ((r = ws.alloc(&bad, 1)) != KNN_OK) return r;
        if (!w && (r = ws.alloc(&w, (size_t)n * k)) != KNN_OK) return r;
        KNN_HIP(hipMemsetAsync(bad, 0, 4, st));
        fuzzy_rows_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(knn_idx, knn_dist, n, k, rho, sigma, w, ck,
                                                                     rk, id, bad);
        KNN_HIP(hipGetLastError());
        // by column (keys < n), then stably by row (keys <= n: invalid edges last)
        uint32_t *a0 = ck, *b0 = id, *a1 = k1, *b1 = v1;
        if ((r = radix_sort_bits(a0, b0, a1, b1, m, counts, st, bits_for(n - 1), 1)) != KNN_OK) return r;
        // a1 is free scratch now: the row keys in column order
        fuzzy_gather_kernel<<<(unsigned)ceil_div(m, 256), 256, 0, st>>>(b0, rk, m, a1);
        uint32_t *c0 = a1, *d0 = b0, *c1 = a0, *d1 = b1;
        if ((r = radix_sort_bits(c0, d0, c1, d1, m, counts, st, bits_for(n), 1)) != KNN_OK) return r;
        fuzzy_count_kernel<<<(unsigned)ntile, kFzThreads, 0, st>>>(d0, knn_idx, k, n, m, tiles);
        fuzzy_scan_kernel<<<1, 256, 0, st>>>(tiles, ntile);
        fill_i64_kernel<<<(unsigned)std::min<int64_t>(ceil_div(n + 1, 256), 1024), 256, 0, st>>>(row_ptr, n + 1, 0);
        fuzzy_emit_kernel<<<(unsigned)ntile, kFzThreads, 0, st>>>(d0, knn_idx, w, k, n, m, tiles, row_ptr, col, val);
        KNN_HIP(hipGetLastError());
        unsigned host[2] = {0, 0};
        KNN_HIP(hipMemcpyAsync(&host[0], bad, 4, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipMemcpyAsync(&host[1], tiles + ntile, 4, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipStreamSynchronize(st));
        if (host[0]) return fail(KNN_EINVAL, "knn_idx holds an entry out of range or equal to its row");
        *nnz = (int64_t)host[1];
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}
