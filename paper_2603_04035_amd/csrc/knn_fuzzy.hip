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
//            Each edge e = (i -> j) emits one entry keyed by its target j.
// 2. sort:   the entries are sorted by target with a stable LSD radix sort
//            (32-bit keys, the edge number as payload), so the edges into a
//            row form one segment ordered by source: the row's transposed
//            entries, already in column order.  Deterministic whatever the
//            thread order.
// 3. union:  one wave per row merges its own k entries (ranked by column in
//            registers) with that segment: a column in both gets the
//            probabilistic union a + b - ab (folded in double in the order
//            of the entries' numbers, 2e for (i, j) and 2e' + 1 for the
//            transposed (j, i) of e' = (j -> i)), the others keep their
//            weight; each entry's CSR position follows from the counts of
//            smaller columns on both sides.  A count pass and a scan over
//            the rows give row_ptr, then the same pass writes the entries.
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
    uint32_t* __restrict__ tgtkey, uint32_t* __restrict__ eid, unsigned* __restrict__ bad)
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
            // keyed by target; invalid edges sort last (key n)
            tgtkey[e] = valid ? (uint32_t)j : (uint32_t)n;
            eid[e] = (uint32_t)e;
        }
    }
    if (!ok) atomicOr(bad, 1u);
}

// ------------------------------------------------------------------ union

// in_ptr[r] = the first sorted position whose target is >= r, r = 0..n.
__global__ __launch_bounds__(256) void fuzzy_inptr_kernel(const uint32_t* __restrict__ key, int64_t m, int64_t n,
                                                          uint32_t* __restrict__ in_ptr)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < m; p += (int64_t)gridDim.x * 256) {
        const int64_t r = key[p], prev = p > 0 ? (int64_t)key[p - 1] : -1;
        for (int64_t rr = prev + 1; rr <= r; ++rr) in_ptr[rr] = (uint32_t)p;
        if (p == m - 1)
            for (int64_t rr = r + 1; rr <= n; ++rr) in_ptr[rr] = (uint32_t)m;
    }
}

__device__ inline uint32_t lane_u32(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ inline float lane_f32(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }

// One wave per row i.  Lanes r < k hold the row's own entries (i, idx_ir);
// the transposed entries (i, j) of the edges j -> i are the segment
// [in_ptr[i], in_ptr[i + 1]) of the sorted edges, in column order.  The
// count pass (EMIT false) stores the union's size in cnt[i], flags a
// column repeated in a row's list and keeps each own entry's partner and
// count of smaller transposed columns; the emit pass writes the union at
// row_ptr[i], columns ascending.
template <bool EMIT>
__global__ __launch_bounds__(256) void fuzzy_union_kernel(
    const int32_t* __restrict__ idx, const float* __restrict__ w, int k, int64_t n,
    const uint32_t* __restrict__ sorted_e, const uint32_t* __restrict__ in_ptr, uint32_t* __restrict__ cnt,
    uint32_t* __restrict__ own_less, float* __restrict__ own_wm, const int64_t* __restrict__ row_ptr,
    int32_t* __restrict__ col_out, float* __restrict__ val_out, unsigned* __restrict__ bad)
{
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
        // own entries; an invalid one (reported by the rows kernel) takes no part
        const int32_t jj = lane < k ? idx[i * k + lane] : -1;
        const bool ov = jj >= 0 && (int64_t)jj < n && (int64_t)jj != i;
        const uint32_t oc = ov ? (uint32_t)jj : 0xFFFFFFFFu;
        const float ow = ov ? w[i * k + lane] : 0.0f;
        uint32_t orank = 0;   // own entries with a smaller column
        bool rep = false;     // an earlier lane holds the same column
        for (int r = 0; r < k; ++r) {
            const uint32_t c2 = lane_u32(oc, r);
            orank += c2 < oc ? 1u : 0u;
            rep = rep || (ov && r < lane && c2 == oc);
        }
        if (!EMIT && ballot(rep) && lane == 0) atomicOr(bad, 2u);
        const int64_t b = in_ptr[i], e = in_ptr[i + 1];
        // per own entry: its transposed partner (matched, with weight wm) and
        // the transposed entries with a smaller column; found by the count
        // pass, which keeps them per edge (oless | matched << 31, wm) for the
        // emit pass
        bool om = false;
        float wm = 0.0f;
        uint32_t oless = 0;
        if (EMIT) {
            const uint32_t ol = lane < k ? own_less[i * k + lane] : 0u;
            om = ov && (ol >> 31) != 0u;
            oless = ol & 0x7FFFFFFFu;
            wm = lane < k ? own_wm[i * k + lane] : 0.0f;
        }
        for (int64_t c0 = b; c0 < (EMIT ? b : e); c0 += 64) {
            const int64_t p = c0 + lane;
            const bool iv = p < e;
            const uint32_t ed = iv ? sorted_e[p] : 0u;
            const uint32_t ic = iv ? ed / (uint32_t)k : 0xFFFFFFFFu;
            const float iw = iv ? w[ed] : 0.0f;
            for (int r = 0; r < k; ++r) {
                const uint32_t ocr = lane_u32(oc, r);
                const uint64_t mb = ballot(iv && ic == ocr);
                const uint64_t lt = ballot(iv && ic < ocr);
                const float ws = lane_f32(iw, mb ? __builtin_ctzll(mb) : 0);
                if (lane == r) {
                    oless += (uint32_t)popc64(lt);
                    if (mb) {
                        om = true;
                        wm = ws;
                    }
                }
            }
        }
        const uint32_t nown = (uint32_t)popc64(ballot(ov)), nmatch = (uint32_t)popc64(ballot(om));
        if (!EMIT) {
            if (lane == 0) cnt[i] = nown + (uint32_t)(e - b) - nmatch;
            if (lane < k) {
                own_less[i * k + lane] = oless | (om ? 0x80000000u : 0u);
                own_wm[i * k + lane] = wm;
            }
            continue;
        }
        const int64_t base = row_ptr[i];
        uint32_t mless = 0;   // matched own entries with a smaller column
        for (int r = 0; r < k; ++r) {
            const uint32_t c2 = lane_u32(oc, r), m2 = lane_u32(om ? 1u : 0u, r);
            mless += m2 && c2 < oc ? 1u : 0u;
        }
        if (ov) {
            const int64_t pos = base + orank + oless - mless;
            col_out[pos] = (int32_t)oc;
            float v = ow;
            if (om) {
                // entry 2e of (i, j) precedes entry 2e' + 1 of (j, i) iff i < j
                const double x[2] = {(double)((int64_t)i < (int64_t)oc ? ow : wm),
                                     (double)((int64_t)i < (int64_t)oc ? wm : ow)};
                double u = 0.0;
                for (int t = 0; t < 2; ++t) u = u + x[t] - u * x[t];
                v = (float)u;
            }
            val_out[pos] = v;
        }
        // transposed entries without a partner: position = their index in the
        // segment plus the unmatched own entries with a smaller column
        for (int64_t c0 = b; c0 < e; c0 += 64) {
            const int64_t p = c0 + lane;
            const bool iv = p < e;
            const uint32_t ed = iv ? sorted_e[p] : 0u;
            const uint32_t ic = iv ? ed / (uint32_t)k : 0xFFFFFFFFu;
            bool im = false;
            uint32_t uless = 0;
            for (int r = 0; r < k; ++r) {
                const uint32_t ocr = lane_u32(oc, r), m2 = lane_u32(om ? 1u : 0u, r);
                im = im || ic == ocr;
                uless += !m2 && ocr < ic ? 1u : 0u;
            }
            if (iv && !im) {
                const int64_t pos = base + (p - b) + uless;
                col_out[pos] = (int32_t)ic;
                val_out[pos] = w[ed];
            }
        }
    }
}

// Row counts to row_ptr: per-block sums over 1024 rows, their exclusive scan
// (fuzzy_scan_kernel, one block), then each block's rows.
constexpr int kFzScanRows = 1024;

// Exclusive scan of a[0..m) in place by one block (in order, with a
// carry); a[m] receives the total.
__global__ __launch_bounds__(256) void fuzzy_scan_kernel(uint32_t* __restrict__ a, int64_t m)
{
    __shared__ uint32_t s[256];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < m; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t x = b < m ? a[b] : 0u;
        __syncthreads();
        s[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const uint32_t y = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (b < m) a[b] = carry + s[threadIdx.x] - x;
        carry += s[255];
    }
    if (threadIdx.x == 0) a[m] = carry;
}

__global__ __launch_bounds__(256) void fuzzy_block_sum_kernel(const uint32_t* __restrict__ cnt, int64_t n,
                                                              uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t s[4];
    uint32_t t = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = (int64_t)blockIdx.x * kFzScanRows + threadIdx.x * 4 + q;
        t += i < n ? cnt[i] : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) t += shfl_u32(t, (threadIdx.x & 63) ^ o);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(256) void fuzzy_rowptr_kernel(const uint32_t* __restrict__ cnt, int64_t n,
                                                           const uint32_t* __restrict__ boff, int64_t nb,
                                                           int64_t* __restrict__ row_ptr)
{
    __shared__ uint32_t s[256];
    uint32_t c[4], t = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = (int64_t)blockIdx.x * kFzScanRows + threadIdx.x * 4 + q;
        c[q] = i < n ? cnt[i] : 0u;
        t += c[q];
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t y = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    int64_t run = (int64_t)boff[blockIdx.x] + s[threadIdx.x] - t;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = (int64_t)blockIdx.x * kFzScanRows + threadIdx.x * 4 + q;
        if (i < n) row_ptr[i] = run;
        run += c[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) row_ptr[n] = boff[nb];
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
        const int64_t m = n * (int64_t)k;   // edges
        if (2 * m >= ((int64_t)1 << 32)) return fail(KNN_ENOTSUP, "2 n k must be below 2^32");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        knn_status r;
        uint32_t *key, *eid, *k1, *v1, *counts, *inptr, *cnt, *bsum, *oless;
        float* owm;
        unsigned* bad;
        float* w = weights;
        const int64_t nb = ceil_div(n, kFzScanRows);
        if ((r = ws.alloc(&key, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&eid, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&k1, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&v1, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&counts, radix_counts_words(m))) != KNN_OK) return r;
        if ((r = ws.alloc(&inptr, (size_t)n + 1)) != KNN_OK) return r;
        if ((r = ws.alloc(&cnt, (size_t)n)) != KNN_OK) return r;
        if ((r = ws.alloc(&bsum, (size_t)nb + 1)) != KNN_OK) return r;
        if ((r = ws.alloc(&oless, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&owm, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&bad, 1)) != KNN_OK) return r;
        if (!w && (r = ws.alloc(&w, (size_t)n * k)) != KNN_OK) return r;
        KNN_HIP(hipMemsetAsync(bad, 0, 4, st));
        fuzzy_rows_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(knn_idx, knn_dist, n, k, rho, sigma, w, key,
                                                                     eid, bad);
        KNN_HIP(hipGetLastError());
        // by target (keys <= n: invalid edges last), stably
        if ((r = radix_sort_bits(key, eid, k1, v1, m, counts, st, bits_for(n), 1)) != KNN_OK) return r;
        fuzzy_inptr_kernel<<<(unsigned)std::min<int64_t>(ceil_div(m, 256), 8192), 256, 0, st>>>(key, m, n, inptr);
        const unsigned ugrid = (unsigned)std::min<int64_t>(ceil_div(n, 4), 65536);
        fuzzy_union_kernel<false><<<ugrid, 256, 0, st>>>(knn_idx, w, k, n, eid, inptr, cnt, oless, owm, nullptr,
                                                         nullptr, nullptr, bad);
        fuzzy_block_sum_kernel<<<(unsigned)nb, 256, 0, st>>>(cnt, n, bsum);
        fuzzy_scan_kernel<<<1, 256, 0, st>>>(bsum, nb);
        fuzzy_rowptr_kernel<<<(unsigned)nb, 256, 0, st>>>(cnt, n, bsum, nb, row_ptr);
        fuzzy_union_kernel<true><<<ugrid, 256, 0, st>>>(knn_idx, w, k, n, eid, inptr, cnt, oless, owm, row_ptr, col,
                                                        val, bad);
        KNN_HIP(hipGetLastError());
        unsigned host[2] = {0, 0};
        KNN_HIP(hipMemcpyAsync(&host[0], bad, 4, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipMemcpyAsync(&host[1], bsum + nb, 4, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipStreamSynchronize(st));
        if (host[0] & 1u) return fail(KNN_EINVAL, "knn_idx holds an entry out of range or equal to its row");
        if (host[0] & 2u) return fail(KNN_EINVAL, "knn_idx holds a column twice in one row");
        *nnz = (int64_t)host[1];
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}
