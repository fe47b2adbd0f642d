// Learned seeding for NNDescent: an MLP encoder d -> 64 -> 32 (ReLU) trained
// with a triplet loss on k-NN graphs the library builds, and sorted
// projections of its embedding that give every point initial candidates.
//
// Training kernels (all FP32, deterministic):
//   triplets   anchor / positive (one of the anchor's k neighbours) / negative
//              drawn from the counter-based hash;
//   forward    one thread per batch row: h = relu(b1 + x W1), z = b2 + h W2;
//   loss       one thread per triplet: max(0, m + |za-zp|^2 - |za-zn|^2) and
//              dL/dz for the three rows; the loss is summed by a fixed tree;
//   backward   dh = (dz W2^T) masked by h > 0; every weight gradient is a sum
//              over batch rows, taken in two stages (per-chunk partial sums
//              in row order, then a sum over chunks in order), never with
//              floating-point atomics, so results are bitwise reproducible;
//   adam       elementwise update with bias correction.
// Seeding: keys z . r_p for P seeded unit directions, mapped to order-
// preserving u32 and sorted with a stable LSD radix sort (4 x 8-bit passes,
// index payload, so equal keys stay in index order); each point then takes
// the w predecessors and successors in every order, drops itself and
// repeats, ranks them by FP32 squared input distance and keeps the best K.
#include <math.h>

#include <vector>

#include "knn_common.hpp"

struct knn_encoder {
    int d = 0;
    int P = 0;          // parameter count
    float* params = nullptr;   // W1 [d][64] | b1 [64] | W2 [64][32] | b2 [32]
    float* mom = nullptr;
    float* vel = nullptr;
    int t = 0;          // Adam steps taken
};

namespace knn {

constexpr int H1 = KNN_ENC_H1, H2 = KNN_ENC_H2;

struct Off {
    int W1, b1, W2, b2, P;
    __host__ __device__ explicit Off(int d) : W1(0), b1(d * H1), W2(d * H1 + H1), b2(d * H1 + H1 + H1 * H2),
                          P(d * H1 + H1 + H1 * H2 + H2) {}
};

int encoder_dim(const knn_encoder* enc) { return enc ? enc->d : -1; }

// ---------------------------------------------------------------- forward

// One thread per row (rows[i], or i when rows is null).  H (nullable) gets the
// post-ReLU hidden layer, Z the embedding.  Sums run in input order from the
// bias, as fused multiply-adds.
template <int DT>
__global__ __launch_bounds__(256) void mlp_forward_kernel(const void* __restrict__ X, int64_t ld, int d,
                                                          const int32_t* __restrict__ rows, int64_t m,
                                                          const float* __restrict__ prm,
                                                          float* __restrict__ H, float* __restrict__ Z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const Off o(d);
    const int64_t r = rows ? (int64_t)rows[i] : i;
    float h[H1];
#pragma unroll
    for (int j = 0; j < H1; ++j) h[j] = prm[o.b1 + j];
    for (int t = 0; t < d; ++t) {
        const float x = elem<DT>::ld(X, r * ld + t);
        const float* w = prm + o.W1 + t * H1;
#pragma unroll
        for (int j = 0; j < H1; ++j) h[j] = fmaf(x, w[j], h[j]);
    }
#pragma unroll
    for (int j = 0; j < H1; ++j) h[j] = h[j] > 0.0f ? h[j] : 0.0f;
    if (H) {
#pragma unroll
        for (int j = 0; j < H1; ++j) H[i * H1 + j] = h[j];
    }
    float z[H2];
#pragma unroll
    for (int q = 0; q < H2; ++q) z[q] = prm[o.b2 + q];
#pragma unroll
    for (int j = 0; j < H1; ++j) {
        const float* w = prm + o.W2 + j * H2;
#pragma unroll
        for (int q = 0; q < H2; ++q) z[q] = fmaf(h[j], w[q], z[q]);
    }
#pragma unroll
    for (int q = 0; q < H2; ++q) Z[i * H2 + q] = z[q];
}

// BF16 mode (one wave per 32 rows).  The products of both layers run on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation: X rows and W1 are rounded
// to BF16 (RNE) as they are loaded, b1 and ReLU are applied in FP32, the
// hidden layer is rounded to BF16 and re-laid out through LDS as the first
// operand of the second product (W2 rounded), and b2 is added in FP32.
// Operand layouts: lane (h, c) holds row (or column) c, reduction elements
// [16 kk + 8 h, +8) of step kk; an accumulator holds rows 8 (v / 4) + 4 h +
// v % 4 of column c.  H (nullable) gets the rounded hidden values.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ inline float bf16_round(float v) { return __uint_as_float((uint32_t)f32_to_bf16_rne(v) << 16); }

__device__ inline bf16x8_t pack_bf16x8(const float (&v)[8])
{
    uint4 u;
    u.x = (uint32_t)f32_to_bf16_rne(v[0]) | ((uint32_t)f32_to_bf16_rne(v[1]) << 16);
    u.y = (uint32_t)f32_to_bf16_rne(v[2]) | ((uint32_t)f32_to_bf16_rne(v[3]) << 16);
    u.z = (uint32_t)f32_to_bf16_rne(v[4]) | ((uint32_t)f32_to_bf16_rne(v[5]) << 16);
    u.w = (uint32_t)f32_to_bf16_rne(v[6]) | ((uint32_t)f32_to_bf16_rne(v[7]) << 16);
    return __builtin_bit_cast(bf16x8_t, u);
}

template <int DT>
__global__ __launch_bounds__(64) void mlp_forward_bf16_kernel(const void* __restrict__ X, int64_t ld, int d,
                                                              const int32_t* __restrict__ rows, int64_t m,
                                                              const float* __restrict__ prm,
                                                              float* __restrict__ H, float* __restrict__ Z)
{
    __shared__ __attribute__((aligned(16))) uint16_t hs[32][H1 + 8];
    const int lane = threadIdx.x, c = lane & 31, h = lane >> 5;
    const Off o(d);
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    const int64_t i = r0 + c;
    const bool valid = i < m;
    const int64_t src = valid ? (rows ? (int64_t)rows[i] : i) : 0;
    f32x16_t a0, a1;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        a0[v] = 0.0f;
        a1[v] = 0.0f;
    }
    for (int k0 = 0; k0 < d; k0 += 16) {
        float xv[8], w0[8], w1[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int t = k0 + 8 * h + e;
            const bool in = t < d;
            xv[e] = valid && in ? elem<DT>::ld(X, src * ld + t) : 0.0f;
            w0[e] = in ? prm[o.W1 + t * H1 + c] : 0.0f;
            w1[e] = in ? prm[o.W1 + t * H1 + 32 + c] : 0.0f;
        }
        const bf16x8_t xa = pack_bf16x8(xv);
        a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, pack_bf16x8(w0), a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa, pack_bf16x8(w1), a1, 0, 0, 0);
    }
    const float bj0 = prm[o.b1 + c], bj1 = prm[o.b1 + 32 + c];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int r = 8 * (v >> 2) + 4 * h + (v & 3);
        const float h0 = bf16_round(fmaxf(a0[v] + bj0, 0.0f));
        const float h1 = bf16_round(fmaxf(a1[v] + bj1, 0.0f));
        hs[r][c] = (uint16_t)(__float_as_uint(h0) >> 16);
        hs[r][32 + c] = (uint16_t)(__float_as_uint(h1) >> 16);
        if (H && r0 + r < m) {
            H[(r0 + r) * H1 + c] = h0;
            H[(r0 + r) * H1 + 32 + c] = h1;
        }
    }
    __syncthreads();
    f32x16_t az;
#pragma unroll
    for (int v = 0; v < 16; ++v) az[v] = 0.0f;
#pragma unroll
    for (int kk = 0; kk < H1 / 16; ++kk) {
        const bf16x8_t ha = __builtin_bit_cast(bf16x8_t, *(const uint4*)&hs[c][16 * kk + 8 * h]);
        float wv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) wv[e] = prm[o.W2 + (16 * kk + 8 * h + e) * H2 + c];
        az = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha, pack_bf16x8(wv), az, 0, 0, 0);
    }
    const float bq = prm[o.b2 + c];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int r = 8 * (v >> 2) + 4 * h + (v & 3);
        if (r0 + r < m) Z[(r0 + r) * H2 + c] = az[v] + bq;
    }
}

// ------------------------------------------------------------------- loss

__global__ __launch_bounds__(256) void triplet_sample_kernel(int64_t n, const int32_t* __restrict__ knn_idx,
                                                             int k, int B, uint64_t seed, int step,
                                                             int32_t* __restrict__ rows)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const uint64_t s = seed ^ kTagTriplet;
    const uint32_t a = bounded(hash4(s, (uint64_t)step, (uint64_t)b, 0), (uint32_t)n);
    const uint32_t pj = bounded(hash4(s, (uint64_t)step, (uint64_t)b, 1), (uint32_t)k);
    int32_t p = knn_idx[(int64_t)a * k + pj];
    if (p < 0 || p >= n) p = (int32_t)a;
    const uint32_t q = bounded(hash4(s, (uint64_t)step, (uint64_t)b, 2), (uint32_t)n);
    rows[b] = (int32_t)a;
    rows[B + b] = p;
    rows[2 * B + b] = (int32_t)q;
}

// One thread per triplet; Z rows are [anchors; positives; negatives].
__global__ __launch_bounds__(256) void triplet_loss_kernel(const float* __restrict__ Z, int B, float margin,
                                                           float* __restrict__ dZ, float* __restrict__ lterm)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float* za = Z + (int64_t)b * H2;
    const float* zp = Z + (int64_t)(B + b) * H2;
    const float* zn = Z + (int64_t)(2 * B + b) * H2;
    float dp = 0.0f, dn = 0.0f;
#pragma unroll
    for (int q = 0; q < H2; ++q) {
        const float ep = za[q] - zp[q], en = za[q] - zn[q];
        dp = fmaf(ep, ep, dp);
        dn = fmaf(en, en, dn);
    }
    const float g = margin + dp - dn;
    const bool act = g > 0.0f;
    lterm[b] = act ? g : 0.0f;
    const float sc = 2.0f / (float)B;
#pragma unroll
    for (int q = 0; q < H2; ++q) {
        dZ[(int64_t)b * H2 + q] = act ? sc * (zn[q] - zp[q]) : 0.0f;
        dZ[(int64_t)(B + b) * H2 + q] = act ? sc * (zp[q] - za[q]) : 0.0f;
        dZ[(int64_t)(2 * B + b) * H2 + q] = act ? sc * (za[q] - zn[q]) : 0.0f;
    }
}

// Fixed-order sum of m values by one workgroup: each thread sums a strided
// slice in order, then a tree over threads.  out[0] = sum * scale.
__global__ __launch_bounds__(256) void ordered_sum_kernel(const float* __restrict__ v, int64_t m,
                                                          float scale, float* __restrict__ out)
{
    __shared__ float s[256];
    float a = 0.0f;
    for (int64_t i = threadIdx.x; i < m; i += 256) a += v[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0] * scale;
}

// --------------------------------------------------------------- backward

// dH[i][j] = (sum_q dZ[i][q] W2[j][q]) if H[i][j] > 0 else 0.  In the BF16
// mode (BF) the product operands dZ and W2 are rounded to BF16 first.
template <bool BF>
__global__ __launch_bounds__(256) void mlp_dh_kernel(int64_t m, int d, const float* __restrict__ prm,
                                                     const float* __restrict__ H, const float* __restrict__ dZ,
                                                     float* __restrict__ dH)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const Off o(d);
    float dz[H2];
#pragma unroll
    for (int q = 0; q < H2; ++q) dz[q] = BF ? bf16_round(dZ[i * H2 + q]) : dZ[i * H2 + q];
    for (int j = 0; j < H1; ++j) {
        const float* w = prm + o.W2 + j * H2;
        float a = 0.0f;
#pragma unroll
        for (int q = 0; q < H2; ++q) a = fmaf(dz[q], BF ? bf16_round(w[q]) : w[q], a);
        dH[i * H1 + j] = H[i * H1 + j] > 0.0f ? a : 0.0f;
    }
}

constexpr int kGradChunk = 256;   // batch rows per partial sum

// partial[c][p] = sum over the rows of chunk c (in order) of the product that
// defines gradient p: gW1[t][j] = x_t dh_j, gb1[j] = dh_j, gW2[j][q] = h_j dz_q,
// gb2[q] = dz_q.  In the BF16 mode (BF) the factors of the weight-gradient
// products are rounded to BF16 (the bias gradients are plain FP32 sums).
template <int DT, bool BF>
__global__ __launch_bounds__(256) void mlp_grad_partial_kernel(const void* __restrict__ X, int64_t ld, int d,
                                                               const int32_t* __restrict__ rows, int64_t m,
                                                               const float* __restrict__ H,
                                                               const float* __restrict__ dZ,
                                                               const float* __restrict__ dH,
                                                               float* __restrict__ partial)
{
    const Off o(d);
    const int p = blockIdx.y * blockDim.x + threadIdx.x;
    if (p >= o.P) return;
    const int c = blockIdx.x;
    const int64_t i0 = (int64_t)c * kGradChunk;
    const int64_t i1 = i0 + kGradChunk < m ? i0 + kGradChunk : m;
    float a = 0.0f;
    if (p < o.b1) {
        const int t = p / H1, j = p % H1;
        for (int64_t i = i0; i < i1; ++i) {
            const int64_t r = rows ? (int64_t)rows[i] : i;
            const float x = elem<DT>::ld(X, r * ld + t), g = dH[i * H1 + j];
            a = BF ? fmaf(bf16_round(x), bf16_round(g), a) : fmaf(x, g, a);
        }
    } else if (p < o.W2) {
        const int j = p - o.b1;
        for (int64_t i = i0; i < i1; ++i) a += dH[i * H1 + j];
    } else if (p < o.b2) {
        const int j = (p - o.W2) / H2, q = (p - o.W2) % H2;
        for (int64_t i = i0; i < i1; ++i)
            a = BF ? fmaf(bf16_round(H[i * H1 + j]), bf16_round(dZ[i * H2 + q]), a)
                   : fmaf(H[i * H1 + j], dZ[i * H2 + q], a);
    } else {
        const int q = p - o.b2;
        for (int64_t i = i0; i < i1; ++i) a += dZ[i * H2 + q];
    }
    partial[(int64_t)c * o.P + p] = a;
}

__global__ __launch_bounds__(256) void grad_reduce_kernel(const float* __restrict__ partial, int nch, int P,
                                                          float* __restrict__ g)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float a = 0.0f;
    for (int c = 0; c < nch; ++c) a += partial[(int64_t)c * P + p];
    g[p] = a;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                                                   float* __restrict__ mo, float* __restrict__ ve, int P,
                                                   float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float gg = g[p];
    const float mm = b1 * mo[p] + (1.0f - b1) * gg;
    const float vv = b2 * ve[p] + (1.0f - b2) * gg * gg;
    mo[p] = mm;
    ve[p] = vv;
    w[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ------------------------------------------------------------ radix sort

constexpr int kRsThreads = 256, kRsItems = 16, kRsTile = kRsThreads * kRsItems;

__host__ __device__ inline size_t rs_counts(int64_t n)
{
    return (size_t)256 * ((n + kRsTile - 1) / kRsTile) + 256;
}

// Sorts run on blockIdx.y independent arrays of n elements at once: array
// y's elements (and outputs) start at y * n, its counts at y * rs_counts(n).
__global__ __launch_bounds__(256) void rs_hist_kernel(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                      uint32_t* __restrict__ counts, int nblk)
{
    __shared__ uint32_t hist[256];
    keys += (int64_t)blockIdx.y * n;
    counts += (int64_t)blockIdx.y * rs_counts(n);
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int it = 0; it < kRsItems; ++it) {
        const int64_t e = base + it * kRsThreads + threadIdx.x;
        if (e < n) atomicAdd(&hist[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = hist[threadIdx.x];
}

// Exclusive scan of one value per thread of a 256-thread block (LDS
// Hillis-Steele); *total receives the sum.
__device__ inline uint32_t block_exscan256(uint32_t x, uint32_t* s, uint32_t* total)
{
    const int t = threadIdx.x;
    __syncthreads();
    s[t] = x;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {
        const uint32_t y = t >= w ? s[t - w] : 0u;
        __syncthreads();
        s[t] += y;
        __syncthreads();
    }
    const uint32_t incl = s[t];
    *total = s[255];
    return incl - x;
}

// Counts are digit-major (c[digit * nblk + tile]).  Block `digit` turns its
// row into exclusive prefix sums over the tiles and writes the row total to
// tot[digit]; the scatter adds the exclusive prefix of the totals.
__global__ __launch_bounds__(256) void rs_scan_kernel(uint32_t* __restrict__ c, int64_t n, int nblk)
{
    __shared__ uint32_t s[256];
    c += (int64_t)blockIdx.y * rs_counts(n);
    uint32_t* tot = c + (int64_t)256 * nblk;
    uint32_t* row = c + (int64_t)blockIdx.x * nblk;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        const int b = b0 + (int)threadIdx.x;
        const uint32_t x = b < nblk ? row[b] : 0u;
        uint32_t sum;
        const uint32_t ex = block_exscan256(x, s, &sum);
        if (b < nblk) row[b] = carry + ex;
        carry += sum;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Stable scatter of one 8-bit digit: elements of a tile are visited in index
// order (item-major, then thread); within a wave, lanes with equal digits are
// ranked by a ballot match over the 8 digit bits; across waves by per-wave
// counts in LDS; across tiles by the scanned histogram.
__global__ __launch_bounds__(256) void rs_scatter_kernel(const uint32_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin,
                                                         uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                         int64_t n, int shift,
                                                         const uint32_t* __restrict__ offs, int nblk)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t sc[256];
    const int64_t so = (int64_t)blockIdx.y * n;
    kin += so;
    vin += so;
    kout += so;
    vout += so;
    offs += (int64_t)blockIdx.y * rs_counts(n);
    const uint32_t* tot = offs + (int64_t)256 * nblk;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t all;
    const uint32_t dbase = block_exscan256(tot[tid], sc, &all);
    run[tid] = dbase + offs[(int64_t)tid * nblk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < kRsItems; ++it) {
        const int64_t e = base + it * kRsThreads + tid;
        const bool valid = e < n;
        const uint32_t key = valid ? kin[e] : 0u;
        const uint32_t val = valid ? vin[e] : 0u;
        const uint32_t dig = (key >> shift) & 255u;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t bal = ballot(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt);
        const int cnt = __popcll(peers);
        wcnt[0][tid] = 0;
        wcnt[1][tid] = 0;
        wcnt[2][tid] = 0;
        wcnt[3][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wcnt[wv][dig] = (uint32_t)cnt;
        __syncthreads();
        if (valid) {
            uint32_t pos = run[dig] + (uint32_t)rank;
            for (int w = 0; w < wv; ++w) pos += wcnt[w][dig];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

knn_status radix_sort_bits(uint32_t*& k0, uint32_t*& v0, uint32_t*& k1, uint32_t*& v1, int64_t n,
                           uint32_t* counts, hipStream_t st, int bits, int S);

// Sort S independent arrays of (key, value) pairs, n each and contiguous
// (k0 + y n, ...), by key, stable; results in (k0, v0).  k1 / v1 hold S n
// words and counts S rs_counts(n) words.
static knn_status radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                                   uint32_t* counts, hipStream_t st, int S = 1)
{
    return radix_sort_bits(k0, v0, k1, v1, n, counts, st, 32, S);
}

size_t radix_counts_words(int64_t n) { return rs_counts(n); }

// As radix_sort_pairs, on keys below 2^bits: ceil(bits / 8) passes (bits in
// 1..32).  An odd pass count leaves the result in (k1, v1): the pointers are
// swapped so that (k0, v0) name the sorted arrays on return.
knn_status radix_sort_bits(uint32_t*& k0, uint32_t*& v0, uint32_t*& k1, uint32_t*& v1, int64_t n,
                           uint32_t* counts, hipStream_t st, int bits, int S)
{
    const int nblk = (int)ceil_div(n, kRsTile);
    const int npass = (bits + 7) / 8;
    for (int pass = 0; pass < npass; ++pass) {
        const int shift = 8 * pass;
        rs_hist_kernel<<<dim3((unsigned)nblk, (unsigned)S), kRsThreads, 0, st>>>(k0, n, shift, counts, nblk);
        rs_scan_kernel<<<dim3(256, (unsigned)S), 256, 0, st>>>(counts, n, nblk);
        rs_scatter_kernel<<<dim3((unsigned)nblk, (unsigned)S), kRsThreads, 0, st>>>(k0, v0, k1, v1, n, shift,
                                                                                   counts, nblk);
        KNN_HIP(hipGetLastError());
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    return KNN_OK;
}

// -------------------------------------------------------------- seeding

// Y[q][i] = Z_i . dirs_q (FP32 fused multiply-adds in coordinate order) for
// the P*D directions q.  The row of Z is read once into registers (M = m when
// m <= 32, else a strided fallback).
template <int M>
__global__ __launch_bounds__(256) void proj_vals_kernel(const float* __restrict__ Z, int64_t n, int m,
                                                        const float* __restrict__ dirs, int PD,
                                                        float* __restrict__ Y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if constexpr (M > 0) {
        float z[M];
        if (m == M && ((uintptr_t)Z & 15u) == 0) {   // 16-byte aligned rows of M floats: read as vectors
#pragma unroll
            for (int t = 0; t < M; t += 4) {
                const float4 v = *(const float4*)(Z + i * M + t);
                z[t] = v.x;
                z[t + 1] = v.y;
                z[t + 2] = v.z;
                z[t + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < M; ++t) z[t] = t < m ? Z[i * m + t] : 0.0f;
        }
        for (int q = 0; q < PD; ++q) {
            float s = 0.0f;
#pragma unroll
            for (int t = 0; t < M; ++t)
                if (t < m) s = fmaf(z[t], dirs[q * m + t], s);
            Y[(int64_t)q * n + i] = s;
        }
    } else {
        for (int q = 0; q < PD; ++q) {
            float s = 0.0f;
            for (int t = 0; t < m; ++t) s = fmaf(Z[i * m + t], dirs[q * m + t], s);
            Y[(int64_t)q * n + i] = s;
        }
    }
}

__device__ inline uint32_t f32_order(float f)
{
    if (f == 0.0f) return 0x80000000u;
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float f32_unorder(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

__global__ __launch_bounds__(64) void lohi_init_kernel(unsigned* __restrict__ lohi, int nq)
{
    const int q = threadIdx.x;
    if (q < nq) {
        lohi[2 * q] = 0xFFFFFFFFu;
        lohi[2 * q + 1] = 0u;
    }
}

// Per direction q: lohi[2q] = min, lohi[2q+1] = max of Y[q][*] as ordered
// uint32 (integer atomics: exact and order-free), one atomic pair per block
// after an in-block reduction.  lohi starts at (~0, 0) (lohi_init_kernel).
__global__ __launch_bounds__(256) void minmax_kernel(const float* __restrict__ Y, int64_t n,
                                                     unsigned* __restrict__ lohi)
{
    __shared__ uint32_t slo[4], shi[4];
    const int q = blockIdx.y;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = f32_order(Y[(int64_t)q * n + i]);
        lo = u < lo ? u : lo;
        hi = u > hi ? u : hi;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t a = xor_u32(lo, o), b = xor_u32(hi, o);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        slo[wv] = lo;
        shi[wv] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            lo = slo[w] < lo ? slo[w] : lo;
            hi = shi[w] > hi ? shi[w] : hi;
        }
        atomicMin(&lohi[2 * q], lo);
        atomicMax(&lohi[2 * q + 1], hi);
    }
}

// Blocks per direction for minmax_kernel: enough to stream Y, few atomics.
static unsigned minmax_blocks(int64_t n) { return (unsigned)std::min<int64_t>(ceil_div(n, 256), 64); }

// keys[p][i]: D = 1 -> the ordered projection; D > 1 -> Z-order code of the D
// projections, each quantised to b = 32/D bits over [lo, hi]:
// q = min(floor((y - lo) * (2^b / (hi - lo))), 2^b - 1), bits interleaved
// from the most significant level down.
template <int D>
__global__ __launch_bounds__(256) void morton_kernel(const float* __restrict__ Y, int64_t n, int P,
                                                     const unsigned* __restrict__ lohi,
                                                     uint32_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int bits = 32 / D;
    for (int p = 0; p < P; ++p) {
        uint32_t key;
        if constexpr (D == 1) {
            key = f32_order(Y[(int64_t)p * n + i]);
        } else {
            uint32_t code[D];
            constexpr uint32_t qmax = (1u << bits) - 1u;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int q = p * D + j;
                const float lo = f32_unorder(lohi[2 * q]), hi = f32_unorder(lohi[2 * q + 1]);
                const float sc = hi > lo ? (float)(1u << bits) / (hi - lo) : 0.0f;
                const float f = floorf((Y[(int64_t)q * n + i] - lo) * sc);
                const uint32_t c = f <= 0.0f ? 0u : (uint32_t)f;
                code[j] = c < qmax ? c : qmax;
            }
            key = 0;
#pragma unroll
            for (int l = bits - 1; l >= 0; --l)
#pragma unroll
                for (int j = 0; j < D; ++j) key = (key << 1) | ((code[j] >> l) & 1u);
        }
        keys[(int64_t)p * n + i] = key;
        vals[(int64_t)p * n + i] = (uint32_t)i;
    }
}

static void launch_morton(const float* Y, int64_t n, int P, int D, const unsigned* lohi, uint32_t* keys,
                          uint32_t* vals, hipStream_t st)
{
    const unsigned g = (unsigned)ceil_div(n, 256);
    if (D == 1) morton_kernel<1><<<g, 256, 0, st>>>(Y, n, P, lohi, keys, vals);
    else if (D == 2) morton_kernel<2><<<g, 256, 0, st>>>(Y, n, P, lohi, keys, vals);
    else if (D == 4) morton_kernel<4><<<g, 256, 0, st>>>(Y, n, P, lohi, keys, vals);
    else morton_kernel<8><<<g, 256, 0, st>>>(Y, n, P, lohi, keys, vals);
}

__global__ __launch_bounds__(256) void inverse_perm_kernel(const uint32_t* __restrict__ order, int64_t n,
                                                           uint32_t* __restrict__ pos)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) pos[order[r]] = (uint32_t)r;
}

// Y[j][i] = X_i . dirs_j over the d input coordinates, D <= 8 directions.
// 16 lanes per row (coalesced row reads), each summing a strided subset of
// the coordinates, then a 16-lane reduction.  With Staged the directions
// are first copied to LDS (D * d floats of dynamic shared memory).
template <int DT, bool Staged>
__global__ __launch_bounds__(256) void xproj_kernel(const void* __restrict__ X, int64_t ld, int d, int64_t n,
                                                    const float* __restrict__ dirs_g, int D,
                                                    float* __restrict__ Y)
{
    extern __shared__ float sdirs[];
    if (Staged) {
        for (int q = threadIdx.x; q < D * d; q += 256) sdirs[q] = dirs_g[q];
        __syncthreads();
    }
    const float* dirs = Staged ? sdirs : dirs_g;
    const int g = threadIdx.x & 15;
    const int64_t i = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const bool live = i < n;
    float y[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) y[j] = 0.0f;
    if (live) {
        for (int t = g; t < d; t += 16) {
            const float x = elem<DT>::ld(X, i * ld + t);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j < D) y[j] = fmaf(x, dirs[j * d + t], y[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) y[j] += xor_f32(y[j], o);
    if (live) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < D && g == j) Y[(int64_t)j * n + i] = y[j];
    }
}

// Window distances of one sorted order (blockIdx.y = p).  A block owns the
// 256 - w positions [t0, t0 + 256 - w) and its thread j takes position
// t = t0 - w + j: the canonical FP32 distances from that point to the points
// at t + 1 .. t + w (sequential fused multiply-adds over the coordinates in
// order, one lane per pair), so each window pair is computed once per order.
// The rows of the block's 256 + w positions are staged in LDS 128 bytes
// (CH elements) at a time, zero past d (a zero difference leaves a sum
// unchanged), with a 16-byte pad per row so that lanes reading consecutive
// rows hit distinct banks.  Owned positions then list their w predecessors
// (slots 0 .. w-1, nearest first; the distances come from the predecessors'
// threads through LDS) and w successors (slots w .. 2w-1) in their point's
// row of win_idx / win_d2, order p at slots [2wp, 2wp + 2w); positions past
// either end get index -1.  The squared difference of two values does not
// depend on their order, so a pair's distance is the one the point on
// either side would compute.
template <int DT, int W>
__global__ __launch_bounds__(256) void window_dist_kernel(const void* __restrict__ X, int64_t ld, int d, int64_t n,
                                                          const uint32_t* __restrict__ order, int w, int PW, bool vec,
                                                          int32_t* __restrict__ win_idx, float* __restrict__ win_d2)
{
    using T = typename elem<DT>::T;
    constexpr int V = 16 / (int)sizeof(T);   // elements per 16-byte vector
    constexpr int CH = 8 * V;                // elements per staged chunk (128 bytes of a row)
    constexpr int RS = 9;                    // LDS row stride in 16-byte vectors
    extern __shared__ uint4 tile[];          // (256 + w) x RS vectors; reused for the distances
    __shared__ uint32_t rid[256 + 32];
    const int p = blockIdx.y, j = threadIdx.x, nr = 256 + w;
    const int64_t base = (int64_t)blockIdx.x * (256 - w) - w;   // position of staged row 0 (= thread 0)
    const uint32_t* ord = order + (int64_t)p * n;
    for (int r = j; r < nr; r += 256) {
        const int64_t t = base + r;
        rid[r] = t >= 0 && t < n ? ord[t] : 0xFFFFFFFFu;
    }
    __syncthreads();
    float sum[W];
#pragma unroll
    for (int o = 0; o < W; ++o) sum[o] = 0.0f;
    for (int c0 = 0; c0 < d; c0 += CH) {
        // a thread stages at most 9 vectors ((256 + 32) x 8 / 256): all of
        // its loads are issued before the first LDS store
        uint4 xs[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            const int q = j + 256 * u;
            const int r = q >> 3, e0 = c0 + (q & 7) * V;
            const uint32_t id = q < nr * 8 ? rid[r] : 0xFFFFFFFFu;
            xs[u] = make_uint4(0u, 0u, 0u, 0u);
            if (id != 0xFFFFFFFFu && e0 < d) {
                const T* src = (const T*)X + (int64_t)id * ld + e0;
                if (vec && e0 + V <= d) {
                    xs[u] = *(const uint4*)src;
                } else {
                    T tmp[V];
#pragma unroll
                    for (int e = 0; e < V; ++e) tmp[e] = e0 + e < d ? src[e] : T(0);
                    __builtin_memcpy(&xs[u], tmp, sizeof(uint4));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            const int q = j + 256 * u;
            if (q < nr * 8) tile[(q >> 3) * RS + (q & 7)] = xs[u];
        }
        __syncthreads();
        const int nv = min(8, (d - c0 + V - 1) / V);
        for (int v = 0; v < nv; ++v) {
            const uint4 ua = tile[j * RS + v];
            const T* pa = (const T*)&ua;
#pragma unroll
            for (int o = 0; o < W; ++o) {
                if (o < w) {
                    const uint4 ub = tile[(j + o + 1) * RS + v];
                    const T* pb = (const T*)&ub;
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        const float x = elem<DT>::ld(pa, e) - elem<DT>::ld(pb, e);
                        sum[o] = fmaf(x, x, sum[o]);
                    }
                }
            }
        }
        __syncthreads();
    }
    float* fd = (float*)tile;   // fd[o * 256 + j]: distance of staged row j to row j + o + 1
    const int64_t t = base + j;
    const bool live = t >= 0 && t < n;
#pragma unroll
    for (int o = 0; o < W; ++o)
        if (o < w) fd[o * 256 + j] = sum[o];
    __syncthreads();
    if (j < w || !live) return;
    const int64_t row = (int64_t)rid[j] * PW + (int64_t)p * 2 * w;
    if (w == W) {
        // the 2W entries are contiguous and 16-byte aligned (PW = 2WP):
        // written as 16-byte vectors
        int32_t oi[2 * W];
        float od[2 * W];
#pragma unroll
        for (int o = 1; o <= W; ++o) {
            const bool lv = t - o >= 0, rv = t + o < n;
            oi[o - 1] = lv ? (int32_t)rid[j - o] : -1;
            od[o - 1] = lv ? fd[(o - 1) * 256 + j - o] : 0.0f;
            oi[W + o - 1] = rv ? (int32_t)rid[j + o] : -1;
            od[W + o - 1] = rv ? fd[(o - 1) * 256 + j] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < W / 2; ++u) {
            *(int4*)(win_idx + row + 4 * u) = make_int4(oi[4 * u], oi[4 * u + 1], oi[4 * u + 2], oi[4 * u + 3]);
            *(float4*)(win_d2 + row + 4 * u) = make_float4(od[4 * u], od[4 * u + 1], od[4 * u + 2], od[4 * u + 3]);
        }
        return;
    }
    for (int o = 1; o <= w; ++o) {
        const bool lv = t - o >= 0, rv = t + o < n;
        win_idx[row + o - 1] = lv ? (int32_t)rid[j - o] : -1;
        win_d2[row + o - 1] = lv ? fd[(o - 1) * 256 + j - o] : 0.0f;
        win_idx[row + w + o - 1] = rv ? (int32_t)rid[j + o] : -1;
        win_d2[row + w + o - 1] = rv ? fd[(o - 1) * 256 + j] : 0.0f;
    }
}

// One wave per point: its PW = 2wP window entries (lane = (p, side,
// offset)), repeats and self dropped (a repeat carries the same distance),
// best K by (distance, index), sorted.
__global__ __launch_bounds__(256) void proj_seed_kernel(int64_t n, const int32_t* __restrict__ win_idx,
                                                        const float* __restrict__ win_d2, int PW, int K,
                                                        int32_t* __restrict__ out_idx, float* __restrict__ out_d2)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const uint32_t cand = lane < PW ? (uint32_t)win_idx[i * PW + lane] : 0xFFFFFFFFu;
    const float cd = lane < PW ? win_d2[i * PW + lane] : 0.0f;
    // repeats: every lane compares with all earlier lanes through LDS broadcasts
    __shared__ __attribute__((aligned(16))) uint32_t sc[4][64];
    const int wv = threadIdx.x >> 6;
    sc[wv][lane] = cand;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    bool ok = cand != 0xFFFFFFFFu && cand != (uint32_t)i;
#pragma unroll 4
    for (int o = 0; o < 64; o += 4) {
        const uint4 x = *(const uint4*)&sc[wv][o];
        ok = ok && !(o + 0 < lane && x.x == cand) && !(o + 1 < lane && x.y == cand) &&
             !(o + 2 < lane && x.z == cand) && !(o + 3 < lane && x.w == cand);
    }
    uint64_t key = ok ? make_key(cd, cand) : kEmptyCand;
    key = seg_sort<64>(key);
    if (lane < K) {
        const bool v = key_valid(key);
        out_idx[i * K + lane] = v ? (int32_t)key_idx(key) : -1;
        out_d2[i * K + lane] = v ? key_d2(key) : __builtin_inff();
    }
}

template <typename F>
static void by_dtype(int dt, F&& f)
{
    if (dt == KNN_F32) f(std::integral_constant<int, KNN_F32>());
    else if (dt == KNN_BF16) f(std::integral_constant<int, KNN_BF16>());
    else f(std::integral_constant<int, KNN_F16>());
}

// Seeds from sorted projections.  With `win_idx` the ranking is left to the
// caller: the 2wP window entries of every point (index, squared distance;
// n x 2wP each) are returned there and out_idx / out_d2 are not written.
static knn_status proj_seed_impl(const knn_matrix& X, const float* Z, int m, const float* dirs, int P, int D,
                                 int w, int K, int32_t* out_idx, float* out_d2, Workspace& ws, hipStream_t st,
                                 int32_t** win_idx = nullptr, float** win_d2 = nullptr)
{
    const int64_t n = X.n;
    uint32_t *keys, *vals, *k1, *v1, *counts, *lohi;
    float* Y;
    knn_status r;
    if ((r = ws.alloc(&Y, (size_t)n * P * D)) != KNN_OK) return r;
    if ((r = ws.alloc(&lohi, (size_t)2 * P * D)) != KNN_OK) return r;
    if ((r = ws.alloc(&keys, (size_t)n * P)) != KNN_OK) return r;
    if ((r = ws.alloc(&vals, (size_t)n * P)) != KNN_OK) return r;
    if ((r = ws.alloc(&k1, (size_t)n * P)) != KNN_OK) return r;
    if ((r = ws.alloc(&v1, (size_t)n * P)) != KNN_OK) return r;
    if ((r = ws.alloc(&counts, rs_counts(n) * P)) != KNN_OK) return r;
    const unsigned g = (unsigned)ceil_div(n, 256);
    if (m <= 32) proj_vals_kernel<32><<<g, 256, 0, st>>>(Z, n, m, dirs, P * D, Y);
    else proj_vals_kernel<0><<<g, 256, 0, st>>>(Z, n, m, dirs, P * D, Y);
    if (D > 1) {
        lohi_init_kernel<<<1, 64, 0, st>>>(lohi, P * D);
        minmax_kernel<<<dim3(minmax_blocks(n), (unsigned)(P * D)), 256, 0, st>>>(Y, n, lohi);
    }
    launch_morton(Y, n, P, D, lohi, keys, vals, st);
    KNN_HIP(hipGetLastError());
    // the P orders are sorted together
    if ((r = radix_sort_pairs(keys, vals, k1, v1, n, counts, st, P)) != KNN_OK) return r;
    // window distances per order, then each point's best K of its windows
    const int PW = 2 * w * P;
    int32_t* wi;
    float* wd;
    if ((r = ws.alloc(&wi, (size_t)n * PW)) != KNN_OK) return r;
    if ((r = ws.alloc(&wd, (size_t)n * PW)) != KNN_OK) return r;
    const int64_t eb = X.dtype == KNN_F32 ? 4 : 2;
    const bool vec = ((uintptr_t)X.data % 16 == 0) && ((X.ld * eb) % 16 == 0);
    const dim3 wgrid((unsigned)ceil_div(n, 256 - w), (unsigned)P);
    // staged rows, or the distances of every thread, whichever is larger
    const size_t lds = std::max((size_t)(256 + w) * 9 * 16, (size_t)w * 256 * sizeof(float));
    by_dtype(X.dtype, [&](auto dt) {
        constexpr int DT = decltype(dt)::value;
        if (w <= 8)
            window_dist_kernel<DT, 8><<<wgrid, 256, lds, st>>>(X.data, X.ld, X.d, n, vals, w, PW, vec, wi, wd);
        else if (w <= 16)
            window_dist_kernel<DT, 16><<<wgrid, 256, lds, st>>>(X.data, X.ld, X.d, n, vals, w, PW, vec, wi, wd);
        else
            window_dist_kernel<DT, 32><<<wgrid, 256, lds, st>>>(X.data, X.ld, X.d, n, vals, w, PW, vec, wi, wd);
    });
    KNN_HIP(hipGetLastError());
    if (win_idx) {
        *win_idx = wi;
        *win_d2 = wd;
        return KNN_OK;
    }
    proj_seed_kernel<<<(unsigned)ceil_div(n, 4), 256, 0, st>>>(n, wi, wd, PW, K, out_idx, out_d2);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}


// P seeded directions on the unit sphere in R^m: Gaussians from the
// Box-Muller transform of the counter-based hash (FP64), normalised.  One
// wave per direction.
__global__ __launch_bounds__(64) void dirs_kernel(int m, uint64_t seed, float* __restrict__ out)
{
    const int p = blockIdx.x, lane = threadIdx.x;
    double ss = 0.0;
    for (int t = lane; t < m; t += 64) {
        const uint64_t h = hash4(seed ^ kTagDirs, (uint64_t)p, (uint64_t)t, 0);
        const double u1 = ((h >> 11) + 1.0) * (1.0 / 9007199254740993.0);
        const double u2 = (double)(hash4(seed ^ kTagDirs, (uint64_t)p, (uint64_t)t, 1) >> 11) *
                          (1.0 / 9007199254740992.0);
        const double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        out[(int64_t)p * m + t] = (float)g;
        ss += g * g;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t b = __double_as_longlong(ss);
        const uint32_t lo = xor_u32((uint32_t)b, o), hi = xor_u32((uint32_t)(b >> 32), o);
        ss += __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
    }
    const double inv = 1.0 / sqrt(ss);
    for (int t = lane; t < m; t += 64) out[(int64_t)p * m + t] = (float)((double)out[(int64_t)p * m + t] * inv);
}

// Internal processing order of the points: the Z-order curve of D seeded
// random projections of X (4-bit codes for D = 8), ties by index.  Points
// that are close get close positions, so rows and candidate slots touched
// together share cache lines.  perm[new] = old, inv[old] = new.
knn_status morton_order(const knn_matrix& X, int D, uint64_t seed, Workspace& ws, uint32_t** perm,
                        uint32_t** inv, hipStream_t st)
{
    const int64_t n = X.n;
    knn_status r;
    float *Y, *dirs;
    uint32_t *keys, *k1, *v1, *lohi, *counts;
    if ((r = ws.alloc(&Y, (size_t)n * D)) != KNN_OK) return r;
    if ((r = ws.alloc(&dirs, (size_t)D * X.d)) != KNN_OK) return r;
    if ((r = ws.alloc(&keys, (size_t)n)) != KNN_OK) return r;
    if ((r = ws.alloc(perm, (size_t)n)) != KNN_OK) return r;
    if ((r = ws.alloc(inv, (size_t)n)) != KNN_OK) return r;
    if ((r = ws.alloc(&k1, (size_t)n)) != KNN_OK) return r;
    if ((r = ws.alloc(&v1, (size_t)n)) != KNN_OK) return r;
    if ((r = ws.alloc(&lohi, (size_t)2 * D)) != KNN_OK) return r;
    if ((r = ws.alloc(&counts, rs_counts(n))) != KNN_OK) return r;
    dirs_kernel<<<D, 64, 0, st>>>(X.d, seed ^ 0x5DEECE66Dull, dirs);
    const unsigned g = (unsigned)ceil_div(n, 256);
    const bool staged = (size_t)D * X.d * sizeof(float) <= 32768;
    const size_t lds = staged ? (size_t)D * X.d * sizeof(float) : 0;
    const unsigned xg = (unsigned)ceil_div(n, 16);
    by_dtype(X.dtype, [&](auto dt) {
        constexpr int DT = decltype(dt)::value;
        if (staged) xproj_kernel<DT, true><<<xg, 256, lds, st>>>(X.data, X.ld, X.d, n, dirs, D, Y);
        else xproj_kernel<DT, false><<<xg, 256, 0, st>>>(X.data, X.ld, X.d, n, dirs, D, Y);
    });
    lohi_init_kernel<<<1, 64, 0, st>>>(lohi, D);
    minmax_kernel<<<dim3(minmax_blocks(n), (unsigned)D), 256, 0, st>>>(Y, n, lohi);
    launch_morton(Y, n, 1, D, lohi, keys, *perm, st);
    KNN_HIP(hipGetLastError());
    if ((r = radix_sort_pairs(keys, *perm, k1, v1, n, counts, st)) != KNN_OK) return r;
    inverse_perm_kernel<<<g, 256, 0, st>>>(*perm, n, *inv);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

// Forward pass of rows (nullable: 0..m-1) in the given precision.
static knn_status forward_impl(const knn_encoder* enc, const knn_matrix& X, const int32_t* rows, int64_t m,
                               int precision, float* H, float* Z, hipStream_t st)
{
    by_dtype(X.dtype, [&](auto dt) {
        if (precision == KNN_PREC_BF16)
            mlp_forward_bf16_kernel<decltype(dt)::value><<<(unsigned)ceil_div(m, 32), 64, 0, st>>>(
                X.data, X.ld, X.d, rows, m, enc->params, H, Z);
        else
            mlp_forward_kernel<decltype(dt)::value><<<(unsigned)ceil_div(m, 256), 256, 0, st>>>(
                X.data, X.ld, X.d, rows, m, enc->params, H, Z);
    });
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

// Seed lists from the encoder: X is embedded in the given precision, the
// seeds' distances are taken on Xd (the same points; the BF16 copy in the
// BF16 form).
knn_status encoder_seed(const knn_encoder* enc, const knn_matrix& X, const knn_matrix& Xd, int precision, int P,
                        int D, int w, uint64_t seed, Workspace& ws, int32_t** seed_idx, float** seed_d2,
                        hipStream_t st)
{
    if (2 * w * P > 64) return fail(KNN_EINVAL, "2 * proj_window * proj_count must be <= 64");
    if (D < 1 || D > 8 || 32 % D) return fail(KNN_EINVAL, "proj_dims must be 1, 2, 4 or 8");
    knn_status r;
    float *Z, *dirs;
    if ((r = ws.alloc(&Z, (size_t)X.n * H2)) != KNN_OK) return r;
    if ((r = ws.alloc(&dirs, (size_t)P * D * H2)) != KNN_OK) return r;
    dirs_kernel<<<P * D, 64, 0, st>>>(H2, seed, dirs);
    KNN_HIP(hipGetLastError());
    if ((r = forward_impl(enc, X, nullptr, X.n, precision, nullptr, Z, st)) != KNN_OK) return r;
    return proj_seed_impl(Xd, Z, H2, dirs, P, D, w, 0, nullptr, nullptr, ws, st, seed_idx, seed_d2);
}

// Forward + loss + backward of one batch (rows: 3B device ints).  Leaves the
// loss sum in loss_dev[0] (already divided by B) and the gradient in grad.
static knn_status batch_grads(const knn_encoder* enc, const knn_matrix& X, const int32_t* rows, int B,
                              float margin, int precision, float* H, float* Z, float* dZ, float* dH,
                              float* lterm, float* partial, float* grad, float* loss_dev, hipStream_t st)
{
    const int64_t m = 3 * (int64_t)B;
    const Off o(enc->d);
    const bool bf = precision == KNN_PREC_BF16;
    knn_status r = forward_impl(enc, X, rows, m, precision, H, Z, st);
    if (r != KNN_OK) return r;
    triplet_loss_kernel<<<(unsigned)ceil_div(B, 256), 256, 0, st>>>(Z, B, margin, dZ, lterm);
    ordered_sum_kernel<<<1, 256, 0, st>>>(lterm, B, 1.0f / (float)B, loss_dev);
    if (bf) mlp_dh_kernel<true><<<(unsigned)ceil_div(m, 256), 256, 0, st>>>(m, enc->d, enc->params, H, dZ, dH);
    else mlp_dh_kernel<false><<<(unsigned)ceil_div(m, 256), 256, 0, st>>>(m, enc->d, enc->params, H, dZ, dH);
    const int nch = (int)ceil_div(m, kGradChunk);
    dim3 g((unsigned)nch, (unsigned)ceil_div(o.P, 256));
    by_dtype(X.dtype, [&](auto dt) {
        if (bf)
            mlp_grad_partial_kernel<decltype(dt)::value, true><<<g, 256, 0, st>>>(X.data, X.ld, X.d, rows, m, H,
                                                                                  dZ, dH, partial);
        else
            mlp_grad_partial_kernel<decltype(dt)::value, false><<<g, 256, 0, st>>>(X.data, X.ld, X.d, rows, m, H,
                                                                                   dZ, dH, partial);
    });
    grad_reduce_kernel<<<(unsigned)ceil_div(o.P, 256), 256, 0, st>>>(partial, nch, o.P, grad);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

// Adam step number t (1-based) on the encoder's FP32 weights with gradient
// grad: the bias corrections 1 - beta^t are computed on the host in double
// (in FP32, 1 - 0.999^t loses about 2^-24 / (1 - 0.999^t) relative to the
// cancellation: 3e-5 at t = 2) and rounded once.
static knn_status adam_apply(knn_encoder* enc, const float* grad, const knn_train_params& tp, int t,
                             hipStream_t st)
{
    const float c1 = (float)(1.0 - pow((double)tp.beta1, (double)t));
    const float c2 = (float)(1.0 - pow((double)tp.beta2, (double)t));
    adam_kernel<<<(unsigned)ceil_div(enc->P, 256), 256, 0, st>>>(enc->params, grad, enc->mom, enc->vel, enc->P,
                                                                 tp.lr, tp.beta1, tp.beta2, tp.eps, c1, c2);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

}  // namespace knn

using namespace knn;

extern "C" knn_status knn_encoder_create(int32_t d, uint64_t seed, knn_encoder** enc)
{
    try {
        if (!enc) return fail(KNN_EINVAL, "enc is null");
        *enc = nullptr;
        if (d < 1) return fail(KNN_EINVAL, "d must be >= 1");
        const Off o(d);
        knn_encoder* e = new knn_encoder();
        e->d = d;
        e->P = o.P;
        if (hipMalloc(&e->params, (size_t)o.P * 4) != hipSuccess || hipMalloc(&e->mom, (size_t)o.P * 4) != hipSuccess ||
            hipMalloc(&e->vel, (size_t)o.P * 4) != hipSuccess) {
            (void)hipGetLastError();
            knn_encoder_destroy(e);
            return fail(KNN_ENOMEM, "encoder allocation failed");
        }
        // He-uniform weights, zero biases
        std::vector<float> h((size_t)o.P, 0.0f);
        const double a1 = sqrt(6.0 / d), a2 = sqrt(6.0 / H1);
        for (int p = 0; p < o.b1; ++p)
            h[p] = (float)(a1 * (2.0 * ((hash4(seed ^ kTagWeights, 1, (uint64_t)p, 0) >> 11) * (1.0 / 9007199254740992.0)) - 1.0));
        for (int p = o.W2; p < o.b2; ++p)
            h[p] = (float)(a2 * (2.0 * ((hash4(seed ^ kTagWeights, 2, (uint64_t)p, 0) >> 11) * (1.0 / 9007199254740992.0)) - 1.0));
        if (hipMemcpy(e->params, h.data(), (size_t)o.P * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(e->mom, 0, (size_t)o.P * 4) != hipSuccess || hipMemset(e->vel, 0, (size_t)o.P * 4) != hipSuccess) {
            (void)hipGetLastError();
            knn_encoder_destroy(e);
            return fail(KNN_EDEVICE, "encoder initialisation failed");
        }
        *enc = e;
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" void knn_encoder_destroy(knn_encoder* enc)
{
    if (!enc) return;
    if (enc->params) (void)hipFree(enc->params);
    if (enc->mom) (void)hipFree(enc->mom);
    if (enc->vel) (void)hipFree(enc->vel);
    delete enc;
}

extern "C" knn_status knn_encoder_set_weights(knn_encoder* enc, const float* W1, const float* b1,
                                              const float* W2, const float* b2)
{
    if (!enc || !W1 || !b1 || !W2 || !b2) return fail(KNN_EINVAL, "null argument");
    const Off o(enc->d);
    KNN_HIP(hipMemcpy(enc->params + o.W1, W1, (size_t)enc->d * H1 * 4, hipMemcpyHostToDevice));
    KNN_HIP(hipMemcpy(enc->params + o.b1, b1, (size_t)H1 * 4, hipMemcpyHostToDevice));
    KNN_HIP(hipMemcpy(enc->params + o.W2, W2, (size_t)H1 * H2 * 4, hipMemcpyHostToDevice));
    KNN_HIP(hipMemcpy(enc->params + o.b2, b2, (size_t)H2 * 4, hipMemcpyHostToDevice));
    KNN_HIP(hipMemset(enc->mom, 0, (size_t)o.P * 4));
    KNN_HIP(hipMemset(enc->vel, 0, (size_t)o.P * 4));
    enc->t = 0;
    return KNN_OK;
}

extern "C" knn_status knn_encoder_get_weights(const knn_encoder* enc, float* W1, float* b1, float* W2, float* b2)
{
    if (!enc || !W1 || !b1 || !W2 || !b2) return fail(KNN_EINVAL, "null argument");
    const Off o(enc->d);
    KNN_HIP(hipMemcpy(W1, enc->params + o.W1, (size_t)enc->d * H1 * 4, hipMemcpyDeviceToHost));
    KNN_HIP(hipMemcpy(b1, enc->params + o.b1, (size_t)H1 * 4, hipMemcpyDeviceToHost));
    KNN_HIP(hipMemcpy(W2, enc->params + o.W2, (size_t)H1 * H2 * 4, hipMemcpyDeviceToHost));
    KNN_HIP(hipMemcpy(b2, enc->params + o.b2, (size_t)H2 * 4, hipMemcpyDeviceToHost));
    return KNN_OK;
}

extern "C" knn_status knn_encoder_embed(const knn_encoder* enc, knn_matrix X, int32_t precision, float* Z,
                                        void* stream)
{
    try {
        if (!enc || !Z) return fail(KNN_EINVAL, "null argument");
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if (X.d != enc->d) return fail(KNN_EINVAL, "X.d != encoder input width");
        if (precision != KNN_PREC_FP32 && precision != KNN_PREC_BF16) return fail(KNN_EINVAL, "unknown precision");
        hipStream_t st = (hipStream_t)stream;
        if ((r = forward_impl(enc, X, nullptr, X.n, precision, nullptr, Z, st)) != KNN_OK) return r;
        KNN_HIP(hipStreamSynchronize(st));
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status knn_encoder_grads(knn_encoder* enc, knn_matrix X, const int32_t* rows, int32_t B,
                                        float margin, int32_t precision, float* loss_out, float* grads,
                                        void* stream)
{
    try {
        if (!enc || !rows || !loss_out) return fail(KNN_EINVAL, "null argument");
        if (precision != KNN_PREC_FP32 && precision != KNN_PREC_BF16) return fail(KNN_EINVAL, "unknown precision");
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if (X.d != enc->d) return fail(KNN_EINVAL, "X.d != encoder input width");
        if (B < 1) return fail(KNN_EINVAL, "B must be >= 1");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        const int64_t m = 3 * (int64_t)B;
        const Off o(enc->d);
        float *H, *Z, *dZ, *dH, *lterm, *partial, *grad, *loss_dev;
        if ((r = ws.alloc(&H, (size_t)m * H1)) != KNN_OK) return r;
        if ((r = ws.alloc(&Z, (size_t)m * H2)) != KNN_OK) return r;
        if ((r = ws.alloc(&dZ, (size_t)m * H2)) != KNN_OK) return r;
        if ((r = ws.alloc(&dH, (size_t)m * H1)) != KNN_OK) return r;
        if ((r = ws.alloc(&lterm, (size_t)B)) != KNN_OK) return r;
        if ((r = ws.alloc(&partial, (size_t)ceil_div(m, kGradChunk) * o.P)) != KNN_OK) return r;
        grad = grads;
        if (!grad && (r = ws.alloc(&grad, (size_t)o.P)) != KNN_OK) return r;
        if ((r = ws.alloc(&loss_dev, 1)) != KNN_OK) return r;
        r = batch_grads(enc, X, rows, B, margin, precision, H, Z, dZ, dH, lterm, partial, grad, loss_dev, st);
        if (r != KNN_OK) return r;
        KNN_HIP(hipMemcpyAsync(loss_out, loss_dev, 4, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipStreamSynchronize(st));
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" void knn_train_default_params(knn_train_params* t)
{
    if (!t) return;
    t->steps = 2000;
    t->batch = 4096;
    t->lr = 1e-3f;
    t->beta1 = 0.9f;
    t->beta2 = 0.999f;
    t->eps = 1e-8f;
    t->margin = 1.0f;
    t->seed = 0;
    t->precision = KNN_PREC_FP32;
}

extern "C" knn_status knn_encoder_train(knn_encoder* enc, knn_matrix X, const int32_t* knn_idx, int32_t k,
                                        const knn_train_params* tp, float* loss_log, void* stream)
{
    try {
        if (!enc || !knn_idx || !tp) return fail(KNN_EINVAL, "null argument");
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if (X.d != enc->d) return fail(KNN_EINVAL, "X.d != encoder input width");
        if (k < 1 || tp->steps < 0 || tp->batch < 1) return fail(KNN_EINVAL, "bad training parameters");
        if (tp->precision != KNN_PREC_FP32 && tp->precision != KNN_PREC_BF16)
            return fail(KNN_EINVAL, "unknown precision");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        const int B = tp->batch;
        const int64_t m = 3 * (int64_t)B;
        const Off o(enc->d);
        int32_t* rows;
        float *H, *Z, *dZ, *dH, *lterm, *partial, *grad, *losses;
        if ((r = ws.alloc(&rows, (size_t)m)) != KNN_OK) return r;
        if ((r = ws.alloc(&H, (size_t)m * H1)) != KNN_OK) return r;
        if ((r = ws.alloc(&Z, (size_t)m * H2)) != KNN_OK) return r;
        if ((r = ws.alloc(&dZ, (size_t)m * H2)) != KNN_OK) return r;
        if ((r = ws.alloc(&dH, (size_t)m * H1)) != KNN_OK) return r;
        if ((r = ws.alloc(&lterm, (size_t)B)) != KNN_OK) return r;
        if ((r = ws.alloc(&partial, (size_t)ceil_div(m, kGradChunk) * o.P)) != KNN_OK) return r;
        if ((r = ws.alloc(&grad, (size_t)o.P)) != KNN_OK) return r;
        if ((r = ws.alloc(&losses, (size_t)(tp->steps > 0 ? tp->steps : 1))) != KNN_OK) return r;
        for (int s = 0; s < tp->steps; ++s) {
            triplet_sample_kernel<<<(unsigned)ceil_div(B, 256), 256, 0, st>>>(X.n, knn_idx, k, B, tp->seed,
                                                                              enc->t + s, rows);
            r = batch_grads(enc, X, rows, B, tp->margin, tp->precision, H, Z, dZ, dH, lterm, partial, grad,
                            losses + s, st);
            if (r != KNN_OK) return r;
            if ((r = adam_apply(enc, grad, *tp, enc->t + s + 1, st)) != KNN_OK) return r;
        }
        enc->t += tp->steps;
        if (loss_log && tp->steps > 0)
            KNN_HIP(hipMemcpyAsync(loss_log, losses, (size_t)tp->steps * 4, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipStreamSynchronize(st));
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status knn_encoder_triplets(int64_t n, const int32_t* knn_idx, int32_t k, int32_t B,
                                           uint64_t seed, int32_t step, int32_t* rows, void* stream)
{
    try {
        if (!knn_idx || !rows) return fail(KNN_EINVAL, "null argument");
        if (n < 1 || n >= (int64_t)0x7FFFFFFF || k < 1 || B < 1 || step < 0)
            return fail(KNN_EINVAL, "bad triplet arguments");
        hipStream_t st = (hipStream_t)stream;
        triplet_sample_kernel<<<(unsigned)ceil_div(B, 256), 256, 0, st>>>(n, knn_idx, k, B, seed, step, rows);
        KNN_HIP(hipGetLastError());
        KNN_HIP(hipStreamSynchronize(st));
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status knn_encoder_step(knn_encoder* enc, knn_matrix X, const int32_t* rows, int32_t B,
                                       const knn_train_params* tp, float* loss_out, void* stream)
{
    try {
        if (!enc || !rows || !tp) return fail(KNN_EINVAL, "null argument");
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if (X.d != enc->d) return fail(KNN_EINVAL, "X.d != encoder input width");
        if (B < 1) return fail(KNN_EINVAL, "B must be >= 1");
        if (tp->precision != KNN_PREC_FP32 && tp->precision != KNN_PREC_BF16)
            return fail(KNN_EINVAL, "unknown precision");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        const int64_t m = 3 * (int64_t)B;
        const Off o(enc->d);
        float *H, *Z, *dZ, *dH, *lterm, *partial, *grad, *loss_dev;
        if ((r = ws.alloc(&H, (size_t)m * H1)) != KNN_OK) return r;
        if ((r = ws.alloc(&Z, (size_t)m * H2)) != KNN_OK) return r;
        if ((r = ws.alloc(&dZ, (size_t)m * H2)) != KNN_OK) return r;
        if ((r = ws.alloc(&dH, (size_t)m * H1)) != KNN_OK) return r;
        if ((r = ws.alloc(&lterm, (size_t)B)) != KNN_OK) return r;
        if ((r = ws.alloc(&partial, (size_t)ceil_div(m, kGradChunk) * o.P)) != KNN_OK) return r;
        if ((r = ws.alloc(&grad, (size_t)o.P)) != KNN_OK) return r;
        if ((r = ws.alloc(&loss_dev, 1)) != KNN_OK) return r;
        r = batch_grads(enc, X, rows, B, tp->margin, tp->precision, H, Z, dZ, dH, lterm, partial, grad, loss_dev, st);
        if (r != KNN_OK) return r;
        if ((r = adam_apply(enc, grad, *tp, enc->t + 1, st)) != KNN_OK) return r;
        enc->t += 1;
        if (loss_out) KNN_HIP(hipMemcpyAsync(loss_out, loss_dev, 4, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipStreamSynchronize(st));
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status knn_encoder_get_adam(const knn_encoder* enc, float* m, float* v, int32_t* t)
{
    if (!enc || !m || !v || !t) return fail(KNN_EINVAL, "null argument");
    KNN_HIP(hipMemcpy(m, enc->mom, (size_t)enc->P * 4, hipMemcpyDeviceToHost));
    KNN_HIP(hipMemcpy(v, enc->vel, (size_t)enc->P * 4, hipMemcpyDeviceToHost));
    *t = enc->t;
    return KNN_OK;
}

extern "C" knn_status knn_proj_seed(knn_matrix X, const float* Z, int32_t m, const float* dirs, int32_t P,
                                    int32_t D, int32_t w, int32_t K, int32_t* out_idx, float* out_dist,
                                    void* stream)
{
    try {
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if (!Z || !dirs || !out_idx || !out_dist) return fail(KNN_EINVAL, "null argument");
        if (X.n < 2 || m < 1 || m > 64 || P < 1 || w < 1 || K < 1 || K > 64)
            return fail(KNN_EINVAL, "bad sizes (need n >= 2, 1 <= m <= 64, P >= 1, w >= 1, 1 <= K <= 64)");
        if (D < 1 || D > 8 || 32 % D) return fail(KNN_EINVAL, "D must be 1, 2, 4 or 8");
        if (2 * w * P > 64) return fail(KNN_EINVAL, "2 * w * P must be <= 64");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        r = proj_seed_impl(X, Z, m, dirs, P, D, w, K, out_idx, out_dist, ws, st);
        if (r != KNN_OK) return r;
        KNN_HIP(hipStreamSynchronize(st));
        return KNN_OK;
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}
