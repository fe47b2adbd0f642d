// Exact k nearest neighbours: tiled MFMA distance GEMM + fused top-k'.
//
// The paper ranks its quality metrics by exact pairwise Euclidean distances
// computed by chunked matrix multiplication, with the norm expansion
// |a - b|^2 = |a|^2 + |b|^2 - 2 a.b of its k-NN section.  Here:
//
//  1. stage: inputs are copied into a zero-padded, 128-byte-aligned layout
//     (FP32, or BF16 rounded to nearest even), with FP32 row norms of the
//     staged values and the largest reference norm;
//  2. tile: each workgroup owns 128 query rows and streams 128-row reference
//     tiles through LDS; MFMA (32x32x2 FP32, or 32x32x16 BF16 with FP32
//     accumulation) produces dot products, the epilogue forms squared
//     distances and keeps, per query row, the best k' candidates in
//     registers with wave-wide bitonic merges (threshold-gated, so merges
//     are rare once lists fill).  The reference set can be split across
//     workgroups to fill the chip; each split keeps its own lists;
//  3. merge + re-rank: the splits' lists are merged, the best k' by GEMM
//     distance are re-ranked with FP32 direct differences on the original
//     input values, and the best k kept.  In FP32 precision a row is
//     certified when its k-th re-ranked distance is below the k'-th GEMM
//     distance minus the worst-case GEMM error bound; other rows are
//  4. recomputed exhaustively with direct differences.
#include <algorithm>
#include <mutex>

#include "knn_common.hpp"

namespace knn {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTileRows = 128;    // queries per workgroup and references per tile
constexpr int kListW = 32;        // list width per query row (k' <= 32)

// ------------------------------------------------------------------ stage

// Waves take groups of 4 rows grid-stride: padded copy (zeros beyond d) and
// the squared norm of the stored values: FP64 sums rounded once to FP32
// (within u of the exact norm), or with `aux` FP32 sums (the norms
// NNDescent's distances use).  maxnorm (nullable) receives the
// largest norm's float bits: one atomic per block after an in-block
// reduction.  With `aux`, the last 8 bytes of each row hold two FP32 words
// instead of zeros: the norm and +inf (a per-row value that NNDescent keeps
// current).
template <int DT, int OUT>
__global__ __launch_bounds__(256) void stage_kernel(const void* __restrict__ X, int64_t n, int d,
                                                    int64_t ld, void* __restrict__ Xs, int ldp,
                                                    float* __restrict__ norms,
                                                    unsigned* __restrict__ maxnorm,
                                                    const uint32_t* __restrict__ rowmap, int aux)
{
    constexpr int RB = 4;   // rows per wave and step: their loads are issued together
    __shared__ unsigned smax[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr bool HALF = OUT != KNN_F32;   // 2-byte staged elements
    const int lim = aux ? ldp - (HALF ? 4 : 2) : ldp;
    unsigned wmax = 0;
    for (int64_t row0 = ((int64_t)blockIdx.x * 4 + wv) * RB; row0 < n; row0 += (int64_t)gridDim.x * 4 * RB) {
        int64_t src[RB];
        float s[RB];
        double sd[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int64_t row = row0 + q < n ? row0 + q : row0;
            src[q] = rowmap ? (int64_t)rowmap[row] : row;
            s[q] = 0.0f;
            sd[q] = 0.0;
        }
        for (int t = lane; t < lim; t += 64) {
            float v[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) v[q] = t < d ? elem<DT>::ld(X, src[q] * ld + t) : 0.0f;
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                if (row0 + q >= n) continue;
                const int64_t row = row0 + q;
                float x = v[q];
                if constexpr (OUT == KNN_BF16) {
                    uint16_t b = f32_to_bf16_rne(x);
                    ((uint16_t*)Xs)[row * ldp + t] = b;
                    x = __uint_as_float((uint32_t)b << 16);
                } else if constexpr (OUT == KNN_F16) {
                    const _Float16 hv = (_Float16)x;   // round to nearest even
                    ((_Float16*)Xs)[row * ldp + t] = hv;
                    x = (float)hv;
                } else {
                    ((float*)Xs)[row * ldp + t] = x;
                }
                if (aux)
                    s[q] = fmaf(x, x, s[q]);
                else
                    sd[q] = fma((double)x, (double)x, sd[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            if (aux) {
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) s[q] += xor_f32(s[q], o);
            } else {
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const uint64_t b = (uint64_t)__double_as_longlong(sd[q]);
                    const uint64_t y = ((uint64_t)xor_u32((uint32_t)(b >> 32), o) << 32) | xor_u32((uint32_t)b, o);
                    sd[q] += __longlong_as_double((long long)y);
                }
                s[q] = (float)sd[q];
            }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int64_t row = row0 + q;
            if (row >= n) break;
            if (lane == 0) {
                norms[row] = s[q];
                if (aux) {
                    float* a = (float*)((char*)Xs + (row + 1) * (int64_t)ldp * (HALF ? 2 : 4)) - 2;
                    a[0] = s[q];
                    a[1] = __builtin_inff();
                }
            }
            const unsigned u = __float_as_uint(s[q]);
            wmax = u > wmax ? u : wmax;
        }
    }
    if (maxnorm) {
        if (lane == 0) smax[wv] = wmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned m = smax[0];
            for (int w = 1; w < 4; ++w) m = smax[w] > m ? smax[w] : m;
            atomicMax(maxnorm, m);
        }
    }
}

// ------------------------------------------------------------------ tile

// Tile geometry per staged element kind (KNN_F32, KNN_BF16, KNN_F16).
template <int OUT>
struct TileCfg {
    using E = float;
    static constexpr int KC = 32;    // elements per K chunk (128 bytes per row)
    static constexpr int LROW = 36;  // LDS row stride in elements (144 bytes)
    static constexpr int AMAX = 64;  // query rows stay in LDS when ldp <= AMAX
    static constexpr int AROW = 68;  // their LDS row stride
};
template <>
struct TileCfg<KNN_BF16> {
    using E = uint16_t;
    static constexpr int KC = 64;
    static constexpr int LROW = 72;
    static constexpr int AMAX = 64;
    static constexpr int AROW = 72;
};
template <>
struct TileCfg<KNN_F16> : TileCfg<KNN_BF16> {};

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Output D of a 32x32 MFMA: lane l, accumulator v holds row
// 8*(v/4) + 4*(l/32) + v%4 and column l%32 of the 32x32 block.
__device__ inline int mfma_row(int v, int half) { return 8 * (v >> 2) + 4 * half + (v & 3); }

// Adds the keys of the lanes in `m` (lanes 0..31 for the list held by lanes
// 0..31, lanes 32..63 for the one held by lanes 32..63) to the two sorted
// 32-key lists, keeping each list's 32 smallest.  A few keys are inserted one
// at a time per half: lanes whose entry exceeds the key move up one place and
// the first of them takes the key.  Many keys are sorted and merged by
// bitonic networks.  Both routes give the same list.
__device__ inline uint64_t list_add(uint64_t list, uint64_t key, uint64_t m, int lane)
{
    uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
    if (__builtin_popcount(m0) > 3 || __builtin_popcount(m1) > 3) {
        const uint64_t ck = seg_sort<32>(key);
        return seg_merge_sorted<32>(list, ck);
    }
    const bool hi = lane >= 32;
    const int from = (lane & 31) == 0 ? lane : lane - 1;
    while (m0 | m1) {
        const uint64_t x0 = m0 ? bcast_u64(key, __builtin_ctz(m0)) : kEmptyCand;
        const uint64_t x1 = m1 ? bcast_u64(key, 32 + __builtin_ctz(m1)) : kEmptyCand;
        const uint64_t x = hi ? x1 : x0;
        const bool gt = list > x;
        const uint64_t gm = ballot(gt);
        // the lane below (inside the same half) also moves up
        const bool pgt = (lane & 31) != 0 && ((gm >> ((lane - 1) & 63)) & 1ull);
        const uint64_t prev = shfl_u64(list, from);
        list = gt ? (pgt ? prev : x) : list;
        m0 &= m0 - 1u;
        m1 &= m1 - 1u;
    }
    return list;
}

// Rows of one pipeline step, loaded into registers: this thread's four
// 16-byte pieces of reference row r (and of query row r when the query rows
// stream) for chunk k0, and the reference norm of tile row tid at a tile's
// first chunk.
template <typename E, bool ARES>
__device__ inline void load_step(const E* Qe, const E* Re, int64_t qrow, int64_t rt, int64_t rend, int r,
                                 int col, int k0, int ldp, const float* rn, int tid, uint4& b0, uint4& b1,
                                 uint4& b2, uint4& b3, uint4& a0, uint4& a1, uint4& a2, uint4& a3, float& rnv)
{
    const int64_t rr = rt + r < rend ? rt + r : rend - 1;
    const uint4* rsrc = (const uint4*)(Re + rr * ldp + k0 + col);
    b0 = rsrc[0];
    b1 = rsrc[1];
    b2 = rsrc[2];
    b3 = rsrc[3];
    if (!ARES) {
        const uint4* qsrc = (const uint4*)(Qe + qrow * ldp + k0 + col);
        a0 = qsrc[0];
        a1 = qsrc[1];
        a2 = qsrc[2];
        a3 = qsrc[3];
    }
    rnv = 0.0f;
    if (k0 == 0 && tid < kTileRows && rt + tid < rend) rnv = rn[rt + tid];
}

// All K chunks of reference tile rt (rows rt .. rt + 127, clamped to rend)
// against the workgroup's 128 query rows: wave w's four 32x32 accumulators
// (query rows 32w + .., reference columns 32b + ..) are returned in acc.
// Each step stores the registers loaded by the previous one into LDS and
// issues the loads of the next step (the next tile's first chunk after the
// last chunk), so the loads of a step overlap the MFMAs of the one before.
// With ARES the query rows are already in As (row stride AROW).
template <int OUT, bool ARES>
__device__ __attribute__((always_inline)) inline void tile_gemm(
    uint4& nb0, uint4& nb1, uint4& nb2, uint4& nb3, uint4& na0, uint4& na1, uint4& na2, uint4& na3, float& nrn,
    f32x16 (&acc)[4], typename TileCfg<OUT>::E* As, typename TileCfg<OUT>::E* Bs, float* srn,
    const typename TileCfg<OUT>::E* Qe, const typename TileCfg<OUT>::E* Re, int64_t qrow, int64_t rt,
    int64_t rend, int ldp, const float* rn, int tid, int w, int h, int c)
{
    using C = TileCfg<OUT>;
    using E = typename C::E;
    constexpr int KC = C::KC, LROW = C::LROW, PER = KC / 2;
    constexpr int AROW = ARES ? C::AROW : LROW;
    constexpr int NV = PER * (int)sizeof(E) / 16;   // 16-byte loads per thread and chunk
    static_assert(NV == 4, "four 16-byte pieces per thread and chunk");
    const int r = tid >> 1, ph = tid & 1;              // staging: row r, half ph of the chunk
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;

    for (int k0 = 0; k0 < ldp; k0 += KC) {
        __syncthreads();   // the previous step's LDS reads are done
        {
            uint4* bdst = (uint4*)(Bs + r * LROW + ph * PER);
            bdst[0] = nb0;
            bdst[1] = nb1;
            bdst[2] = nb2;
            bdst[3] = nb3;
            if (!ARES) {
                uint4* adst = (uint4*)(As + r * LROW + ph * PER);
                adst[0] = na0;
                adst[1] = na1;
                adst[2] = na2;
                adst[3] = na3;
            }
            if (k0 == 0 && tid < kTileRows) srn[tid] = nrn;
        }
        __syncthreads();
        // the next step's rows are in flight during this step's arithmetic
        {
            const bool last = k0 + KC >= ldp;
            load_step<E, ARES>(Qe, Re, qrow, last ? rt + kTileRows : rt, rend, r, ph * PER, last ? 0 : k0 + KC,
                               ldp, rn, tid, nb0, nb1, nb2, nb3, na0, na1, na2, na3, nrn);
        }
        // K permutation: half h of the wave supplies chunk columns
        // h*PER .. h*PER+PER-1, the same for A and B, so every column
        // enters the dot product exactly once.
        const uint4* ap = (const uint4*)(As + (w * 32 + c) * AROW + (ARES ? k0 : 0) + h * PER);
        uint4 a4[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) a4[i] = ap[i];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint4* bp = (const uint4*)(Bs + (b * 32 + c) * LROW + h * PER);
            uint4 b4[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) b4[i] = bp[i];
            if constexpr (OUT == KNN_BF16) {
#pragma unroll
                for (int i = 0; i < NV; ++i) {
                    bf16x8 av = __builtin_bit_cast(bf16x8, a4[i]);
                    bf16x8 bv = __builtin_bit_cast(bf16x8, b4[i]);
                    acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[b], 0, 0, 0);
                }
            } else if constexpr (OUT == KNN_F16) {
#pragma unroll
                for (int i = 0; i < NV; ++i) {
                    f16x8 av = __builtin_bit_cast(f16x8, a4[i]);
                    f16x8 bv = __builtin_bit_cast(f16x8, b4[i]);
                    acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, acc[b], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int i = 0; i < NV; ++i) {
                    f32x4 av = __builtin_bit_cast(f32x4, a4[i]);
                    f32x4 bv = __builtin_bit_cast(f32x4, b4[i]);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[e], bv[e], acc[b], 0, 0, 0);
                }
            }
        }
    }
}

// One workgroup (4 waves) owns 128 query rows and streams the reference
// rows [rbeg, rend) of its split in 128-row tiles, K chunk by K chunk.  The
// sequence of (tile, chunk) steps is software-pipelined: the global loads of
// step t+1 are issued into registers before step t's MFMAs and epilogue run
// and are written to LDS at the top of step t+1, so HBM/L2 latency overlaps
// the arithmetic.  With ARES (row length ldp <= AMAX) the query rows are
// loaded into LDS once and only reference rows stream.  Wave w computes
// query rows 32w..32w+31 against the tile's 128 references (four 32x32
// MFMA blocks).
template <int OUT, bool ARES>
__global__ __launch_bounds__(256, 2) void exact_tile_kernel(
    const void* __restrict__ Qs, const float* __restrict__ qn, int64_t nq,
    const void* __restrict__ Rs, const float* __restrict__ rn, int64_t nr, int ldp,
    const int32_t* __restrict__ q_self, int self_mode, int64_t self_base, int kp, int64_t split_len, int S,
    const unsigned* __restrict__ rmax_bits, uint64_t* __restrict__ part)
{
    using C = TileCfg<OUT>;
    using E = typename C::E;
    constexpr int KC = C::KC, LROW = C::LROW, PER = KC / 2;
    constexpr int AROW = ARES ? C::AROW : LROW;
    constexpr int NV = PER * (int)sizeof(E) / 16;   // 16-byte loads per thread and chunk
    __shared__ __attribute__((aligned(16))) E As[kTileRows * AROW];
    __shared__ __attribute__((aligned(16))) E Bs[kTileRows * LROW];
    __shared__ float srn[kTileRows];
    __shared__ float sqn[kTileRows];
    __shared__ int32_t sself[kTileRows];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, h = lane >> 5, c = lane & 31;
    const int64_t q0 = (int64_t)blockIdx.x * kTileRows;
    const int s = blockIdx.y;
    const int64_t rbeg = (int64_t)s * split_len;
    const int64_t rend = rbeg + split_len < nr ? rbeg + split_len : nr;

    if (tid < kTileRows) {
        const int64_t qr = q0 + tid;
        sqn[tid] = qr < nq ? qn[qr] : 0.0f;
        sself[tid] = qr >= nq ? -1 : (self_mode == 1 ? (int32_t)(self_base + qr) : (self_mode == 2 ? q_self[qr] : -1));
    }
    // Per-row lists of this lane's 16 accumulator rows and their gates.
    // A candidate enters a list when d2 = |q|^2 + |r|^2 - 2 q.r <= thr (the
    // list's k'-th distance).  The gate tests the equivalent
    // q.r - |r|^2/2 >= (|q|^2 - thr)/2 with two operations per element;
    // lim is lowered by a slack that covers the FP32 rounding of both forms
    // (8u (|q|^2 + thr + max|r|^2)), so every candidate the exact test
    // accepts passes the gate, and the exact test decides.  Rows past nq
    // get lim = +inf and never pass.
    const float rmax = __uint_as_float(*rmax_bits);
    uint64_t list[16];
    float lim[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        list[v] = kEmptyList;
        lim[v] = q0 + w * 32 + mfma_row(v, h) < nq ? -__builtin_inff() : __builtin_inff();
    }

    const E* Qe = (const E*)Qs;
    const E* Re = (const E*)Rs;
    const int r = tid >> 1, ph = tid & 1;              // staging: row r, half ph of the chunk
    const int64_t qrow = q0 + r < nq ? q0 + r : nq - 1;
    if (ARES) {
        // whole query rows (ldp <= AMAX elements) into LDS once
        const uint4* src = (const uint4*)(Qe + qrow * ldp + ph * (ldp / 2));
        uint4* dst = (uint4*)(As + r * AROW + ph * (ldp / 2));
        const int nv = ldp / 2 * (int)sizeof(E) / 16;
        for (int i = 0; i < nv; ++i) dst[i] = src[i];
    }

    // prologue: the first step's rows (addresses are clamped to valid rows,
    // so a load past the split's end is harmless)
    static_assert(NV == 4, "four 16-byte pieces per thread and chunk");
    uint4 nb0, nb1, nb2, nb3, na0 = {}, na1 = {}, na2 = {}, na3 = {};
    float nrn;
    load_step<E, ARES>(Qe, Re, qrow, rbeg, rend, r, ph * PER, 0, ldp, rn, tid, nb0, nb1, nb2, nb3, na0, na1,
                       na2, na3, nrn);
    for (int64_t rt = rbeg; rt < rend; rt += kTileRows) {
        f32x16 acc[4];
        tile_gemm<OUT, ARES>(nb0, nb1, nb2, nb3, na0, na1, na2, na3, nrn, acc, As, Bs, srn, Qe, Re, qrow, rt, rend,
                            ldp, rn, tid, w, h, c);

        // epilogue: distances, threshold gate, list updates
        for (int blk = 0; blk < 4; ++blk) {
            const f32x16 cur = blk == 0 ? acc[0] : (blk == 1 ? acc[1] : (blk == 2 ? acc[2] : acc[3]));
            const float rnj = srn[blk * 32 + c];
            const float hr = 0.5f * rnj;
            // gate all 16 rows first: one branch per block when nothing passes
            uint64_t gm[16], any = 0;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                gm[v] = ballot(cur[v] - hr >= lim[v]);
                any |= gm[v];
            }
            if (!any) continue;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                if (gm[v]) {
                    // exact test; the list's current k'-th distance is the threshold
                    const int lr = w * 32 + mfma_row(v, h);
                    const float sq = sqn[lr];
                    const int64_t j = rt + blk * 32 + c;
                    const uint64_t t0 = bcast_u64(list[v], kp - 1), t1 = bcast_u64(list[v], 32 + kp - 1);
                    const float thr = key_d2(h ? t1 : t0);
                    float d2 = fmaf(-2.0f, cur[v], sq + rnj);
                    d2 = d2 > 0.0f ? d2 : 0.0f;
                    const bool ok = j < rend && (int32_t)j != sself[lr] && d2 <= thr && lim[v] < __builtin_inff();
                    const uint64_t okm = ballot(ok);
                    if (okm) {
                        const uint64_t ck = ok ? make_key(d2, (uint32_t)j) : kEmptyCand;
                        list[v] = list_add(list[v], ck, okm, lane);
                        const uint64_t u0 = bcast_u64(list[v], kp - 1), u1 = bcast_u64(list[v], 32 + kp - 1);
                        const float t = key_d2(h ? u1 : u0);
                        const float nl = 0.5f * (sq - t) - 4.76837158e-07f * (sq + t + rmax);   // 8u = 2^-21
                        lim[v] = lim[v] < __builtin_inff() ? nl : lim[v];
                    }
                }
            }
        }
    }

#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int64_t row = q0 + w * 32 + mfma_row(v, h);
        if (row < nq) part[(row * S + s) * kListW + c] = list[v];
    }
}

// ------------------------------------------------------------ rank counts

constexpr int kRankP = 16;   // probes per query row (the quality metrics' k <= 16)
constexpr int kRankM = 16;   // queued pairs per thread in one pass over a tile's rows
// For every query row q and each of its probes (keys (canonical d2, index),
// ascending; kEmptyCand pads), counts[q][p] = the number of reference rows
// m != self(q) whose key (canonical FP32 d2(q, m), m) is below the probe's
// key: the probe's rank minus one.  The same tiles and pipeline as
// exact_tile_kernel (FP32 MFMA Gram, norm expansion, S reference splits
// whose counts are added into counts, zeroed beforehand; query rows
// streamed); the epilogue puts each reference row that can be below a
// probe of its query into a per-row histogram over the probe boundaries (in
// LDS), so counts are prefix sums.  A GEMM distance within the slack of a
// probe's distance (the GEMM error bound for the pair's own norms plus the
// canonical distance's) is undecided: the pair is queued in the
// workgroup's global queue (room for a whole tile, 128 x 128 pairs) and,
// after the tile's epilogue, the tile's query and reference rows are
// streamed again through the tile buffers in 32-coordinate chunks; 16-lane
// groups sum the queued pairs' canonical FP32 distances from LDS (lane g:
// coordinates g, g + 16, ... in order, then the fixed 16-lane tree, the sums
// dist_g16 makes) and put them into the histogram.  No pair is decided any
// other way.  With LISTS the pass also keeps, per query row and split, the
// kp smallest GEMM keys (GEMM distance, index) as exact_tile_kernel does,
// and writes them to part in its split-list layout (row-major over query
// rows, then splits, kListW keys each), for merge_rerank_kernel; without
// LISTS, kp and part are unused.
template <bool LISTS>
__global__ __launch_bounds__(256, 2) void rank_tile_kernel(
    const float* __restrict__ Qs, const float* __restrict__ qn, int64_t nq, const float* __restrict__ Rs,
    const float* __restrict__ rn, int64_t nr, int ldp, int d, int self_mode, int64_t self_base,
    const uint64_t* __restrict__ probes, const unsigned* __restrict__ rmax_bits, float ec_dot, float ec_norm,
    float edir, int S, int64_t split_len, uint32_t* __restrict__ counts, uint32_t* __restrict__ gqueue, int kp,
    uint64_t* __restrict__ part)
{
    using C = TileCfg<KNN_F32>;
    constexpr int LROW = C::LROW, KC = C::KC, PER = KC / 2;
    __shared__ __attribute__((aligned(16))) float ABs[2 * kTileRows * LROW];
    float* As = ABs;
    float* Bs = ABs + kTileRows * LROW;
    // this workgroup's undecided pairs of the current tile:
    // column in tile << 17 | query row << 10 | a << 5 | b
    uint32_t* queue = gqueue + (int64_t)blockIdx.x * (kTileRows * kTileRows);
    __shared__ float srn[kTileRows];
    __shared__ f32x4 srow[kTileRows];   // per query row: |q|^2, gate, excluded index (bits), |q|
    __shared__ float smx[kTileRows];
    __shared__ __attribute__((aligned(16))) uint64_t skey[kTileRows * kRankP];
    __shared__ __attribute__((aligned(16))) float sthr[kTileRows * kRankP];   // the probes' distances (+inf: none)
    __shared__ uint32_t hist[kTileRows * (kRankP + 1)];
    __shared__ uint32_t qcount;   // queue fill

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, h = lane >> 5, c = lane & 31;
    // workgroup = (query block, reference split): splits rbeg .. rend
    const int64_t q0 = (int64_t)(blockIdx.x / S) * kTileRows;
    const int64_t rbeg = (int64_t)(blockIdx.x % S) * split_len;
    const int64_t rend = rbeg + split_len < nr ? rbeg + split_len : nr;
    const float ra = sqrtf(__uint_as_float(*rmax_bits));
    for (int e = tid; e < kTileRows * kRankP; e += 256) {
        const int64_t qr = q0 + e / kRankP;
        const uint64_t key = qr < nq ? probes[qr * kRankP + e % kRankP] : kEmptyCand;
        skey[e] = key;
        sthr[e] = key == kEmptyCand ? __builtin_inff() : key_d2(key);
    }
    for (int e = tid; e < kTileRows * (kRankP + 1); e += 256) hist[e] = 0u;
    if (tid == 0) qcount = 0u;
    __syncthreads();
    if (tid < kTileRows) {
        const int64_t qr = q0 + tid;
        const float sq = qr < nq ? qn[qr] : 0.0f;
        const int32_t self = qr >= nq ? -1 : (self_mode == 1 ? (int32_t)(self_base + qr) : -1);
        float mx = -1.0f;
        for (int p = 0; p < kRankP; ++p) {
            const uint64_t key = skey[tid * kRankP + p];
            if (key != kEmptyCand) mx = key_d2(key);
        }
        const float qa = sqrtf(sq), E = ec_dot * qa * ra + ec_norm * (sq + ra * ra);
        const float sl = E + 2.0f * edir * (mx + E);
        smx[tid] = mx;
        // rows without probes never pass (the gate takes the largest reference norm)
        const f32x4 ri = {sq, mx < 0.0f ? -1.0f : mx + sl, __int_as_float(self), qa};
        srow[tid] = ri;
    }

    // With LISTS, the split's best kp keys (GEMM distance, index) of each
    // query row as well, kept as exact_tile_kernel keeps them (lane (h, c)
    // holds entry c of row 32 w + mfma_row(v, h)'s list) and written to part
    // in its layout: the same pass gives the rows' exact k-NN after the
    // merge, re-rank and certificate.  lthr is the list's kp-th distance
    // (-inf for rows past nq, which take nothing).
    uint64_t list[16];
    float lthr[16];
    if constexpr (LISTS) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            list[v] = kEmptyList;
            lthr[v] = q0 + w * 32 + mfma_row(v, h) < nq ? __builtin_inff() : -__builtin_inff();
        }
    }
    const float* Qe = Qs;
    const float* Re = Rs;
    const int r = tid >> 1, ph = tid & 1;
    const int64_t qrow = q0 + r < nq ? q0 + r : nq - 1;
    uint4 nb0, nb1, nb2, nb3, na0 = {}, na1 = {}, na2 = {}, na3 = {};
    float nrn;
    load_step<float, false>(Qe, Re, qrow, rbeg, rend, r, ph * PER, 0, ldp, rn, tid, nb0, nb1, nb2, nb3, na0, na1,
                            na2, na3, nrn);
    for (int64_t rt = rbeg; rt < rend; rt += kTileRows) {
        f32x16 acc[4];
        tile_gemm<KNN_F32, false>(nb0, nb1, nb2, nb3, na0, na1, na2, na3, nrn, acc, As, Bs, srn, Qe, Re, qrow, rt,
                                rend, ldp, rn, tid, w, h, c);
        // row and column bases, opaque to the compiler here so that the 64
        // (block, row) offsets derived from them are formed where they are
        // used instead of being held in registers across the whole loop
        int lr0 = w * 32 + 4 * h, c0 = c;
        asm volatile("" : "+v"(lr0), "+v"(c0));
        float rnj[4], raj[4];   // the lane's four reference columns: |r|^2, |r|
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            rnj[blk] = srn[blk * 32 + c0];
            raj[blk] = sqrtf(rnj[blk]);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int lr = lr0 + mfma_row(v, 0);
            const f32x4 ri = srow[lr];   // the row's |q|^2, gate, excluded index, |q|
#pragma unroll
            for (int blk = 0; blk < 4; ++blk) {
                const int col = blk * 32 + c0;
                const int64_t j = rt + col;
                float d2 = fmaf(-2.0f, acc[blk][v], ri[0] + rnj[blk]);
                d2 = d2 > 0.0f ? d2 : 0.0f;
                if constexpr (LISTS) {
                    const bool okl = d2 <= lthr[v] && j < rend && (int32_t)j != __float_as_int(ri[2]);
                    const uint64_t okm = ballot(okl);
                    if (okm) {
                        list[v] = list_add(list[v], okl ? make_key(d2, (uint32_t)j) : kEmptyCand, okm, lane);
                        const uint64_t t0 = bcast_u64(list[v], kp - 1), t1 = bcast_u64(list[v], 32 + kp - 1);
                        lthr[v] = key_d2(h ? t1 : t0);
                    }
                }
                const bool pass = d2 <= ri[1] && j < rend && (int32_t)j != __float_as_int(ri[2]);
                if (!ballot(pass)) continue;
                if (pass) {
                    // the slack of this pair: the GEMM bound with its own
                    // reference norm, plus the canonical distance's
                    const float E = ec_dot * ri[3] * raj[blk] + ec_norm * (ri[0] + rnj[blk]);
                    const float sl = E + 2.0f * edir * (smx[lr] + E);
                    const f32x4* pt = (const f32x4*)(sthr + lr * kRankP);
                    const float hi = d2 + sl, lo = d2 - sl;
                    int a = 0, b = 0;   // probes with thr <= d2 + sl, with thr < d2 - sl
#pragma unroll
                    for (int p4 = 0; p4 < kRankP / 4; ++p4) {
                        const f32x4 t4 = pt[p4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            a += t4[e] <= hi ? 1 : 0;
                            b += t4[e] < lo ? 1 : 0;
                        }
                    }
                    // probes a.. have this row below them; b..a-1 are undecided
                    if (b == a && a < kRankP) atomicAdd(&hist[lr * (kRankP + 1) + a], 1u);
                    if (b < a) {
                        const uint32_t slot = atomicAdd(&qcount, 1u);
                        queue[slot] = ((uint32_t)col << 17) | ((uint32_t)lr << 10) | ((uint32_t)a << 5) | (uint32_t)b;
                    }
                }
            }
        }
        __syncthreads();   // the queue is complete; every wave's MFMA operands are read
        const int nqd = (int)qcount;
        // thread (tid / 16, g = tid % 16) takes pairs base + tid / 16 + 16 m;
        // a thread past the end reads row 0 of both buffers and drops the sum
        const int g = tid & 15;
        for (int base = 0; base < nqd; base += 16 * kRankM) {
            uint32_t qo[kRankM], ro[kRankM];
            float dsum[kRankM];
#pragma unroll
            for (int m = 0; m < kRankM; ++m) {
                const int e = base + (tid >> 4) + 16 * m;
                const uint32_t ent = e < nqd ? queue[e] : 0u;
                qo[m] = ((ent >> 10) & 127u) * LROW + g;
                ro[m] = (ent >> 17) * LROW + g;
                dsum[m] = 0.0f;
            }
            // the chunks pass through registers: chunk k0 + KC is loaded
            // while chunk k0's sums are formed
            const int rr = tid >> 1, hh = tid & 1;
            const f32x4* qs = (const f32x4*)(Qs + (q0 + rr < nq ? q0 + rr : nq - 1) * ldp + hh * PER);
            const f32x4* rs = (const f32x4*)(Rs + (rt + rr < rend ? rt + rr : rend - 1) * ldp + hh * PER);
            f32x4 x0 = qs[0], x1 = qs[1], x2 = qs[2], x3 = qs[3];
            f32x4 y0 = rs[0], y1 = rs[1], y2 = rs[2], y3 = rs[3];
            for (int k0 = 0; k0 < d; k0 += KC) {
                __syncthreads();   // the previous chunk is read
                {
                    f32x4* qd = (f32x4*)(As + rr * LROW + hh * PER);
                    f32x4* rd = (f32x4*)(Bs + rr * LROW + hh * PER);
                    qd[0] = x0;
                    qd[1] = x1;
                    qd[2] = x2;
                    qd[3] = x3;
                    rd[0] = y0;
                    rd[1] = y1;
                    rd[2] = y2;
                    rd[3] = y3;
                }
                __syncthreads();
                {
                    // the last chunk loads itself again (in bounds, unused)
                    const int kn = (k0 + KC < d ? k0 + KC : k0) / 4;
                    x0 = qs[kn];
                    x1 = qs[kn + 1];
                    x2 = qs[kn + 2];
                    x3 = qs[kn + 3];
                    y0 = rs[kn];
                    y1 = rs[kn + 1];
                    y2 = rs[kn + 2];
                    y3 = rs[kn + 3];
                }
                // coordinates past d add nothing: fmaf(0, 0, s) == s
                const bool lo = k0 + g < d, hi = k0 + g + 16 < d;
#pragma unroll
                for (int m = 0; m < kRankM; ++m) {
                    const float d0 = As[qo[m]] - Bs[ro[m]], d1 = As[qo[m] + 16] - Bs[ro[m] + 16];
                    const float e0 = lo ? d0 : 0.0f, e1 = hi ? d1 : 0.0f;
                    dsum[m] = fmaf(e1, e1, fmaf(e0, e0, dsum[m]));
                }
                // the next chunk's loads belong to this step: issued before
                // the sums above, not moved to the top of the next step
                asm volatile("" : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3), "+v"(y0), "+v"(y1), "+v"(y2), "+v"(y3));
            }
#pragma unroll
            for (int m = 0; m < kRankM; ++m) {
                const float dc = wave_sum16(dsum[m]);
                const int e = base + (tid >> 4) + 16 * m;
                if (e < nqd && g == 0) {
                    const uint32_t ent = queue[e];
                    const int lr = (int)((ent >> 10) & 127u), a = (int)((ent >> 5) & 31u), b = (int)(ent & 31u);
                    const uint64_t km = make_key(dc, (uint32_t)(rt + (ent >> 17)));
                    const uint64_t* pk = skey + lr * kRankP;
                    int at = a;
                    for (int p = b; p < a; ++p) {
                        if (km < pk[p]) {
                            at = p;
                            break;
                        }
                    }
                    if (at < kRankP) atomicAdd(&hist[lr * (kRankP + 1) + at], 1u);
                }
            }
        }
        __syncthreads();   // the queue and the tile buffers are free for the next tile
        if (tid == 0) qcount = 0u;
    }
    if constexpr (LISTS) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t row = q0 + w * 32 + mfma_row(v, h);
            if (row < nq) part[(row * S + blockIdx.x % S) * kListW + c] = list[v];
        }
    }
    __syncthreads();
    for (int e = tid; e < kTileRows * kRankP; e += 256) {
        const int lr = e / kRankP, p = e % kRankP;
        const int64_t qr = q0 + lr;
        if (qr >= nq) continue;
        uint32_t cnt = 0;
        for (int a = 0; a <= p; ++a) cnt += hist[lr * (kRankP + 1) + a];
        atomicAdd(&counts[qr * kRankP + p], cnt);   // the splits' counts add up
    }
}

// Canonical FP32 squared distance for d <= DT <= 16 coordinates: the
// squares of coordinates t < d (t mod 16 = t), then the fixed tree at
// strides 8, 4, 2, 1 (terms known to be zero left out); every square and
// sum rounded, as dist_g16 rounds them.
template <int DT>
__device__ __attribute__((always_inline)) inline float direct_d2(const float (&xq)[DT], const float* xr, int d)
{
#pragma clang fp contract(off)
    float sq[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        if (t < DT) {
            const float e = xq[t] - xr[t];
            sq[t] = t < d ? e * e : 0.0f;
        }
    }
#pragma unroll
    for (int j = 8; j > 0; j >>= 1) {
#pragma unroll
        for (int g = 0; g < j; ++g) {
            if (g + j < DT) sq[g] = sq[g] + sq[g + j];
        }
    }
    return sq[0];
}

// The same counts for a low-dimensional space (d <= kRankDirectD, e.g. a 2-D
// embedding), by direct canonical FP32 distances: there the norm
// expansion's error bound is wider than neighbour distances, so a GEMM pass
// would recheck nearly every pair.  Thread = query row; its probe keys and
// counts sit in registers; the reference rows of the workgroup's split
// stream through LDS in tiles of 256, and the splits' counts are added into
// counts (zeroed beforehand).  Exact in the canonical precision, no
// ambiguity.
constexpr int kRankDirectD = 16;
// Workgroups per rank_tile_kernel launch: each holds a 64 KiB queue of
// undecided pairs (256 MiB per launch).
constexpr int64_t kRankBlocks = 4096;
constexpr int kRankMaxSplits = 8;   // reference splits of the rank pass

// DC = d when it is a compile-time constant (2, 3), 0 for any d <= 16.
template <int DC>
__global__ __launch_bounds__(256) void rank_direct_kernel(const float* __restrict__ Xs, int64_t n, int ldp, int dd,
                                                          const uint64_t* __restrict__ probes, int64_t split_len,
                                                          uint32_t* __restrict__ counts)
{
    const int d = DC ? DC : dd;
    constexpr int DT = DC ? DC : kRankDirectD;   // coordinates held per row
    __shared__ float tile[256][DT + 1];
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t rbeg = (int64_t)blockIdx.y * split_len, rend = rbeg + split_len < n ? rbeg + split_len : n;
    const bool live = q < n;
    float xq[DT];
#pragma unroll
    for (int t = 0; t < DT; ++t) xq[t] = live && t < d ? Xs[q * ldp + t] : 0.0f;
    uint64_t pk[kRankP];
    uint32_t cnt[kRankP];
    float mx = -1.0f;
#pragma unroll
    for (int p = 0; p < kRankP; ++p) {
        pk[p] = live ? probes[q * kRankP + p] : kEmptyCand;
        cnt[p] = 0u;
        if (pk[p] != kEmptyCand) mx = key_d2(pk[p]);
    }
    for (int64_t r0 = rbeg; r0 < rend; r0 += 256) {
        __syncthreads();
        {
            const int64_t r = r0 + threadIdx.x;
#pragma unroll
            for (int t = 0; t < DT; ++t) tile[threadIdx.x][t] = r < rend && t < d ? Xs[r * ldp + t] : 0.0f;
        }
        __syncthreads();
        const int nr = (int)(rend - r0 < 256 ? rend - r0 : 256);
        // 8 references at a time: their distances first (the tile reads
        // issued together), then the probe comparisons of those that can
        // be below a probe
        for (int j0 = 0; j0 < nr; j0 += 8) {
            float d2[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) d2[u] = direct_d2<DT>(xq, tile[j0 + u < nr ? j0 + u : j0], d);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t m = r0 + j0 + u;
                if (j0 + u < nr && d2[u] <= mx && m != q) {
                    const uint64_t km = make_key(d2[u], (uint32_t)m);
#pragma unroll
                    for (int p = 0; p < kRankP; ++p) cnt[p] += km < pk[p] ? 1u : 0u;
                }
            }
        }
    }
    if (live) {
#pragma unroll
        for (int p = 0; p < kRankP; ++p) atomicAdd(&counts[q * kRankP + p], cnt[p]);   // the splits' counts add up
    }
}

// Exact k-NN in a low-dimensional space (d <= kRankDirectD, e.g. a 2-D
// embedding): there the norm expansion's error bound exceeds neighbour
// distances, so GEMM certificates fail; instead every pair's canonical FP32
// distance is formed directly (thread = query row, reference rows through
// LDS, the canonical sum as in rank_direct_kernel) and each thread keeps
// its KM smallest keys (canonical d2, index) in registers.  Workgroup
// (query block, reference split) writes its sorted list, padded to kListW,
// in the split-list layout merge_rerank_kernel merges.
template <int DT, int DC, int KM>
__global__ __launch_bounds__(256) void exact_direct_kernel(
    const void* __restrict__ Q, int64_t ldq, int64_t nq, const void* __restrict__ R, int64_t ldr, int64_t nr,
    int dd, const int32_t* __restrict__ q_self, int self_mode, int64_t self_base, int k, int64_t split_len, int S,
    uint64_t* __restrict__ part)
{
    const int d = DC ? DC : dd;
    constexpr int DT_ = DC ? DC : kRankDirectD;
    __shared__ float tile[256][DT_ + 1];
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int64_t rbeg = (int64_t)s * split_len, rend = rbeg + split_len < nr ? rbeg + split_len : nr;
    const bool live = q < nq;
    const int64_t self = !live ? -1 : (self_mode == 1 ? self_base + q : (self_mode == 2 ? (int64_t)q_self[q] : -1));
    float xq[DT_];
#pragma unroll
    for (int t = 0; t < DT_; ++t) xq[t] = live && t < d ? elem<DT>::ld(Q, q * ldq + t) : 0.0f;
    uint64_t list[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) list[j] = kEmptyList;
    uint64_t kth = kEmptyList;   // list[k - 1]
    for (int64_t r0 = rbeg; r0 < rend; r0 += 256) {
        __syncthreads();
        {
            const int64_t r = r0 + threadIdx.x;
#pragma unroll
            for (int t = 0; t < DT_; ++t) tile[threadIdx.x][t] = r < rend && t < d ? elem<DT>::ld(R, r * ldr + t) : 0.0f;
        }
        __syncthreads();
        const int nt = (int)(rend - r0 < 256 ? rend - r0 : 256);
        // 32 references at a time: first the gate against the list's k-th key
        // as it stood (a bit per passing reference), then the passing ones
        // inserted in index order, each re-tested against the current k-th
        // key, so a wave runs as many insertion steps as its busiest lane
        for (int j0 = 0; j0 < nt; j0 += 32) {
            const int jn = nt - j0 < 32 ? nt - j0 : 32;
            uint32_t mask = 0u;
            for (int jj = 0; jj < jn; ++jj) {
                const int64_t m = r0 + j0 + jj;
                const uint64_t key = make_key(direct_d2<DT_>(xq, tile[j0 + jj], d), (uint32_t)m);
                mask |= (key < kth && m != self) ? 1u << jj : 0u;
            }
            while (mask) {
                const int jj = __builtin_ctz(mask);
                mask &= mask - 1u;
                const uint64_t key = make_key(direct_d2<DT_>(xq, tile[j0 + jj], d), (uint32_t)(r0 + j0 + jj));
                if (key < kth) {
                    // insertion into the ascending list; entries past k stay empty
#pragma unroll
                    for (int j = KM - 1; j >= 1; --j) {
                        const uint64_t a = list[j - 1], b = list[j];
                        list[j] = j < k ? (key < a ? a : (key < b ? key : b)) : b;
                    }
                    list[0] = key < list[0] ? key : list[0];
#pragma unroll
                    for (int j = 0; j < KM; ++j) kth = j == k - 1 ? list[j] : kth;
                }
            }
        }
    }
    if (live) {
        uint64_t* out = part + (q * S + s) * kListW;
#pragma unroll
        for (int c = 0; c < kListW; ++c) out[c] = c < KM ? list[c] : kEmptyList;
    }
}

// ------------------------------------------------------------ merge/rerank

// One wave per query row.  Merges the S split lists (S x 32 keys), keeps
// the best kp by GEMM distance, re-ranks them with the canonical FP32
// direct-difference distance on the original inputs and writes the best k.
template <int DT>
__global__ __launch_bounds__(256) void merge_rerank_kernel(
    const uint64_t* __restrict__ part, int S, int64_t nq, int kp, int k,
    const void* __restrict__ Q, int64_t ldq, const void* __restrict__ R, int64_t ldr, int d,
    const float* __restrict__ qn, const unsigned* __restrict__ rmax_bits, float err_coef,
    float edir, int certify, int out_kind, int32_t* __restrict__ out_idx,
    float* __restrict__ out_dist, int32_t* __restrict__ fb_rows, int* __restrict__ fb_count)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nq) return;
    // split lists (each sorted, 32 keys): even splits merge in lanes 0..31,
    // odd ones in lanes 32..63, keeping each half's 32 smallest; the two
    // halves then form one ascending 64-key sequence
    const int sp = lane >> 5;
    uint64_t acc = sp < S ? part[(row * S + sp) * kListW + (lane & 31)] : kEmptyCand;
    for (int b = 2; b < S; b += 2) {
        const uint64_t nk = b + sp < S ? part[(row * S + b + sp) * kListW + (lane & 31)] : kEmptyCand;
        acc = seg_merge_sorted<32>(acc, nk);
    }
    const uint64_t rv = shfl_xor_u64(acc, 31);
    const uint64_t k0 = seg_bitonic_merge<64>(sp ? rv : acc);
    const uint64_t ck = lane < kp ? k0 : kEmptyCand;
    const bool cvalid = lane < kp && key_valid(ck);
    const int nvalid = popc64(ballot(cvalid));
    const float T = key_d2(bcast_u64(k0, kp - 1));
    const uint32_t myidx = key_idx(ck);

    float dd = 0.0f;
    for (int base = 0; base < kp; base += 4) {
        const int ci = base + (lane >> 4);
        const uint32_t cj = shfl_u32(myidx, ci < 64 ? ci : 0);
        const bool act = ci < kp && cj != 0xFFFFFFFFu;
        const float v = dist_g16<DT>(Q, row * ldq, R, (int64_t)cj * ldr, d, act);
        const float got = shfl_f32(v, ((lane - base) & 3) * 16);
        if (lane >= base && lane < base + 4) dd = got;
    }
    uint64_t nk = cvalid ? make_key(dd, myidx) : kEmptyCand;
    nk = seg_sort<64>(nk);
    if (lane < k) {
        const float d2 = key_d2(nk);
        out_idx[row * k + lane] = (int32_t)key_idx(nk);
        out_dist[row * k + lane] = out_kind == KNN_OUT_L2 ? sqrtf(d2) : d2;
    }
    if (certify) {
        const float Dk = key_d2(bcast_u64(nk, k - 1));
        const float qa = sqrtf(qn[row]);
        const float ra = sqrtf(__uint_as_float(*rmax_bits));
        const float E = err_coef * (qa + ra) * (qa + ra);
        const bool cert = (nvalid < kp) || (Dk * (1.0f + edir) <= T - E);
        if (!cert && lane == 0) {
            int p = atomicAdd(fb_count, 1);
            fb_rows[p] = (int32_t)row;
        }
    }
}

// --------------------------------------------------------------- fallback

// Exhaustive direct-difference k-NN for the rows listed in fb_rows (one
// workgroup of 4 waves per row; each wave scans a quarter of the references
// 64 at a time and merges them into its list; the 4 lists are merged last).
template <int DT>
__global__ __launch_bounds__(256) void exact_fallback_kernel(
    const int32_t* __restrict__ fb_rows, const int* __restrict__ fb_count,
    const void* __restrict__ Q, int64_t ldq, const void* __restrict__ R, int64_t ldr, int64_t nr,
    int d, const int32_t* __restrict__ q_self, int self_mode, int64_t self_base, int k, int out_kind,
    int32_t* __restrict__ out_idx, float* __restrict__ out_dist)
{
    __shared__ uint64_t sl[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cnt = *fb_count;
    for (int f = blockIdx.x; f < cnt; f += gridDim.x) {
        const int64_t row = fb_rows[f];
        const int64_t self = self_mode == 1 ? self_base + row : (self_mode == 2 ? (int64_t)q_self[row] : -1);
        uint64_t list = kEmptyList;
        for (int64_t base = (int64_t)wv * 64; base < nr; base += 256) {
            uint64_t cand = kEmptyCand;
            for (int p = 0; p < 16; ++p) {
                const int64_t j = base + p * 4 + (lane >> 4);
                const bool act = j < nr && j != self;
                const float v = dist_g16<DT>(Q, row * ldq, R, j * ldr, d, act);
                const float got = shfl_f32(v, ((lane - p * 4) & 3) * 16);
                const int64_t jj = base + lane;
                if (lane >= p * 4 && lane < p * 4 + 4 && jj < nr && jj != self)
                    cand = make_key(got, (uint32_t)jj);
            }
            cand = seg_sort<64>(cand);
            list = seg_merge_sorted<64>(list, cand);
        }
        sl[wv][lane] = list;
        __syncthreads();
        if (wv == 0) {
            uint64_t a = sl[0][lane];
            for (int o = 1; o < 4; ++o) a = seg_merge_sorted<64>(a, sl[o][lane]);
            if (lane < k) {
                const float d2 = key_d2(a);
                out_idx[row * k + lane] = (int32_t)key_idx(a);
                out_dist[row * k + lane] = out_kind == KNN_OUT_L2 ? sqrtf(d2) : d2;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host

template <int OUT>
static void launch_stage(const knn_matrix& X, void* Xs, int ldp, float* norms, unsigned* maxn,
                         const uint32_t* rowmap, int aux, hipStream_t st)
{
    dim3 grid((unsigned)std::min<int64_t>(ceil_div(X.n, 16), 4096)), block(256);
    switch (X.dtype) {
    case KNN_F32:
        stage_kernel<KNN_F32, OUT><<<grid, block, 0, st>>>(X.data, X.n, X.d, X.ld, Xs, ldp, norms, maxn, rowmap, aux);
        break;
    case KNN_BF16:
        stage_kernel<KNN_BF16, OUT><<<grid, block, 0, st>>>(X.data, X.n, X.d, X.ld, Xs, ldp, norms, maxn, rowmap, aux);
        break;
    default:
        stage_kernel<KNN_F16, OUT><<<grid, block, 0, st>>>(X.data, X.n, X.d, X.ld, Xs, ldp, norms, maxn, rowmap, aux);
        break;
    }
}

static void launch_stage_kind(int kind, const knn_matrix& X, void* Xs, int ldp, float* norms, unsigned* maxn,
                              const uint32_t* rowmap, int aux, hipStream_t st)
{
    if (kind == KNN_BF16) launch_stage<KNN_BF16>(X, Xs, ldp, norms, maxn, rowmap, aux, st);
    else if (kind == KNN_F16) launch_stage<KNN_F16>(X, Xs, ldp, norms, maxn, rowmap, aux, st);
    else launch_stage<KNN_F32>(X, Xs, ldp, norms, maxn, rowmap, aux, st);
}

// Staged copy of a matrix for the GEMM (FP32 ld = roundup(d, 32) or BF16 /
// FP16 ld = roundup(d, 64), both 128-byte multiples), norms and max norm.
// kind (KNN_F32, KNN_BF16, KNN_F16) is the staged element type; values are
// rounded to nearest even.  Row r of the copy is row rowmap[r] of X (rowmap
// nullable: identity).  With aux, ld leaves room for the two trailing FP32
// words (see stage_kernel).
knn_status stage_matrix(ScratchAlloc& ws, const knn_matrix& X, int kind, void** Xs, int* ldp,
                        float** norms, unsigned* maxnorm, hipStream_t st, const uint32_t* rowmap,
                        int aux)
{
    const bool half = kind != KNN_F32;
    const int64_t need = X.d + (aux ? (half ? 4 : 2) : 0);
    *ldp = half ? (int)round_up(need, 64) : (int)round_up(need, 32);
    knn_status r = ws.alloc(Xs, (size_t)X.n * (size_t)(*ldp) * (half ? 2 : 4));
    if (r != KNN_OK) return r;
    r = ws.alloc(norms, (size_t)X.n);
    if (r != KNN_OK) return r;
    launch_stage_kind(kind, X, *Xs, *ldp, *norms, maxnorm, rowmap, aux, st);
    KNN_HIP(hipGetLastError());
    return KNN_OK;
}

// Zero n words (a fill kernel rather than hipMemsetAsync, so that no memset
// node is recorded when a caller captures the stream).
__global__ __launch_bounds__(64) void zero_words_kernel(unsigned* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 64) p[i] = 0u;
}

// Reference splits of a query chunk of qn rows: enough workgroups to fill
// the chip (about 2048), at most 4; every split starts from empty lists,
// which costs merges.
static int exact_splits(int64_t qn)
{
    const int64_t nblk = ceil_div(qn, kTileRows);
    const int64_t S = ceil_div(2048, nblk);
    return (int)(S < 1 ? 1 : (S > 4 ? 4 : S));
}

static size_t elem_bytes(int dtype) { return dtype == KNN_F32 ? 4 : 2; }

// Scratch bytes of one exact call with query chunks of qc rows (every
// request rounded to 256 bytes, as the allocators carve them).
static size_t exact_scratch(const knn_matrix& Q, const knn_matrix& R, bool same, bool bf, int64_t qc)
{
    auto r256 = [](size_t b) { return (size_t)round_up((int64_t)(b ? b : 1), 256); };
    const int ldp = bf ? (int)round_up(R.d, 64) : (int)round_up(R.d, 32);
    const size_t eb = bf ? 2 : 4;
    size_t b = r256(16) + r256((size_t)R.n * ldp * eb) + r256((size_t)R.n * 4);
    if (!same) b += r256((size_t)qc * ldp * eb) + r256((size_t)qc * 4);
    const int S = exact_splits(qc);
    const int64_t slen = round_up(ceil_div(R.n, S), kTileRows);
    const int Sx = (int)ceil_div(R.n, slen);
    b += r256((size_t)qc * Sx * kListW * 8) + r256((size_t)qc * 4);
    return b;
}

// The exact k-NN of Q's rows among R's rows.  Queries are processed in
// chunks of qc rows (all of them when budget is 0) so that the scratch,
// taken from ws, stays within `budget` bytes: the staged reference set
// plus, per chunk, the staged query rows, the split lists and the fallback
// list.  A smaller budget means more chunks, each a pass over R: time for
// memory.  self_mode 1 excludes reference row q for query q (Q == R);
// self_mode 2 excludes q_self[q].
// The exact path for d <= kRankDirectD in FP32: direct canonical distances
// (exact_direct_kernel) over S reference splits, merged by
// merge_rerank_kernel without a certificate (the lists are canonical).
// Scratch: the split lists, S * kListW * 8 bytes per query row of a chunk.
template <int DT>
static void launch_exact_direct(int dc, int km, dim3 grid, hipStream_t st, const void* Qd, int64_t ldq,
                                int64_t nq, const knn_matrix& R, const int32_t* qself, int self_mode,
                                int64_t q0, int k, int64_t split_len, int S, uint64_t* part)
{
#define KNN_ED(DC, KM)                                                                                 \
    exact_direct_kernel<DT, DC, KM><<<grid, 256, 0, st>>>(Qd, ldq, nq, R.data, R.ld, R.n, R.d, qself,  \
                                                          self_mode, q0, k, split_len, S, part)
    if (km == 16) {
        if (dc == 2) KNN_ED(2, 16);
        else if (dc == 3) KNN_ED(3, 16);
        else KNN_ED(0, 16);
    } else {
        if (dc == 2) KNN_ED(2, 32);
        else if (dc == 3) KNN_ED(3, 32);
        else KNN_ED(0, 32);
    }
#undef KNN_ED
}

static knn_status exact_direct_impl(const knn_matrix& Q, const knn_matrix& R, const int32_t* q_self,
                                    int self_mode, int32_t k, int32_t out_kind, int32_t* out_idx,
                                    float* out_dist, hipStream_t st, ScratchAlloc& ws, int64_t budget)
{
    const int64_t nblk = ceil_div(Q.n, 256);
    int S = (int)std::min<int64_t>(16, std::max<int64_t>(1, ceil_div(2048, nblk)));
    S = (int)std::min<int64_t>(S, ceil_div(R.n, 256));
    const int64_t split_len = round_up(ceil_div(R.n, S), 256);
    S = (int)ceil_div(R.n, split_len);
    const size_t per_row = (size_t)S * kListW * 8;
    int64_t qc = Q.n;
    if (budget > 0 && (size_t)round_up((int64_t)(qc * per_row), 256) > (size_t)budget) {
        qc = (budget / (int64_t)per_row) / 256 * 256;
        if (qc < 256)
            return fail(KNN_ENOMEM, "workspace limit of " + std::to_string(budget) + " bytes is below the " +
                                        std::to_string(256 * per_row) + " bytes one 256-query chunk needs");
    }
    uint64_t* part = nullptr;
    knn_status r = ws.alloc(&part, (size_t)qc * S * kListW);
    if (r != KNN_OK) return r;
    const int km = k <= 16 ? 16 : 32;
    const int dc = R.d == 2 || R.d == 3 ? R.d : 0;
    const size_t qeb = elem_bytes(Q.dtype);
    for (int64_t q0 = 0; q0 < Q.n; q0 += qc) {
        const int64_t nq = Q.n - q0 < qc ? Q.n - q0 : qc;
        const void* Qd = (const char*)Q.data + (size_t)q0 * Q.ld * qeb;
        const int32_t* qself = self_mode == 2 ? q_self + q0 : nullptr;
        const dim3 grid((unsigned)ceil_div(nq, 256), (unsigned)S);
        if (Q.dtype == KNN_F32)
            launch_exact_direct<KNN_F32>(dc, km, grid, st, Qd, Q.ld, nq, R, qself, self_mode, q0, k, split_len, S, part);
        else if (Q.dtype == KNN_BF16)
            launch_exact_direct<KNN_BF16>(dc, km, grid, st, Qd, Q.ld, nq, R, qself, self_mode, q0, k, split_len, S,
                                          part);
        else
            launch_exact_direct<KNN_F16>(dc, km, grid, st, Qd, Q.ld, nq, R, qself, self_mode, q0, k, split_len, S,
                                         part);
        KNN_HIP(hipGetLastError());
        int32_t* oi = out_idx + q0 * k;
        float* od = out_dist + q0 * k;
        const dim3 mgrid((unsigned)ceil_div(nq, 4));
#define KNN_MR(DT)                                                                                       \
    merge_rerank_kernel<DT><<<mgrid, 256, 0, st>>>(part, S, nq, k, k, Qd, Q.ld, R.data, R.ld, R.d, nullptr, \
                                                   nullptr, 0.0f, 0.0f, 0, out_kind, oi, od, nullptr, nullptr)
        if (Q.dtype == KNN_F32) KNN_MR(KNN_F32);
        else if (Q.dtype == KNN_BF16) KNN_MR(KNN_BF16);
        else KNN_MR(KNN_F16);
#undef KNN_MR
        KNN_HIP(hipGetLastError());
    }
    return KNN_OK;
}

static knn_status exact_impl(const knn_matrix& Q, const knn_matrix& R, bool same,
                             const int32_t* q_self, int self_mode, int32_t k, int32_t precision,
                             int32_t rerank_k, int32_t out_kind, int32_t* out_idx, float* out_dist,
                             hipStream_t st, ScratchAlloc& ws, int64_t budget)
{
    if (precision != KNN_PREC_FP32 && precision != KNN_PREC_BF16 && precision != KNN_PREC_FP16)
        return fail(KNN_EINVAL, "precision must be KNN_PREC_FP32, KNN_PREC_BF16 or KNN_PREC_FP16");
    if (out_kind != KNN_OUT_L2 && out_kind != KNN_OUT_SQL2)
        return fail(KNN_EINVAL, "out_kind must be KNN_OUT_L2 or KNN_OUT_SQL2");
    if (!out_idx || !out_dist) return fail(KNN_EINVAL, "null output pointer");
    const int64_t avail = R.n - (self_mode ? 1 : 0);
    if (k < 1 || (int64_t)k > avail) return fail(KNN_EINVAL, "k must satisfy 1 <= k <= number of candidates");
    int kp = rerank_k;
    if (kp == 0) kp = 2 * k < kListW ? 2 * k : kListW;
    if (kp < k) return fail(KNN_EINVAL, "rerank_k must be >= k");
    if (kp > kListW || k > KNN_MAX_K)
        return fail(KNN_ENOTSUP, "rerank_k and k above 32 are not supported by the exact path");
    if (budget < 0) return fail(KNN_EINVAL, "workspace limit must be >= 0");
    if (Q.n == 0) return KNN_OK;
    // staged element kind: FP32, or the 16-bit type of the MFMA form
    const int kind = precision == KNN_PREC_BF16 ? KNN_BF16 : (precision == KNN_PREC_FP16 ? KNN_F16 : KNN_F32);
    const bool bf = kind != KNN_F32;
    if (kind == KNN_F32 && R.d <= kRankDirectD)
        return exact_direct_impl(Q, R, q_self, self_mode, k, out_kind, out_idx, out_dist, st, ws, budget);

    // query chunk: the largest multiple of the tile height that fits
    int64_t qc = Q.n;
    if (budget > 0 && exact_scratch(Q, R, same, bf, qc) > (size_t)budget) {
        int64_t lo = 0, hi = ceil_div(Q.n, kTileRows);   // in tiles: lo fits (0 = none), hi does not
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (exact_scratch(Q, R, same, bf, mid * kTileRows) <= (size_t)budget) lo = mid;
            else hi = mid;
        }
        if (lo == 0)
            return fail(KNN_ENOMEM, "workspace limit of " + std::to_string(budget) + " bytes is below the " +
                                        std::to_string(exact_scratch(Q, R, same, bf, kTileRows)) +
                                        " bytes the staged reference set and one 128-query chunk need");
        qc = lo * kTileRows;
    }

    knn_status r;
    unsigned* small = nullptr;   // [0] = max ref norm bits, [1] = fallback count
    r = ws.alloc(&small, 4);
    if (r != KNN_OK) return r;
    zero_words_kernel<<<1, 64, 0, st>>>(small, 4);
    void *Rs = nullptr, *Qb = nullptr;
    float *rn = nullptr, *qnb = nullptr;
    int ldp = 0;
    r = stage_matrix(ws, R, kind, &Rs, &ldp, &rn, small, st, nullptr, 0);
    if (r != KNN_OK) return r;
    const size_t eb = bf ? 2 : 4;
    if (!same) {
        if ((r = ws.alloc(&Qb, (size_t)qc * ldp * eb)) != KNN_OK) return r;
        if ((r = ws.alloc(&qnb, (size_t)qc)) != KNN_OK) return r;
    }
    const int S0 = exact_splits(qc);
    const int64_t split_len = round_up(ceil_div(R.n, S0), kTileRows);
    const int S = (int)ceil_div(R.n, split_len);
    uint64_t* part = nullptr;
    r = ws.alloc(&part, (size_t)qc * S * kListW);
    if (r != KNN_OK) return r;
    int32_t* fb_rows = nullptr;
    r = ws.alloc(&fb_rows, (size_t)qc);
    if (r != KNN_OK) return r;

    const bool ares = ldp <= (bf ? TileCfg<KNN_BF16>::AMAX : TileCfg<KNN_F32>::AMAX);
    // GEMM error bound (FP32): (d + 3) u (|q| + max|r|)^2 with u = 2^-24;
    // re-rank bound: (d/16 + 8) u relative.
    const float u = 5.9604645e-08f;
    const float err_coef = (float)(R.d + 3) * u * 1.01f;
    const float edir = (float)(R.d / 16 + 8) * u;
    const int certify = bf ? 0 : 1;
    int* fb_count = (int*)(small + 1);
    const size_t qeb = elem_bytes(Q.dtype);

    for (int64_t q0 = 0; q0 < Q.n; q0 += qc) {
        const int64_t nq = Q.n - q0 < qc ? Q.n - q0 : qc;
        const void* Qs;
        const float* qn;
        if (same) {
            Qs = (const char*)Rs + (size_t)q0 * ldp * eb;
            qn = rn + q0;
        } else {
            const knn_matrix Qc = {(const char*)Q.data + (size_t)q0 * Q.ld * qeb, nq, Q.d, Q.ld, Q.dtype};
            launch_stage_kind(kind, Qc, Qb, ldp, qnb, nullptr, nullptr, 0, st);
            Qs = Qb;
            qn = qnb;
        }
        const int32_t* qself = self_mode == 2 ? q_self + q0 : nullptr;
        if (q0 > 0) zero_words_kernel<<<1, 64, 0, st>>>(small + 1, 1);
        dim3 tgrid((unsigned)ceil_div(nq, kTileRows), (unsigned)S);
#define KNN_TILE(BFV, AR)                                                                        \
    exact_tile_kernel<BFV, AR><<<tgrid, 256, 0, st>>>(Qs, qn, nq, Rs, rn, R.n, ldp, qself,       \
                                                      self_mode, q0, kp, split_len, S, small, part)
        if (kind == KNN_BF16) {
            if (ares) KNN_TILE(KNN_BF16, true);
            else KNN_TILE(KNN_BF16, false);
        } else if (kind == KNN_F16) {
            if (ares) KNN_TILE(KNN_F16, true);
            else KNN_TILE(KNN_F16, false);
        } else {
            if (ares) KNN_TILE(KNN_F32, true);
            else KNN_TILE(KNN_F32, false);
        }
#undef KNN_TILE
        KNN_HIP(hipGetLastError());

        const void* Qd = (const char*)Q.data + (size_t)q0 * Q.ld * qeb;
        int32_t* oi = out_idx + q0 * k;
        float* od = out_dist + q0 * k;
        dim3 mgrid((unsigned)ceil_div(nq, 4));
#define KNN_MR(DT)                                                                              \
    merge_rerank_kernel<DT><<<mgrid, 256, 0, st>>>(part, S, nq, kp, k, Qd, Q.ld, R.data, R.ld,  \
                                                   R.d, qn, small, err_coef, edir, certify,     \
                                                   out_kind, oi, od, fb_rows, fb_count)
        if (Q.dtype == KNN_F32) KNN_MR(KNN_F32);
        else if (Q.dtype == KNN_BF16) KNN_MR(KNN_BF16);
        else KNN_MR(KNN_F16);
#undef KNN_MR
        KNN_HIP(hipGetLastError());
        if (certify) {
            dim3 fgrid(1024);
#define KNN_FB(DT)                                                                              \
    exact_fallback_kernel<DT><<<fgrid, 256, 0, st>>>(fb_rows, fb_count, Qd, Q.ld, R.data, R.ld, \
                                                     R.n, R.d, qself, self_mode, q0, k,         \
                                                     out_kind, oi, od)
            if (Q.dtype == KNN_F32) KNN_FB(KNN_F32);
            else if (Q.dtype == KNN_BF16) KNN_FB(KNN_BF16);
            else KNN_FB(KNN_F16);
#undef KNN_FB
            KNN_HIP(hipGetLastError());
        }
    }
    KNN_HIP(hipStreamSynchronize(st));
    return KNN_OK;
}

// ------------------------------------------------------------ quality

// One wave per row i.  N(i) (row i of Hn, the exact lists in X) sits in
// lanes 0..k-1, L(i) (row i of Ln, the lists in the embedding Y) likewise.
// U = L \ N are the trustworthiness probes: their canonical FP32 distances
// in X as keys; V = N \ L the continuity probes, keyed by their distances in
// Y.  Both are sorted ascending and padded with kEmptyCand to kRankP (k <=
// kRankP); hits[i] = |N intersect L|.  With all_l, U is all of L (N is not
// needed; Hn may be null).  pu, pv and hits may each be null: that output
// is not formed.
__global__ __launch_bounds__(256) void quality_probes_kernel(int64_t n, int k, const int32_t* __restrict__ Hn,
                                                             const int32_t* __restrict__ Ln,
                                                             const float* __restrict__ Xs, int ldx, int dx,
                                                             const float* __restrict__ Ys, int ldy, int dy,
                                                             uint64_t* __restrict__ pu, uint64_t* __restrict__ pv,
                                                             int32_t* __restrict__ hits, int all_l)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;   // uniform across the wave
    const int32_t hv = lane < k && Hn ? Hn[i * k + lane] : -1;
    const int32_t lv = lane < k ? Ln[i * k + lane] : -1;
    bool l_in_n = false, n_in_l = false;
    for (int r = 0; r < k; ++r) {
        // lane r's entries by readlane, outside any lane-dependent branch
        const int32_t hr = (int32_t)bcast_u32((uint32_t)hv, r), lr = (int32_t)bcast_u32((uint32_t)lv, r);
        l_in_n |= lv == hr;
        n_in_l |= hv == lr;
    }
    // all_l: every member of L(i) is a probe in X (no N(i) yet); a member
    // of N(i) then has rank <= k and adds nothing to the trust sum.  A side
    // whose output is null computes nothing; without Hn there is no V side
    const bool inU = pu && lane < k && (all_l || !l_in_n), inV = Hn && lane < k && !n_in_l;
    const float du = dist_batch16<KNN_F32, 4>(Xs, ldx, i, (uint32_t)lv, inU, dx);
    const float dv = dist_batch16<KNN_F32, 4>(Ys, ldy, i, (uint32_t)hv, inV, dy);
    uint64_t ku = inU ? make_key(du, (uint32_t)lv) : kEmptyCand;
    uint64_t kv = inV ? make_key(dv, (uint32_t)hv) : kEmptyCand;
    ku = seg_sort<16>(ku);
    kv = seg_sort<16>(kv);
    if (lane < kRankP) {
        if (pu) pu[i * kRankP + lane] = ku;
        if (pv) pv[i * kRankP + lane] = kv;
    }
    const int nv = popc64(ballot(inV));
    if (hits && lane == 0) hits[i] = k - nv;   // |N & L| = k - |N \ L|
}

// Per row: trust = sum over U of (rank - k) = sum of (count + 1 - k), cont
// likewise over V; the three totals by exact integer atomics (order-free).
__global__ __launch_bounds__(256) void quality_reduce_kernel(int64_t n, int k, const uint64_t* __restrict__ pu,
                                                             const uint32_t* __restrict__ cu,
                                                             const uint64_t* __restrict__ pv,
                                                             const uint32_t* __restrict__ cv,
                                                             const int32_t* __restrict__ hits,
                                                             int64_t* __restrict__ trust_row,
                                                             int64_t* __restrict__ cont_row,
                                                             unsigned long long* __restrict__ tot)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long t = 0, c = 0, hsum = 0;
    if (i < n) {
        for (int p = 0; p < kRankP; ++p) {
            // rank - k where the rank exceeds k (probes of rank <= k, members
            // of both lists, add nothing)
            const uint32_t ru = cu[i * kRankP + p] + 1u, rv = cv[i * kRankP + p] + 1u;
            if (pu[i * kRankP + p] != kEmptyCand && ru > (uint32_t)k) t += (unsigned long long)(ru - (uint32_t)k);
            if (pv[i * kRankP + p] != kEmptyCand && rv > (uint32_t)k) c += (unsigned long long)(rv - (uint32_t)k);
        }
        hsum = (unsigned long long)hits[i];
        if (trust_row) trust_row[i] = (int64_t)t;
        if (cont_row) cont_row[i] = (int64_t)c;
    }
    for (int o = 32; o > 0; o >>= 1) {
        t += shfl_u64(t, (threadIdx.x & 63) ^ o);
        c += shfl_u64(c, (threadIdx.x & 63) ^ o);
        hsum += shfl_u64(hsum, (threadIdx.x & 63) ^ o);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&tot[0], hsum);
        atomicAdd(&tot[1], t);
        atomicAdd(&tot[2], c);
    }
}

static knn_status quality_impl(const knn_matrix& X, const knn_matrix& Y, int k, int32_t* hits_out,
                               int64_t* trust_out, int64_t* cont_out, double* metrics, hipStream_t st)
{
    const int64_t n = X.n;
    Workspace ws(st, 0);
    knn_status r;
    int32_t *Hn, *Ln, *hits;
    float *Hd, *Ld;
    if ((r = ws.alloc(&Hn, (size_t)n * k)) != KNN_OK) return r;
    if ((r = ws.alloc(&Ln, (size_t)n * k)) != KNN_OK) return r;
    if ((r = ws.alloc(&Hd, (size_t)n * k)) != KNN_OK) return r;
    if ((r = ws.alloc(&Ld, (size_t)n * k)) != KNN_OK) return r;
    // exact lists in both spaces (FP32, canonical re-rank).  Above
    // kRankDirectD dimensions X's lists come from its rank pass (fused):
    // the same Gram tiles give the ranks and the split lists
    const bool fused = X.d > kRankDirectD;
    if ((r = exact_impl(Y, Y, true, nullptr, 1, k, KNN_PREC_FP32, 0, KNN_OUT_SQL2, Ln, Ld, st, ws, 0)) != KNN_OK)
        return r;
    if (!fused &&
        (r = exact_impl(X, X, true, nullptr, 1, k, KNN_PREC_FP32, 0, KNN_OUT_SQL2, Hn, Hd, st, ws, 0)) != KNN_OK)
        return r;
    unsigned* small;   // [0] max norm of X, [1] max norm of Y; then three u64 totals
    if ((r = ws.alloc(&small, 8)) != KNN_OK) return r;
    zero_words_kernel<<<1, 64, 0, st>>>(small, 8);
    void *Xs, *Ys;
    float *xn, *yn;
    int ldx, ldy;
    if ((r = stage_matrix(ws, X, KNN_F32, &Xs, &ldx, &xn, small, st, nullptr, 0)) != KNN_OK) return r;
    if ((r = stage_matrix(ws, Y, KNN_F32, &Ys, &ldy, &yn, small + 1, st, nullptr, 0)) != KNN_OK) return r;
    uint64_t *pu, *pv;
    uint32_t *cu, *cv;
    if ((r = ws.alloc(&pu, (size_t)n * kRankP)) != KNN_OK) return r;
    if ((r = ws.alloc(&pv, (size_t)n * kRankP)) != KNN_OK) return r;
    if ((r = ws.alloc(&cu, (size_t)n * kRankP)) != KNN_OK) return r;
    if ((r = ws.alloc(&cv, (size_t)n * kRankP)) != KNN_OK) return r;
    hits = hits_out;
    if (!hits && (r = ws.alloc(&hits, (size_t)n)) != KNN_OK) return r;
    // X's probes: L(i) \ N(i), or every member of L(i) when N(i) is not
    // known yet (fused); Y's probes N(i) \ L(i) and |N & L| once it is
    if (fused)
        quality_probes_kernel<<<(unsigned)ceil_div(n, 4), 256, 0, st>>>(n, k, nullptr, Ln, (const float*)Xs, ldx,
                                                                        X.d, (const float*)Ys, ldy, Y.d, pu, nullptr,
                                                                        nullptr, 1);
    else
        quality_probes_kernel<<<(unsigned)ceil_div(n, 4), 256, 0, st>>>(n, k, Hn, Ln, (const float*)Xs, ldx, X.d,
                                                                        (const float*)Ys, ldy, Y.d, pu, pv, hits, 0);
    KNN_HIP(hipGetLastError());
    const float u = 5.9604645e-08f;
    // The tile pass: S reference splits, so that the workgroups fill the
    // chip's resident slots (two per CU) in nearly whole waves; each
    // workgroup holds a queue of undecided pairs of one tile, launches of at
    // most kRankBlocks workgroups.
    int dev = 0, ncu = 256;
    KNN_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 256;
    const int64_t nblk = ceil_div(n, kTileRows), ntile = nblk, slots = 2 * (int64_t)ncu;
    int S = 1;
    for (; S < kRankMaxSplits; ++S) {
        const int64_t b = nblk * S;   // stop once the waves of resident workgroups are 90% full on average
        if (b % slots == 0 || (double)b / (double)slots >= 0.9 * (double)ceil_div(b, slots)) break;
    }
    if (S > ntile) S = (int)ntile;
    const int64_t split_len = ceil_div(ntile, S) * kTileRows;
    S = (int)ceil_div(n, split_len);   // no empty split
    const int64_t per_launch = kRankBlocks / S;   // query blocks per launch
    uint32_t* rq = nullptr;
    if ((X.d > kRankDirectD || Y.d > kRankDirectD) &&
        (r = ws.alloc(&rq, (size_t)std::min<int64_t>(nblk, per_launch) * S * kTileRows * kTileRows)) != KNN_OK)
        return r;
    const int kp = 2 * k < kListW ? 2 * k : kListW;   // the lists' re-rank width, as knn_exact's default
    uint64_t* part = nullptr;
    if (fused && (r = ws.alloc(&part, (size_t)n * S * kListW)) != KNN_OK) return r;
    auto rank_tile = [&](const float* Zs, const float* zn, int ldz, int dz, const uint64_t* pz, const unsigned* mx,
                         uint32_t* cz, uint64_t* lists) {
        // GEMM distance error: 2 gamma_d |q| |r| for the FP32 dot product
        // plus 2u (|q|^2 + |r|^2) for the norms (FP64 sums rounded once)
        // and their sum; the canonical distance's own error (edir) carries
        // the margin for the final rounding
        const float ecd = 2.0f * (float)(dz + 2) * u * 1.01f, ecn = 2.02f * u;
        const float ed = (float)(dz / 16 + 8) * u;
        zero_words_kernel<<<(unsigned)std::min<int64_t>(ceil_div(n * kRankP, 64), 4096), 64, 0, st>>>(cz,
                                                                                                 n * kRankP);
        for (int64_t q0 = 0; q0 < n; q0 += per_launch * kTileRows) {
            const int64_t nq = std::min<int64_t>(n - q0, per_launch * kTileRows);
            const unsigned g = (unsigned)(ceil_div(nq, kTileRows) * S);
            if (lists)
                rank_tile_kernel<true><<<g, 256, 0, st>>>(Zs + q0 * ldz, zn + q0, nq, Zs, zn, n, ldz, dz, 1, q0,
                                                          pz + q0 * kRankP, mx, ecd, ecn, ed, S, split_len,
                                                          cz + q0 * kRankP, rq, kp, lists + q0 * S * kListW);
            else
                rank_tile_kernel<false><<<g, 256, 0, st>>>(Zs + q0 * ldz, zn + q0, nq, Zs, zn, n, ldz, dz, 1, q0,
                                                           pz + q0 * kRankP, mx, ecd, ecn, ed, S, split_len,
                                                           cz + q0 * kRankP, rq, kp, nullptr);
        }
    };
    auto rank_direct = [&](const float* Zs, int ldz, int dz, const uint64_t* pz, uint32_t* cz) {
        // reference splits (counts added) so that enough waves hide the tile reads
        const int64_t nb = ceil_div(n, 256);
        int Sd = (int)std::min<int64_t>(16, std::max<int64_t>(1, ceil_div(2048, nb)));
        Sd = (int)std::min<int64_t>(Sd, ceil_div(n, 256));
        const int64_t sl = round_up(ceil_div(n, Sd), 256);
        Sd = (int)ceil_div(n, sl);
        zero_words_kernel<<<(unsigned)std::min<int64_t>(ceil_div(n * kRankP, 64), 4096), 64, 0, st>>>(cz,
                                                                                                 n * kRankP);
        const dim3 g((unsigned)nb, (unsigned)Sd);
        if (dz == 2)
            rank_direct_kernel<2><<<g, 256, 0, st>>>(Zs, n, ldz, dz, pz, sl, cz);
        else if (dz == 3)
            rank_direct_kernel<3><<<g, 256, 0, st>>>(Zs, n, ldz, dz, pz, sl, cz);
        else
            rank_direct_kernel<0><<<g, 256, 0, st>>>(Zs, n, ldz, dz, pz, sl, cz);
    };
    if (!fused) {
        rank_direct((const float*)Xs, ldx, X.d, pu, cu);
    } else {
        rank_tile((const float*)Xs, xn, ldx, X.d, pu, small, cu, part);
        KNN_HIP(hipGetLastError());
        // X's exact lists from the split lists: merge, canonical re-rank,
        // certificate, and the exhaustive search for rows not certified
        int32_t* fb_rows = nullptr;
        int* fb_count = nullptr;
        if ((r = ws.alloc(&fb_rows, (size_t)n)) != KNN_OK) return r;
        if ((r = ws.alloc(&fb_count, 1)) != KNN_OK) return r;
        zero_words_kernel<<<1, 64, 0, st>>>((unsigned*)fb_count, 1);
        const float err_coef = (float)(X.d + 3) * u * 1.01f, edir = (float)(X.d / 16 + 8) * u;
        const dim3 mgrid((unsigned)ceil_div(n, 4));
#define KNN_QMR(DT)                                                                                            \
    merge_rerank_kernel<DT><<<mgrid, 256, 0, st>>>(part, S, n, kp, k, X.data, X.ld, X.data, X.ld, X.d, xn, small, \
                                                   err_coef, edir, 1, KNN_OUT_SQL2, Hn, Hd, fb_rows, fb_count);    \
    exact_fallback_kernel<DT><<<1024, 256, 0, st>>>(fb_rows, fb_count, X.data, X.ld, X.data, X.ld, n, X.d, nullptr,  \
                                                    1, 0, k, KNN_OUT_SQL2, Hn, Hd)
        if (X.dtype == KNN_F32) {
            KNN_QMR(KNN_F32);
        } else if (X.dtype == KNN_BF16) {
            KNN_QMR(KNN_BF16);
        } else {
            KNN_QMR(KNN_F16);
        }
#undef KNN_QMR
        KNN_HIP(hipGetLastError());
        quality_probes_kernel<<<(unsigned)ceil_div(n, 4), 256, 0, st>>>(n, k, Hn, Ln, (const float*)Xs, ldx, X.d,
                                                                        (const float*)Ys, ldy, Y.d, nullptr, pv,
                                                                        hits, 0);
    }
    if (Y.d <= kRankDirectD)
        rank_direct((const float*)Ys, ldy, Y.d, pv, cv);
    else
        rank_tile((const float*)Ys, yn, ldy, Y.d, pv, small + 1, cv, nullptr);
    KNN_HIP(hipGetLastError());
    unsigned long long* tot = (unsigned long long*)(small + 2);
    quality_reduce_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(n, k, pu, cu, pv, cv, hits, trust_out,
                                                                      cont_out, tot);
    KNN_HIP(hipGetLastError());
    unsigned long long host[3];
    KNN_HIP(hipMemcpyAsync(host, tot, 24, hipMemcpyDeviceToHost, st));
    KNN_HIP(hipStreamSynchronize(st));
    const double nk = (double)n * (double)k;
    const double z = 2.0 / (nk * (2.0 * (double)n - 3.0 * (double)k - 1.0));
    metrics[0] = (double)host[0] / nk;
    metrics[1] = 1.0 - z * (double)host[1];
    metrics[2] = 1.0 - z * (double)host[2];
    return KNN_OK;
}

// ------------------------------------------------------------ no-alloc path

// The static scratch array of knn_exact_noalloc: one copy per device, held
// by the loaded code object until the process ends.  Host code never uses
// this name as an address (on the host it is a stand-in symbol): the device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratch = (size_t)KNN_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratch];

static knn_status static_scratch(void** out)
{
    static std::mutex mu;
    static void* addr[64] = {};
    int dev = -1;
    KNN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(KNN_EDEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(KNN_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[dev] = p;
    }
    *out = addr[dev];
    return KNN_OK;
}

}  // namespace knn

using namespace knn;

extern "C" knn_status knn_exact(knn_matrix X, int32_t k, int32_t precision, int32_t rerank_k,
                                int32_t out_kind, int32_t* out_idx, float* out_dist, void* stream)
{
    try {
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if (X.n < 2) return fail(KNN_EINVAL, "X.n must be >= 2");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        return exact_impl(X, X, true, nullptr, 1, k, precision, rerank_k, out_kind, out_idx,
                          out_dist, st, ws, 0);
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status knn_exact_query(knn_matrix Q, knn_matrix R, const int32_t* q_self,
                                      int32_t k, int32_t precision, int32_t rerank_k,
                                      int32_t out_kind, int32_t* out_idx, float* out_dist,
                                      void* stream)
{
    try {
        knn_status r = check_matrix(Q, "Q");
        if (r != KNN_OK) return r;
        r = check_matrix(R, "R");
        if (r != KNN_OK) return r;
        if (Q.d != R.d) return fail(KNN_EINVAL, "Q.d != R.d");
        if (Q.dtype != R.dtype) return fail(KNN_EINVAL, "Q.dtype != R.dtype");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        return exact_impl(Q, R, false, q_self, q_self ? 2 : 0, k, precision, rerank_k, out_kind,
                          out_idx, out_dist, st, ws, 0);
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status knn_exact_query_limited(knn_matrix Q, knn_matrix R, const int32_t* q_self,
                                              int32_t k, int32_t precision, int32_t rerank_k,
                                              int32_t out_kind, int64_t workspace_limit_bytes,
                                              int32_t* out_idx, float* out_dist, void* stream)
{
    try {
        knn_status r = check_matrix(Q, "Q");
        if (r != KNN_OK) return r;
        r = check_matrix(R, "R");
        if (r != KNN_OK) return r;
        if (Q.d != R.d) return fail(KNN_EINVAL, "Q.d != R.d");
        if (Q.dtype != R.dtype) return fail(KNN_EINVAL, "Q.dtype != R.dtype");
        hipStream_t st = (hipStream_t)stream;
        Workspace ws(st, 0);
        return exact_impl(Q, R, false, q_self, q_self ? 2 : 0, k, precision, rerank_k, out_kind,
                          out_idx, out_dist, st, ws, workspace_limit_bytes);
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status knn_exact_noalloc(knn_matrix X, int32_t k, int32_t precision, int32_t rerank_k,
                                        int32_t out_kind, int32_t* out_idx, float* out_dist, void* stream)
{
    try {
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if (X.n < 2) return fail(KNN_EINVAL, "X.n must be >= 2");
        void* base = nullptr;
        if ((r = static_scratch(&base)) != KNN_OK) return r;
        FixedScratch ws(base, kStaticScratch);
        return exact_impl(X, X, true, nullptr, 1, k, precision, rerank_k, out_kind, out_idx,
                          out_dist, (hipStream_t)stream, ws, (int64_t)kStaticScratch);
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status knn_quality(knn_matrix X, knn_matrix Y, int32_t k, int32_t* hits, int64_t* trust,
                                  int64_t* cont, double* metrics, void* stream)
{
    try {
        knn_status r = check_matrix(X, "X");
        if (r != KNN_OK) return r;
        if ((r = check_matrix(Y, "Y")) != KNN_OK) return r;
        if (!metrics) return fail(KNN_EINVAL, "metrics is null");
        if (X.n != Y.n) return fail(KNN_EINVAL, "X.n != Y.n");
        if (k < 1 || 3 * (int64_t)k >= 2 * X.n - 1) return fail(KNN_EINVAL, "k must satisfy 1 <= k and 3k < 2n - 1");
        if (k > kRankP) return fail(KNN_ENOTSUP, "k above 16 is not supported by the quality metrics");
        return quality_impl(X, Y, k, hits, trust, cont, metrics, (hipStream_t)stream);
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}
