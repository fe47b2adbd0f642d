// Shared device and host helpers of the gfx950 kNN library.
//
// Keys.  A candidate neighbour is a 64-bit key (float bits of the squared
// distance << 32) | index.  Squared distances are clamped to >= +0, and the
// bit patterns of non-negative floats order like unsigned integers, so the
// unsigned order of keys is the (distance, index) order the results use.
//
// Random numbers.  Every random choice is a pure function of
// (seed, stream tag, iteration, row, slot) through a counter-based hash built
// from the splitmix64 finaliser (Steele, Lea & Flood, OOPSLA 2014), so runs
// are reproducible and a build can be resumed bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/knn.h"

namespace knn {

// ------------------------------------------------------------------ keys

constexpr uint64_t kEmptyList = 0x7F800000FFFFFFFFull;  // +inf distance, index ~0
constexpr uint64_t kEmptyCand = ~0ull;                   // above every list key

__device__ inline uint64_t make_key(float d2, uint32_t idx)
{
    d2 = d2 > 0.0f ? d2 : 0.0f;  // also maps -0 and NaN to +0
    return ((uint64_t)__float_as_uint(d2) << 32) | (uint64_t)idx;
}
__device__ inline float key_d2(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ inline uint32_t key_idx(uint64_t k) { return (uint32_t)k; }
__device__ inline bool key_valid(uint64_t k) { return (uint32_t)k != 0xFFFFFFFFu; }

// ------------------------------------------------------------------ RNG

__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Hash of a tuple of counters: each word is absorbed with a distinct odd
// multiplier before a full mix, so (a, b) and (b, a) differ.
__host__ __device__ inline uint64_t hash4(uint64_t seed, uint64_t a, uint64_t b, uint64_t c)
{
    uint64_t h = mix64(seed + 0x9E3779B97F4A7C15ull);
    h = mix64(h ^ (a * 0xD6E8FEB86659FD93ull));
    h = mix64(h ^ (b * 0xA0761D6478BD642Full));
    h = mix64(h ^ (c * 0xE7037ED1A0B428DBull));
    return h;
}

// Uniform integer in [0, m) from 64 random bits (multiply-high reduction).
__host__ __device__ inline uint32_t bounded(uint64_t r, uint32_t m)
{
    return (uint32_t)(((r >> 32) * (uint64_t)m) >> 32);
}

// Stream tags keep independent random decisions apart.
enum : uint64_t {
    kTagInit = 1, kTagSample = 2, kTagRevNew = 3, kTagRevOld = 4, kTagSlot = 5,
    kTagRevSlot = 6, kTagTriplet = 7, kTagDirs = 8, kTagWeights = 9
};

// ------------------------------------------------------------------ waves

__device__ inline int lane_id() { return (int)__lane_id(); }

__device__ inline uint32_t shfl_u32(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ inline uint64_t shfl_u64(uint64_t v, int src)
{
    uint32_t lo = shfl_u32((uint32_t)v, src);
    uint32_t hi = shfl_u32((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline float shfl_f32(float v, int src)
{
    return __uint_as_float(shfl_u32(__float_as_uint(v), src));
}
// Exchange with lane ^ j inside the wave without an LDS round trip:
// j = 1, 2 by DPP quad permutes; j = 4, 8 by DPP row shifts (each lane keeps
// the direction that stays inside its 16-lane row); j = 16, 32 by the gfx950
// permlane swaps (rows 2r+1 <-> 2r, and the two 32-lane halves).  j must be a
// compile-time constant after unrolling.
__device__ __attribute__((always_inline)) inline uint32_t xor_u32(uint32_t v, int j)
{
    const int lane = lane_id();
    if (j == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    if (j == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    if (j == 4) {
        uint32_t a = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x104, 0xF, 0xF, false);
        uint32_t b = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
        return (lane & 4) ? b : a;
    }
    if (j == 8) {
        uint32_t a = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x108, 0xF, 0xF, false);
        uint32_t b = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
        return (lane & 8) ? b : a;
    }
    if (j == 16) {
        auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? p[0] : p[1];
    }
    if (j == 32) {
        auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? p[0] : p[1];
    }
    return shfl_u32(v, lane ^ j);
}
__device__ __attribute__((always_inline)) inline uint64_t shfl_xor_u64(uint64_t v, int j)
{
    uint32_t lo = xor_u32((uint32_t)v, j), hi = xor_u32((uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __attribute__((always_inline)) inline float xor_f32(float v, int j)
{
    return __uint_as_float(xor_u32(__float_as_uint(v), j));
}
// Value of v in lane l (l uniform across the wave): v_readlane, no LDS.
__device__ __attribute__((always_inline)) inline uint32_t bcast_u32(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __attribute__((always_inline)) inline uint64_t bcast_u64(uint64_t v, int l)
{
    uint32_t lo = bcast_u32((uint32_t)v, l), hi = bcast_u32((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ inline uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

// Ascending bitonic sort of independent segments of W lanes (W = 2..64,
// power of two), one key per lane.
template <int W>
__device__ inline uint64_t seg_sort(uint64_t key)
{
    const int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= W; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint64_t o = shfl_xor_u64(key, j);
            bool up = (k == W) ? true : ((lane & k) == 0);
            bool lower = (lane & j) == 0;
            key = (lower == up) ? umin64(key, o) : umax64(key, o);
        }
    }
    return key;
}

// Sort a bitonic sequence held in segments of W lanes into ascending order.
template <int W>
__device__ inline uint64_t seg_bitonic_merge(uint64_t key)
{
    const int lane = lane_id();
#pragma unroll
    for (int j = W >> 1; j > 0; j >>= 1) {
        uint64_t o = shfl_xor_u64(key, j);
        key = ((lane & j) == 0) ? umin64(key, o) : umax64(key, o);
    }
    return key;
}

// Keep the W smallest of the union of two ascending W-lane segments
// (list, cand) as an ascending segment: min(list[i], cand[W-1-i]) is bitonic
// and holds exactly those keys.
template <int W>
__device__ inline uint64_t seg_merge_sorted(uint64_t list, uint64_t cand_sorted)
{
    uint64_t rev = shfl_xor_u64(cand_sorted, W - 1);
    return seg_bitonic_merge<W>(umin64(list, rev));
}

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }
__device__ inline int popc64(uint64_t m) { return __popcll(m); }
// number of set bits of m in lanes below this one
__device__ inline int rank_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline float wave_sum16(float v)
{
    // tree reduction inside aligned groups of 16 lanes (fixed order)
    v += xor_f32(v, 8);
    v += xor_f32(v, 4);
    v += xor_f32(v, 2);
    v += xor_f32(v, 1);
    return v;
}

// ------------------------------------------------------------------ inputs

template <int DT> struct elem;
template <> struct elem<KNN_F32> {
    using T = float;
    __device__ static float ld(const void* p, int64_t i) { return ((const float*)p)[i]; }
};
template <> struct elem<KNN_BF16> {
    using T = uint16_t;
    __device__ static float ld(const void* p, int64_t i)
    {
        return __uint_as_float((uint32_t)((const uint16_t*)p)[i] << 16);
    }
};
template <> struct elem<KNN_F16> {
    using T = _Float16;
    __device__ static float ld(const void* p, int64_t i) { return (float)((const _Float16*)p)[i]; }
};

// FP32 -> BF16 round to nearest even (inputs are finite).
__device__ inline uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Canonical FP32 direct-difference squared distance between row a of A and
// row b of B, computed by an aligned group of 16 lanes: lane g of the group
// accumulates t = g, g + 16, g + 32, ... in order, then a fixed tree sum.
// Every lane of the group returns the same value; the value does not depend
// on which group computes it, and swapping a and b gives the same bits.
template <int DT>
__device__ inline float dist_g16(const void* A, int64_t a_off, const void* B, int64_t b_off,
                                 int d, bool active)
{
    const int g = lane_id() & 15;
    float s = 0.0f;
    if (active) {
        for (int t = g; t < d; t += 16) {
            float e = elem<DT>::ld(A, a_off + t) - elem<DT>::ld(B, b_off + t);
            s = fmaf(e, e, s);
        }
    }
    return wave_sum16(s);
}

// Squared distances from row `a` to the 4 * NP candidates base .. base +
// 4 NP - 1: candidate e is lane e's row `cid` (used when `act`).  Each is
// computed as dist_g16 computes it -- the 16 lanes of a group sum
// coordinates g, g+16, ... in order, then a fixed 16-lane tree -- four
// candidates per pass, and every pass's loads of one coordinate step are
// issued together rather than pass after pass.  Lane e in that range returns
// candidate e's distance (0 when inactive); other lanes return 0.
// Rows are ld elements apart in X; inactive candidates read row a.
template <int DT, int NP>
__device__ inline float dist_batch16(const void* X, int64_t ld, int64_t a, uint32_t cid, bool act, int d,
                                     int base = 0)
{
    const int lane = lane_id(), g = lane & 15;
    int64_t off[NP];
    bool ok[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int ci = (base + 4 * q + (lane >> 4)) & 63;
        const uint32_t cj = shfl_u32(cid, ci);
        ok[q] = shfl_u32(act ? 1u : 0u, ci) != 0u;
        off[q] = (ok[q] ? (int64_t)cj : a) * ld;
    }
    const int64_t ao = a * ld;
    float part[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) part[q] = 0.0f;
    for (int t = g; t < d; t += 16) {
        const float xa = elem<DT>::ld(X, ao + t);
        float xb[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) xb[q] = elem<DT>::ld(X, off[q] + t);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const float e = xa - xb[q];
            part[q] = ok[q] ? fmaf(e, e, part[q]) : part[q];
        }
    }
    float mine = 0.0f;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const float v = wave_sum16(part[q]);
        const float got = shfl_f32(v, ((lane - base - 4 * q) & 3) * 16);
        if (lane >= base + 4 * q && lane < base + 4 * q + 4) mine = got;
    }
    return mine;
}

// ------------------------------------------------------------------ host

void set_error(const std::string& msg);
knn_status fail(knn_status s, const std::string& msg);

#define KNN_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::knn::fail(KNN_EDEVICE, std::string(#call) + ": " +               \
                                                hipGetErrorString(e_));                \
    } while (0)

// Where an entry point's scratch comes from: alloc hands out a 256-byte
// aligned block that stays valid until the call returns.
class ScratchAlloc {
public:
    virtual ~ScratchAlloc() = default;
    // returns KNN_OK or KNN_ENOMEM / KNN_EDEVICE
    virtual knn_status alloc(void** p, size_t bytes) = 0;
    template <typename T>
    knn_status alloc(T** p, size_t count) { return alloc((void**)p, count * sizeof(T)); }
};

// A fixed device block carved front to back; never allocates.  Requests
// past its end fail with KNN_ENOMEM.
class FixedScratch : public ScratchAlloc {
public:
    FixedScratch(void* base, size_t cap) : base_((char*)base), cap_(cap) {}
    using ScratchAlloc::alloc;
    knn_status alloc(void** p, size_t bytes) override;
    size_t used() const { return off_; }

private:
    char* base_;
    size_t cap_;
    size_t off_ = 0;
};

// Scratch for one entry-point call.  Requests are carved (256-byte aligned)
// from a grow-only arena that the library keeps per device, so steady-state
// calls neither allocate nor free device memory.  The arena is held by one
// call at a time (a per-device lock taken by the constructor); the call's
// stream first waits for the previous holder's work, and the destructor
// records the point after which the arena is free again.  A request that
// does not fit is served from a library-owned stream-ordered pool for this
// call, and the arena is regrown to the call's total for the next one.
// Only one Workspace may be alive per thread.
class Workspace : public ScratchAlloc {
public:
    Workspace(hipStream_t s, int64_t limit);
    ~Workspace() override;
    using ScratchAlloc::alloc;
    knn_status alloc(void** p, size_t bytes) override;
    size_t used() const { return used_; }

private:
    hipStream_t stream_;
    int64_t limit_;
    int dev_ = -1;
    size_t used_ = 0;      // bytes handed out by this call (arena + overflow)
    size_t off_ = 0;       // arena bytes used
    void* ptrs_[64];       // overflow allocations of this call
    int nptr_ = 0;
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

knn_status check_matrix(const knn_matrix& X, const char* name);

// 64 bytes of pinned host memory for device -> host counter reads, one block
// per host thread (null if the allocation failed).
unsigned long long* pinned_counters();

}  // namespace knn
