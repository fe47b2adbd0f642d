// NNDescent on gfx950 (Dong, Charikar & Li, WWW 2011), as the paper's
// section "GPU-Native k-NN via NNDescent" uses it: lists start from random
// neighbours, are refined through neighbours of neighbours, and the run
// stops once an iteration's list updates fall below delta * n * K_b with
// delta = 0.015.
//
// State: per point a list of K_b (index, squared distance, new-flag)
// entries sorted by (distance, index).  One iteration is two kernels with
// no host round trip except a 64-byte counter read:
//
//  join     one wave per point v: the new list new_f(v) + reverse-new and the
//           old list old_f(v) + reverse-old are deduplicated (at most 64
//           members; old members past that are not joined and are counted),
//           their rows are gathered straight into MFMA operand registers,
//           the Gram tile new x all is formed on MFMA (32x32x16 BF16 / FP16,
//           or 32x32x2 FP32 for the plain form), and each member receives at
//           most `join_cap` of its best partners that beat its current worst
//           distance, as atomicMin keys into C hashed candidate slots;
//  merge    half a wave per row: the K_b list keys and the C slot keys are
//           deduplicated by index and merged, the first K_b kept; slot
//           entries that enter are flagged new and counted; slots are reset;
//           the row is then sampled for the next iteration (sample_row: up to
//           s = ceil(rho K_b) new entries picked by a per-row random order
//           and marked old, the old entries listed, and both scattered as
//           reverse edges into T hashed slots of the target rows by
//           atomicMin on codes that do not depend on thread order);
//  revsample  before each join (when T > s), per row and list, the s
//           filled reverse slots with the least codes are kept (an
//           s-sample, like the forward one) and the slots emptied; with
//           T = s the join reads and empties the table itself;
//  (host)   stop when updates < delta * n * K_b.
//
// The init kernel builds the first lists (random, given or encoder-seeded)
// and samples the first iteration the same way.  finalize re-ranks the K_b
// entries with FP32 direct differences on the input values and returns the
// first k.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "knn_common.hpp"

namespace knn {

knn_status stage_matrix(ScratchAlloc& ws, const knn_matrix& X, int kind, void** Xs, int* ldp,
                        float** norms, unsigned* maxnorm, hipStream_t st, const uint32_t* rowmap,
                        int aux);
knn_status morton_order(const knn_matrix& X, int D, uint64_t seed, Workspace& ws, uint32_t** perm,
                        uint32_t** inv, hipStream_t st);

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Old (already joined) list entries carry this bit in the index word of
// their sort keys; indices stay below 2^31 - 1.
constexpr uint32_t kWasOld = 1u << 31;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Arguments of the sampling that the init and merge kernels run for the
// iteration that follows them (see sample_row).
struct SampleArgs {
    int s, R;
    int32_t* newf;
    int32_t* oldf;
    uint32_t* revnew;
    uint32_t* revold;
    uint64_t seed;
    int iter;
};

__device__ inline bool sample_row(int64_t row, bool rv, int K, int s, int R, int32_t id, bool isnew, bool isold,
                                  int32_t* __restrict__ newf, int32_t* __restrict__ oldf,
                                  uint32_t* __restrict__ revnew, uint32_t* __restrict__ revold,
                                  uint64_t seed, int iter);

// ------------------------------------------------------------------ init

// One wave per row: entries from init_idx (nullable; invalid, self and
// repeated entries dropped), completed with distinct uniform random indices,
// distances (given, or canonical direct differences on the staged rows),
// sorted, first K kept.  Flags: given (or new).  The K-th distance is also
// written to the row's worst-distance word (worst[row * wstride]).  With
// smp the row is then sampled for the first iteration (sample_row).  The
// row's C candidate slots are emptied.
template <int DT>
__global__ __launch_bounds__(256) void nnd_init_kernel(
    int64_t n, int K, const void* __restrict__ Xs, int64_t ldp, int d,
    const int32_t* __restrict__ init_idx, const float* __restrict__ init_dist,
    const uint8_t* __restrict__ init_flags, int init_k, uint64_t seed,
    int32_t* __restrict__ gidx, float* __restrict__ gd2, uint8_t* __restrict__ gflag,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ inv, float* __restrict__ worst,
    int64_t wstride, SampleArgs sa, bool smp, unsigned long long* __restrict__ cand, int C)
{
    __shared__ __attribute__((aligned(16))) uint32_t s_id[4][64];
    __shared__ float s_d2[4][64];
    __shared__ uint8_t s_fl[4][64];
    __shared__ uint8_t s_has[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + wv;
    if (row >= n) return;

    // 1. given entries
    uint32_t id = 0xFFFFFFFFu;
    bool valid = false;
    float gd = 0.0f;
    uint8_t fl = 1;
    bool hasd = false;
    // lists given in input order are read at the row's input position and
    // their entries mapped to processing order
    const int64_t grow = perm ? (int64_t)perm[row] : row;
    if (init_idx && lane < init_k) {
        int32_t v = init_idx[grow * init_k + lane];
        if (v >= 0 && v < n && v != grow) {
            id = inv ? inv[v] : (uint32_t)v;
            valid = true;
            if (init_dist) {
                gd = init_dist[grow * init_k + lane];
                hasd = true;
            }
            if (init_flags) fl = init_flags[grow * init_k + lane] ? 1 : 0;
        }
    }
    // drop repeats (keep the first valid occurrence): every lane compares
    // with the earlier lanes through LDS broadcasts; only lanes < init_k hold
    // given entries, invalid ones a value no index takes
    const int ngiven = init_idx ? (init_k < 64 ? init_k : 64) : 0;
    if (ngiven > 1) {
        s_id[wv][lane] = valid ? id : 0xFFFFFFFEu;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        bool dup = false;
        for (int o = 0; o < ngiven; o += 4) {
            const uint4 x = *(const uint4*)&s_id[wv][o];
            dup = dup || (o + 0 < lane && x.x == id) || (o + 1 < lane && x.y == id) ||
                  (o + 2 < lane && x.z == id) || (o + 3 < lane && x.w == id);
        }
        valid = valid && !dup;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    uint64_t vm = ballot(valid);
    int nvalid = popc64(vm);
    int pos = rank_below(vm);
    if (valid) {
        s_id[wv][pos] = id;
        s_d2[wv][pos] = gd;
        s_fl[wv][pos] = fl;
        s_has[wv][pos] = hasd ? 1 : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

    // 2. compact into lanes; fill the rest of 0..K-1 at random
    const int have = nvalid;
    id = lane < have ? s_id[wv][lane] : 0xFFFFFFFFu;
    gd = lane < have ? s_d2[wv][lane] : 0.0f;
    fl = lane < have ? s_fl[wv][lane] : 1;
    hasd = lane < have ? (s_has[wv][lane] != 0) : false;
    bool ok = lane < have;
    const int want = K;   // entries needed
    if (have < want) {
        const uint32_t m = (uint32_t)(n - 1);
        if (n - 1 <= 2 * (int64_t)K) {
            // tiny n: take a random rotation of the other points, skipping given ones
            uint32_t start = bounded(hash4(seed ^ kTagInit, (uint64_t)row, 0xFFFFFFFFull, 0), m);
            int filled = have;
            for (uint32_t t = 0; t < m && filled < want; ++t) {
                uint32_t cand = (uint32_t)((row + 1 + (start + t) % m) % n);
                bool dup = false;
                for (int o = 0; o < filled; ++o) dup |= bcast_u32(id, o) == cand;
                if (!dup) {
                    if (lane == filled) {
                        id = cand;
                        ok = true;
                        fl = 1;
                        hasd = false;
                    }
                    ++filled;
                }
            }
        } else {
            uint32_t attempt = 0;
            while (ballot(lane < want && !ok) && attempt < 4096) {
                if (lane < want && !ok) {
                    uint64_t r = hash4(seed ^ kTagInit, (uint64_t)row, (uint64_t)lane, attempt);
                    id = bounded(r, (uint32_t)n);
                }
                bool dup = false;
                for (int o = 0; o < want; ++o) {
                    uint32_t oi = bcast_u32(id, o);
                    bool ook = bcast_u32(ok ? 1u : 0u, o) != 0;
                    dup |= (o != lane) && oi == id && (ook || o < lane);
                }
                if (lane < want && !ok) {
                    ok = (id != (uint32_t)row) && !dup;
                    fl = 1;
                    hasd = false;
                }
                ++attempt;
            }
            if (lane < want && !ok) id = 0xFFFFFFFFu;
        }
    }
    // 3. distances for entries without one (entry e's lands in lane e)
    const int cnt = have > want ? have : want;
    const bool need = lane < cnt && !hasd && id != 0xFFFFFFFFu;
    float dd = 0.0f;
    if (ballot(need)) {   // seeded lists arrive with their distances
        dd = dist_batch16<DT, 8>(Xs, ldp, row, id, need, d);
        if (cnt > 32) dd += dist_batch16<DT, 8>(Xs, ldp, row, id, need, d, 32);
    }
    const float mine = need ? dd : gd;
    // 4. sort by (d2, old after new, id) -- the merge's list order -- and keep
    //    the first K; the old flag rides in the index word
    const bool live = lane < cnt && id != 0xFFFFFFFFu;
    const uint64_t key = live ? make_key(mine, id | (fl ? 0u : kWasOld)) : kEmptyCand;
    const uint64_t sk = seg_sort<64>(key);
    const uint8_t sfl = (key_idx(sk) & kWasOld) ? 0 : 1;
    const bool sv = lane < K && key_valid(sk);
    // 5. with smp, the first iteration's sampling of the row (K <= 32: the
    //    row is the first half-wave's), picks stored old
    bool pick = false;
    if (smp) {
        const int32_t eid = (int32_t)(key_idx(sk) & ~kWasOld);
        pick = sample_row(row, lane < 32, K, sa.s, sa.R, eid, sv && sfl, sv && !sfl, sa.newf, sa.oldf, sa.revnew,
                          sa.revold, sa.seed, sa.iter);
    }
    if (lane < K) {
        gidx[row * K + lane] = sv ? (int32_t)(key_idx(sk) & ~kWasOld) : -1;
        gd2[row * K + lane] = sv ? key_d2(sk) : __builtin_inff();
        gflag[row * K + lane] = sv && !pick ? sfl : 0;
        if (lane == K - 1) worst[row * wstride] = sv ? key_d2(sk) : __builtin_inff();
    }
    // 6. the row's candidate slots start empty (only the joins touch them)
    for (int c = lane; c < C; c += 64) cand[row * C + c] = kEmptyCand;
}

// ---------------------------------------------------------------- sample

// Sampling runs inside the kernels that produce a row's list: the init
// kernel samples the first iteration and each merge the next one, so that
// the sampling's random reverse-slot atomics overlap their other work.
//
// Reverse-slot codes.  A reverse slot of point v holds, as a 32-bit word,
// the least code among the sources u that picked that slot this iteration:
// code = mix(u ^ salt(v)), where mix is an invertible 32-bit mixer and the
// salt is drawn from (seed, stream tag, iteration, v).  The minimum over
// codes is a pseudo-random choice among the sources, fresh per point and
// iteration, and the join recovers u = unmix(code) ^ salt(v).  The empty
// slot is 0xFFFFFFFF (a source whose code is that value, one chance in 2^32,
// is not recorded).  The mixer is Wellons' "lowbias32" from his
// hash-prospector search; the inverse undoes each xor-shift and multiplies
// by the multipliers' inverses modulo 2^32.
__host__ __device__ inline uint32_t rev_mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

__host__ __device__ inline uint32_t rev_unmix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x43021123u;   // inverse of 0x846CA68B modulo 2^32
    x ^= (x >> 15) ^ (x >> 30);
    x *= 0x1D69E2A5u;   // inverse of 0x7FEB352D modulo 2^32
    x ^= x >> 16;
    return x;
}

__host__ __device__ inline uint32_t rev_salt(uint64_t seed, uint64_t tag, int iter, int64_t v)
{
    return (uint32_t)hash4(seed ^ tag, (uint64_t)iter, (uint64_t)v, 3);
}

__host__ __device__ inline uint32_t rev_code(uint32_t u, uint32_t salt) { return rev_mix(u ^ salt); }

// Sampling of one row held by a half-wave (lane hl of the half holds entry
// hl; `isnew` / `isold` mark the valid new and old entries): picks the new
// entries (every one when there are at most s, else the s with the smallest
// random priorities, ties by position), writes them in list order to
// newf(row) and the old entries to oldf(row), -1 past the last, and scatters
// the reverse edges into R (= T) slots per target row.  All reverse edges of one
// source and list use the slot index hash(iteration, source), so a source
// occupies at most one slot of a target's reverse list: the join's repeat
// check relies on this.  Returns whether this lane's entry was picked (the
// caller marks it old).
__device__ inline bool sample_row(int64_t row, bool rv, int K, int s, int R, int32_t id, bool isnew, bool isold,
                                  int32_t* __restrict__ newf, int32_t* __restrict__ oldf,
                                  uint32_t* __restrict__ revnew, uint32_t* __restrict__ revold,
                                  uint64_t seed, int iter)
{
    const int lane = threadIdx.x & 63, hl = lane & 31, hbase = lane & 32;
    const uint64_t nm = ballot(isnew), om = ballot(isold);
    const uint64_t hn = hbase ? (nm >> 32) : (nm & 0xFFFFFFFFull);
    const uint64_t ho = hbase ? (om >> 32) : (om & 0xFFFFFFFFull);
    // the rank loop runs only for a wave that has a row with more than s
    // new entries
    bool pick = isnew;
    if (ballot(__popcll(hn) > (uint64_t)s)) {
        const uint64_t pr = isnew ? hash4(seed ^ kTagSample, (uint64_t)iter, (uint64_t)row, (uint64_t)id)
                                  : ~0ull;
        int prank = 0;
        for (int o = 0; o < 32; ++o) {
            const uint64_t p0 = bcast_u64(pr, o), p1 = bcast_u64(pr, 32 + o);
            const uint64_t po = hbase ? p1 : p0;
            prank += (po < pr || (po == pr && o < hl)) ? 1 : 0;
        }
        pick = isnew && prank < s;
    }
    // picks are written in list order
    const uint64_t pm = ballot(pick);
    const uint64_t hp = hbase ? (pm >> 32) : (pm & 0xFFFFFFFFull);
    const int rank = __popcll(hp & ((1ull << hl) - 1ull));
    const int npick = __popcll(hn) < s ? __popcll(hn) : s;
    const int nold = __popcll(ho);
    const int opos = __popcll(ho & ((1ull << hl) - 1ull));
    // slots past the picks / old entries get -1 (disjoint from the writes below)
    if (rv && hl >= npick && hl < s) newf[row * s + hl] = -1;
    if (rv && hl >= nold && hl < K) oldf[row * K + hl] = -1;
    if (pick) newf[row * s + rank] = id;
    if (isold) oldf[row * K + opos] = id;
    // one reverse edge per picked or old entry: the list, slot stream and
    // salt are chosen first, so a wave evaluates each hash once
    if (pick || isold) {
        const uint32_t slot =
            bounded(hash4(seed ^ kTagRevSlot, (uint64_t)iter, (uint64_t)row, pick ? 1u : 2u), (uint32_t)R);
        uint32_t* rev = pick ? revnew : revold;
        const uint32_t salt = rev_salt(seed, pick ? kTagRevNew : kTagRevOld, iter, id);
        atomicMin(&rev[(int64_t)id * R + slot], rev_code((uint32_t)row, salt));
    }
    return pick;
}

// Undoes the flag changes of a sampling whose iteration is not run: an
// entry of row v that is listed in newf(v) was new before it was picked.
// Half-wave per row.
__global__ __launch_bounds__(256) void nnd_unsample_kernel(int64_t n, int K, int s, const int32_t* __restrict__ gidx,
                                                           uint8_t* __restrict__ gflag,
                                                           const int32_t* __restrict__ newf)
{
    const int lane = threadIdx.x & 63, hl = lane & 31, hbase = lane & 32;
    const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 5;
    if (row >= n) return;   // uniform per half-wave; the shuffles below read the own half only
    const int32_t id = hl < K ? gidx[row * K + hl] : -1;
    const int32_t nf = hl < s ? newf[row * s + hl] : -1;
    bool was = false;
    for (int j = 0; j < s; ++j) {
        const int32_t x = (int32_t)shfl_u32((uint32_t)nf, hbase + j);
        was = was || (id >= 0 && x == id);
    }
    if (was) gflag[row * K + hl] = 1;
}

// Reverse samples.  The sampling scatters each iteration's reverse edges
// into a table of T hashed slots per row and list; this pass keeps, per row
// and list, the (at most) s filled slots with the least codes -- the codes
// are salted bijections of the sources, so that is a pseudo-random choice of
// s reverse edges, as the forward new list is an s-sample -- writes them in
// slot order to samp (s words, 0xFFFFFFFF past the last) and empties the
// table for the next scatter.  One wave per row, lane = slot.
__global__ __launch_bounds__(256) void nnd_revsample_kernel(int64_t n, int s, int T, uint32_t* __restrict__ revnew,
                                                            uint32_t* __restrict__ revold,
                                                            uint32_t* __restrict__ sampnew,
                                                            uint32_t* __restrict__ sampold)
{
    const int lane = threadIdx.x & 63;
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;   // the whole wave
#pragma unroll
    for (int l = 0; l < 2; ++l) {
        uint32_t* tab = l ? revold : revnew;
        uint32_t* out = l ? sampold : sampnew;
        const uint32_t c = lane < T ? tab[v * T + lane] : 0xFFFFFFFFu;
        if (lane < T) tab[v * T + lane] = 0xFFFFFFFFu;
        bool keep = c != 0xFFFFFFFFu;
        const uint64_t m = ballot(keep);
        if (popc64(m) > s) {
            int rank = 0;
            for (uint64_t b = m; b; b &= b - 1) rank += bcast_u32(c, __builtin_ctzll(b)) < c ? 1 : 0;
            keep = keep && rank < s;
        }
        const uint64_t km = ballot(keep);
        const int kept = popc64(km);
        if (keep) out[v * s + rank_below(km)] = c;
        if (lane >= kept && lane < s) out[v * s + lane] = 0xFFFFFFFFu;
    }
}

// ------------------------------------------------------------------ join

struct JoinCfg {
    int s, R, K, C, J;     // new sample, reverse entries (= s), list size, candidate slots, cap
    int reset;             // the reverse entries are the hashed table itself (T = s): empty them after reading
    int lcap;              // max join-list length, <= 64
    int ncap;              // max new-list length
};

constexpr int kJMax = 4;         // largest supported join cap

// Raw join-list entries of one lane: lanes 0..s-1 hold new_f(v), lanes
// s..s+R-1 (R = s) the codes of the reverse-new sample, and likewise
// old_f(v) / reverse-old in `o`; 0xFFFFFFFF marks an empty entry (a -1 forward entry,
// or an empty slot).  Loaded ahead of the join that consumes them.  Every
// lane loads from an in-bounds address (lanes past s+R or K+R re-read a
// slot, and a point past the range reads row 0) and join_lists masks the
// lanes it does not use: one load per list with no branch, so a load still
// in flight never forces a wait on the others.
struct ListRaw {
    uint32_t n, o;
};

__device__ inline ListRaw load_lists(int64_t v, bool valid, const JoinCfg& cfg,
                                     const int32_t* __restrict__ newf,
                                     const uint32_t* __restrict__ revnew,
                                     const int32_t* __restrict__ oldf,
                                     const uint32_t* __restrict__ revold)
{
    const int lane = threadIdx.x;
    const int64_t vv = valid ? v : 0;
    const int rn = min(max(lane - cfg.s, 0), cfg.R - 1), ro = min(max(lane - cfg.K, 0), cfg.R - 1);
    const uint32_t* pn = lane < cfg.s ? (const uint32_t*)(newf + vv * cfg.s + lane) : revnew + vv * cfg.R + rn;
    const uint32_t* po = lane < cfg.K ? (const uint32_t*)(oldf + vv * cfg.K + lane) : revold + vv * cfg.R + ro;
    return {*pn, *po};
}

// Per-point join lists from the raw entries.  The reverse entries are
// either the s-samples nnd_revsample_kernel rewrites before every join or,
// when the table has only s slots (cfg.reset), the table itself, whose
// slots are emptied here for the next iteration.  Repeats are dropped (first position wins), an id
// in both lists stays new, v itself is dropped.  Every lane compares its
// entries with all 128 through LDS broadcast reads (sh: 128 words).  The
// surviving ids are written to ids[0..nn) (new) and ids[nn..nn+no) (old);
// members beyond the caps (old ones first: the list is cut at lcap) are not
// joined and are counted in `dropped`.  Returns nn, sets L.
__device__ inline int join_lists(int64_t v, const ListRaw& raw, const JoinCfg& cfg,
                                 uint32_t* __restrict__ revnew, uint32_t* __restrict__ revold,
                                 uint64_t seed, int iter, uint32_t* sh, uint32_t* ids, int& L, int& dropped)
{
    const int lane = threadIdx.x;
    if (cfg.reset) {
        if (lane >= cfg.s && lane < cfg.s + cfg.R) revnew[v * cfg.R + (lane - cfg.s)] = 0xFFFFFFFFu;
        if (lane >= cfg.K && lane < cfg.K + cfg.R) revold[v * cfg.R + (lane - cfg.K)] = 0xFFFFFFFFu;
    }
    // reverse samples hold codes: recover the source ids
    const uint32_t sn = rev_salt(seed, kTagRevNew, iter, v), so = rev_salt(seed, kTagRevOld, iter, v);
    const uint32_t rn = raw.n == 0xFFFFFFFFu ? raw.n : rev_unmix(raw.n) ^ sn;
    const uint32_t ro = raw.o == 0xFFFFFFFFu ? raw.o : rev_unmix(raw.o) ^ so;
    const uint32_t nid = lane < cfg.s ? raw.n : (lane < cfg.s + cfg.R ? rn : 0xFFFFFFFFu);
    const uint32_t oid = lane < cfg.K ? raw.o : (lane < cfg.K + cfg.R ? ro : 0xFFFFFFFFu);
    sh[lane] = nid;
    sh[64 + lane] = oid;
    __syncthreads();
    int ln = lane;
    asm volatile("" : "+v"(ln));   // keep the position tests per point, not hoisted masks
    bool nv = nid != 0xFFFFFFFFu && nid != (uint32_t)v;
    bool ov = oid != 0xFFFFFFFFu && oid != (uint32_t)v;
    // Repeats keep their first position.  A forward list holds distinct
    // indices, and a reverse list holds a source at most once (a source
    // uses one slot index for all its targets), so a new entry can repeat
    // only a forward-new one (lanes < s), and an old entry a new one or,
    // if it is a reverse-old entry, a forward-old one (lanes < K).
#pragma unroll 2
    for (int q = 0; q < 64; q += 4) {
        const uint4 x = *(const uint4*)(sh + q);
        if (q < cfg.s)
            nv = nv && !(q + 0 < ln && x.x == nid) && !(q + 1 < ln && x.y == nid) &&
                 !(q + 2 < ln && x.z == nid) && !(q + 3 < ln && x.w == nid);
        ov = ov && x.x != oid && x.y != oid && x.z != oid && x.w != oid;
    }
    for (int q = 0; q < cfg.K; q += 4) {
        const uint4 x = *(const uint4*)(sh + 64 + q);
        ov = ov && !(q + 0 < ln && x.x == oid) && !(q + 1 < ln && x.y == oid) &&
             !(q + 2 < ln && x.z == oid) && !(q + 3 < ln && x.w == oid);
    }
    const uint64_t nm = ballot(nv), om = ballot(ov);
    int nn = popc64(nm), no = popc64(om);
    const int all = nn + no;
    if (nn > cfg.ncap) nn = cfg.ncap;
    if (nn + no > cfg.lcap) no = cfg.lcap - nn;
    dropped = all - nn - no;
    const int pn = rank_below(nm), po = rank_below(om);
    if (nv && pn < nn) ids[pn] = nid;
    if (ov && po < no) ids[nn + po] = oid;
    L = nn + no;
    return nn;
}

// Selection keys of the join epilogue: the FP32 bits of a squared distance
// (non-negative, so unsigned order is numeric order) with the low 6 bits
// replaced by the partner's position in the join list.  The truncation is a
// relative 2^-17 of the distance, below the error of the norm-expansion
// distances it orders; ties go to the lower position.
constexpr uint32_t kNoSel = 0xFFFFFFFFu;

// Keep the kJMax smallest keys (ascending).  With the list sorted, the new
// entry q is the median of old entries q-1, q and the key (the minimum of
// old entry 0 and the key for q = 0): one independent min or 3-input median
// (v_med3_u32) per slot.
__device__ inline uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ inline void sel_insert(uint32_t (&best)[kJMax], uint32_t key)
{
    static_assert(kJMax == 4, "four slots");
    const uint32_t b0 = best[0], b1 = best[1], b2 = best[2], b3 = best[3];
    best[0] = min(b0, key);
    best[1] = med3_u32(b0, b1, key);
    best[2] = med3_u32(b1, b2, key);
    best[3] = med3_u32(b2, b3, key);
}

// Keep the kJMax smallest of two ascending lists: min(a[q], b[3-q]) holds
// them as a bitonic sequence, which two compare-exchange stages sort.
__device__ inline void sel_merge(uint32_t (&best)[kJMax], const uint32_t (&other)[kJMax])
{
    static_assert(kJMax == 4, "four slots");
    const uint32_t m0 = min(best[0], other[3]), m1 = min(best[1], other[2]);
    const uint32_t m2 = min(best[2], other[1]), m3 = min(best[3], other[0]);
    const uint32_t p0 = min(m0, m2), p2 = max(m0, m2), p1 = min(m1, m3), p3 = max(m1, m3);
    best[0] = min(p0, p1);
    best[1] = max(p0, p1);
    best[2] = min(p2, p3);
    best[3] = max(p2, p3);
}

// Offers whose slot reads are in flight: a column pass issues them (key,
// slot address, read of the slot) and the next pass -- after its own MFMA
// and selection work -- resolves them with atomicMin where the slot still
// holds a larger key, so the read latency overlaps computation.  Each lane
// carries up to two offers (its member's positions q = h and h + 2).
struct PendingOffers {
    unsigned long long* p[2];
    uint64_t key[2];
    unsigned long long seen[2];
};

__device__ inline void offers_issue(PendingOffers& po, const uint32_t (&best)[kJMax], int J, int h, bool valid,
                                    float cut, const uint32_t* ids, uint32_t me, int C, uint64_t salt,
                                    unsigned long long* __restrict__ cand)
{
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int q = h + 2 * t;
        const uint32_t b = t == 0 ? (h ? best[1] : best[0]) : (h ? best[3] : best[2]);
        po.p[t] = nullptr;
        po.key[t] = ~0ull;
        po.seen[t] = 0ull;
        if (valid && q < J && b != kNoSel && __uint_as_float(b & ~63u) < cut) {
            const uint32_t src = ids[b & 63u];
            po.key[t] = ((uint64_t)(b & ~63u) << 32) | src;
            const uint32_t slot = bounded(mix64(((uint64_t)src << 20) ^ salt), (uint32_t)C);
            po.p[t] = &cand[(int64_t)me * C + slot];
            po.seen[t] = *po.p[t];
        }
    }
}

// A slot read that holds another source's key is a collision: one of the
// two candidates is lost (counted from the pre-check read, so collisions
// between offers racing for one slot are not seen).
__device__ inline bool slot_collides(unsigned long long seen, uint64_t key)
{
    return seen != kEmptyCand && (uint32_t)seen != (uint32_t)key;
}

// Returns the offers sent in the low 32 bits and the collisions seen in the
// high 32.
__device__ inline unsigned long long offers_resolve(const PendingOffers& po)
{
    unsigned long long n = 0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (po.p[t] && slot_collides(po.seen[t], po.key[t])) n += 1ull << 32;
        if (po.p[t] && po.seen[t] > (unsigned long long)po.key[t]) {
            atomicMin(po.p[t], (unsigned long long)po.key[t]);
            ++n;
        }
    }
    return n;
}

// Local join on MFMA, every form (OUT is the staged element type: KNN_F32,
// KNN_BF16 or KNN_F16).  One wave per point v; the grid is split into 8
// groups (blockIdx mod 8, the round-robin XCD assignment of workgroups) that
// each sweep one contiguous range of the processing order, so concurrently
// joined points are Z-order neighbours sharing an L2.
//
// The join list (new members first, then old; L <= 64) is two 32-row
// blocks.  Its L x L Gram is accumulated by 32 x 32 MFMA tiles (FP32
// accumulation) whose operands come straight from the staged rows into
// registers, no LDS copy: lane (h, c) holds 16-byte pieces of rows c and
// 32 + c; piece p covers bytes [32p + 16h, +16) (8 BF16 / FP16 elements, or
// 4 FP32 ones taken by four 32x32x2 steps).  That assigns the reduction
// index to (step, half) one-to-one, which is all a Gram product needs since
// both operands use the same assignment.
//
// Column block cb (members 32cb + c) is finished before the next starts, so
// two accumulator tiles are live.  Member m pairs with every row if it is
// new and with the new rows if it is old; each lane keeps the best J of its
// 32 rows that beat m's current worst distance, the two lanes of column m
// swap and merge their lists, and each offers half of the merged best J.
//
// Row padding is zero except the last 8 bytes: the row's norm (of the stored
// values) and the current worst distance of its list, read once per member
// and zeroed in the operand piece that holds them.
constexpr int kPC = 4;   // pieces per lane per row held in registers at a time

typedef float f32x16 __attribute__((ext_vector_type(16)));

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// The Gram work of one 16-byte piece pair, FP32 accumulation: one 32x32x16
// MFMA step on 16-bit operands (OUT = KNN_BF16 / KNN_F16, the staged element
// type), or four 32x32x2 FP32 steps (OUT = KNN_F32: the piece's four floats
// in turn; with the other half-wave's four, each step sums two elements, so
// every element of the 32-byte piece enters once).
template <int OUT>
__device__ inline f32x16 gram_step(const uint4& a, const uint4& b, f32x16 acc)
{
    if constexpr (OUT == KNN_F32) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
    } else if constexpr (OUT == KNN_F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b),
                                                       acc, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                        acc, 0, 0, 0);
}

// Piece p of a row (r = row base + 16h bytes): the load always reads inside
// the row (p clamped; an absent row points at a listed row).  Values of
// absent rows and of pieces past the data only reach Gram entries that the
// selection and the offers never use, so they are not cleared; the
// trailing norm / worst-distance words are (clear_tail), after all of a
// chunk's loads are issued, and clear_tail stores them to the row's norm
// and threshold slots in LDS: the gather itself delivers them.
__device__ inline uint4 load_piece(const uint8_t* r, int p, int np)
{
    const int pp = p < np ? p : np - 1;
    return *(const uint4*)(r + 32 * (int64_t)pp);
}

__device__ inline void clear_tail(uint4& x, int p, int np, int64_t rowbytes, int h, float* nrm, float* thr)
{
    if (p < np && 32 * (int64_t)p + 16 * h + 16 == rowbytes) {
        *nrm = __uint_as_float(x.z);
        *thr = __uint_as_float(x.w);
        x.z = 0u;
        x.w = 0u;
    }
}

// Candidates of member m from one 32-row block's accumulator column: rows
// 32 blk + 8 (e / 4) + 4 h + e % 4 of tile entry e, branch-free.  Member m
// pairs with rows i < lim (L if m is new, nn if it is old), i != m.  Groups
// of 8 rows at or past rows_end (the same for the whole wave) are skipped.
__device__ inline void scan_block(const f32x16& g, int blk, int h4, int m, int lim, int rows_end, float nm,
                                  const float* nrm, uint32_t (&best)[kJMax])
{
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {
        if (32 * blk + 8 * e4 >= rows_end) break;
        const int i0 = 32 * blk + 8 * e4 + h4;
        const f32x4 ni = *(const f32x4*)(nrm + i0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = i0 + e;
            float d2 = ni[e] + nm - 2.0f * g[4 * e4 + e];
            d2 = d2 > 0.0f ? d2 : 0.0f;
            const bool ok = i < lim && i != m;
            sel_insert(best, ok ? ((__float_as_uint(d2) & ~63u) | (uint32_t)i) : kNoSel);
        }
    }
}

template <int OUT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void nnd_join_mfma_kernel(
    int64_t n, JoinCfg cfg, const uint8_t* __restrict__ Xr, int64_t rowbytes, int np,
    const int32_t* __restrict__ newf, uint32_t* __restrict__ revnew,
    const int32_t* __restrict__ oldf, uint32_t* __restrict__ revold,
    unsigned long long* __restrict__ cand, uint64_t seed, int iter, unsigned long long* __restrict__ counters)
{
    __shared__ uint32_t ids[64];
    __shared__ __attribute__((aligned(16))) float nrm[64];
    __shared__ float thr[64];
    __shared__ __attribute__((aligned(16))) uint32_t sh[128];
    const int lane = threadIdx.x, c = lane & 31, h = lane >> 5;
    // emitted: offers in the low 32 bits, slot collisions in the high 32 (a
    // lane sends far fewer than 2^32 offers), so one register pair counts both
    unsigned long long emitted = 0;
    // wave-uniform tallies (rows gathered, pairs joined, members cut) live in
    // LDS, updated by lane 0, so that they hold no registers in the loop
    __shared__ unsigned long long tally[3];
    if (threadIdx.x == 0) tally[0] = tally[1] = tally[2] = 0ull;
    const uint64_t salt = (uint64_t)iter ^ seed;
    const int J = cfg.J;
    const int nch = (np + kPC - 1) / kPC;
    const bool tail_in_pieces = 32 * (int64_t)np == rowbytes;   // the last piece holds the norm / worst words
    const unsigned grp = blockIdx.x & 7u;
    const int64_t gsz = (int64_t)(gridDim.x >> 3);
    const int64_t lo = n * grp / 8, hi = n * (grp + 1) / 8;

    PendingOffers po;
    po.p[0] = po.p[1] = nullptr;
    int64_t v = lo + (int64_t)(blockIdx.x >> 3);
    ListRaw cur = load_lists(v, v < hi, cfg, newf, revnew, oldf, revold);
    for (; v < hi; v += gsz) {
        int L = 0, dr = 0;
        const int nn = __builtin_amdgcn_readfirstlane(join_lists(v, cur, cfg, revnew, revold, seed, iter, sh, ids, L, dr));
        if (threadIdx.x == 0) tally[2] += (unsigned long long)dr;
        L = __builtin_amdgcn_readfirstlane(L);
        // the next point's lists are in flight while this one is joined
        cur = load_lists(v + gsz, v + gsz < hi, cfg, newf, revnew, oldf, revold);
        __syncthreads();
        if (nn == 0 || L < 2) continue;
        if (threadIdx.x == 0) {
            tally[0] += (unsigned long long)L;
            tally[1] += (unsigned long long)(nn * (nn - 1) / 2 + nn * (L - nn));
        }
        if (!tail_in_pieces && lane < L) {
            // rows whose trailing words lie past the gathered pieces
            const float2 a = *(const float2*)(Xr + (int64_t)ids[lane] * rowbytes + rowbytes - 8);
            nrm[lane] = a.x;
            thr[lane] = a.y;
        }
        const bool two = L > 32;
        const bool v0 = c < L, v1 = 32 + c < L;
        const uint8_t* r0 = Xr + (int64_t)ids[v0 ? c : 0] * rowbytes + 16 * h;
        const uint8_t* r1 = Xr + (int64_t)ids[v1 ? 32 + c : 0] * rowbytes + 16 * h;
        uint4 A0[kPC], A1[kPC];
        for (int cb = 0; cb < (two ? 2 : 1); ++cb) {
            // rows 32..63 x members 32..63 pair old with old when every new
            // member is in the first block
            const bool lower = two && (cb == 0 || nn > 32);
            float z = 0.0f;
            asm volatile("" : "+v"(z));   // one zero register per pass, not sixteen held ones
            f32x16 at, ab;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                at[e] = z;
                ab[e] = z;
            }
            for (int ch = 0; ch < nch; ++ch) {
                if (cb == 0 || nch > 1) {
#pragma unroll
                    for (int q = 0; q < kPC; ++q) A0[q] = load_piece(r0, ch * kPC + q, np);
                    if (two) {
#pragma unroll
                        for (int q = 0; q < kPC; ++q) A1[q] = load_piece(r1, ch * kPC + q, np);
                    }
#pragma unroll
                    for (int q = 0; q < kPC; ++q) clear_tail(A0[q], ch * kPC + q, np, rowbytes, h, nrm + c, thr + c);
                    if (two) {
#pragma unroll
                        for (int q = 0; q < kPC; ++q)
                            clear_tail(A1[q], ch * kPC + q, np, rowbytes, h, nrm + 32 + c, thr + 32 + c);
                    }
                }
                const int pc = min(kPC, np - ch * kPC);
#pragma unroll
                for (int q = 0; q < kPC; ++q) {
                    if (q < pc) {
                        const uint4 b = cb == 0 ? A0[q] : A1[q];
                        at = gram_step<OUT>(A0[q], b, at);
                        if (lower) ab = gram_step<OUT>(A1[q], b, ab);
                    }
                }
            }
            __syncthreads();   // the norms and thresholds stored from the gathered rows
            // lane-dependent indices are re-derived per point (an opaque copy
            // of the lane id) so that they are not held across the loop
            int ln = lane;
            asm volatile("" : "+v"(ln));
            const int m = 32 * cb + (ln & 31), h4 = (ln >> 5) * 4;
            uint32_t best[kJMax];
#pragma unroll
            for (int q = 0; q < kJMax; ++q) best[q] = kNoSel;
            const float nm = nrm[m];
            const int lim = m < nn ? L : nn;
            // a pass whose members are all old needs only the first nn rows
            const int rows_end = 32 * cb >= nn ? nn : L;
            scan_block(at, 0, h4, m, lim, rows_end, nm, nrm, best);
            if (lower) scan_block(ab, 1, h4, m, lim, rows_end, nm, nrm, best);
            uint32_t recv[kJMax];
#pragma unroll
            for (int q = 0; q < kJMax; ++q) recv[q] = xor_u32(best[q], 32);
            sel_merge(best, recv);
            emitted += offers_resolve(po);
            offers_issue(po, best, J, h, m < L, m < L ? thr[m] : 0.0f, ids, ids[m], cfg.C, salt, cand);
        }
    }
    emitted += offers_resolve(po);
    unsigned long long coll = emitted >> 32;
    emitted &= 0xFFFFFFFFull;
    for (int o = 32; o > 0; o >>= 1) {
        emitted += shfl_u64(emitted, lane ^ o);
        coll += shfl_u64(coll, lane ^ o);
    }
    if (lane == 0) {
        atomicAdd(&counters[1], emitted);
        atomicAdd(&counters[2], tally[0]);
        atomicAdd(&counters[3], coll);
        atomicAdd(&counters[4], tally[2]);
        atomicAdd(&counters[5], tally[1]);
    }
}

// ------------------------------------------------------------------ merge

// Merge, one half-wave (32 lanes) per row, two rows per wave; the waves take
// row pairs from 8 contiguous ranges (blockIdx mod 8, as in the sample
// kernel; gridDim.x is a multiple of 8), the next pair's list and first 96
// slots loaded while the current pair is merged.  Lane hl < K holds list
// entry hl.  The C candidate slots are read 32 at a time (and reset); keys
// whose index is already listed (or is the row) are dropped, the rest are
// compacted into LDS.  Up to 8 survivors are inserted one at a time; more
// are sorted 32 at a time and merged into the list by keeping the 32
// smallest of the two sorted halves (a bitonic clean), so the first K lanes
// stay the list.  Old list entries carry kWasOld in the index word, so
// lists are ordered by (distance, old after new, index) -- the order the
// init kernel also sorts by, which makes a resumed run bitwise equal to an
// uninterrupted one.  Entries whose index is not in the previous list came
// from slots: flagged new and counted.  The new K-th distance goes to the
// row's worst-distance word.  With Smp the merged row is also sampled for
// the next iteration (sample_row, the picks stored old), so that the
// reverse-slot atomics of the sampling overlap the merge work of other
// waves; every row is then rewritten.
template <bool Smp>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void nnd_merge_kernel(
    int64_t n, int K, int C, int32_t* __restrict__ gidx, float* __restrict__ gd2,
    uint8_t* __restrict__ gflag, unsigned long long* __restrict__ cand,
    unsigned long long* __restrict__ counters, float* __restrict__ worst, int64_t wstride,
    SampleArgs sa)
{
    extern __shared__ uint64_t sbuf_all[];
    __shared__ __attribute__((aligned(16))) uint32_t slid[8][32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, hl = lane & 31, hf = lane >> 5;
    const int seg = 2 * wv + hf;
    uint64_t* sbuf = sbuf_all + (size_t)seg * C;
    const uint64_t below = (1ull << hl) - 1ull;
    const unsigned grp = blockIdx.x & 7u;
    const int64_t lo = n * grp / 8, hi = n * (grp + 1) / 8;
    const int64_t wstep = (int64_t)(gridDim.x >> 3) * 4;
    unsigned long long upd = 0;
    int64_t pw = (int64_t)(blockIdx.x >> 3) * 4 + wv;
    // raw inputs of the current pair, loaded without branches from in-bounds
    // addresses (a row past the range reads the range's first row, lanes
    // past C or K re-read an entry); the lanes and rows they do not belong
    // to are masked where the values are used
    const int hc0 = hl < C ? hl : C - 1, hc1 = 32 + hl < C ? 32 + hl : C - 1, hk = hl < K ? hl : K - 1;
    const int hc2 = 64 + hl < C ? 64 + hl : C - 1;
    uint64_t s0, s1, s2;
    int32_t id;
    float dd;
    uint8_t fl;
    {
        const int64_t r0 = lo + 2 * pw + hf, row = r0 < hi ? r0 : lo;
        s0 = cand[row * C + hc0];
        s1 = cand[row * C + hc1];
        s2 = cand[row * C + hc2];
        id = gidx[row * K + hk];
        dd = gd2[row * K + hk];
        fl = gflag[row * K + hk];
    }
    for (; lo + 2 * pw < hi; pw += wstep) {
        const int64_t row = lo + 2 * pw + hf;
        const bool rv = row < hi;
        const uint32_t lid = hl < K && id >= 0 ? (uint32_t)id : 0xFFFFFFFFu;
        uint64_t cur = kEmptyCand;
        if (hl < K) cur = id >= 0 ? make_key(dd, lid | (fl ? 0u : kWasOld)) : kEmptyList;
        const uint64_t f0 = hl < C ? s0 : kEmptyCand, f1 = 32 + hl < C ? s1 : kEmptyCand;
        const uint64_t f2 = 64 + hl < C ? s2 : kEmptyCand;
        // next pair's inputs are in flight during this merge
        {
            const int64_t n0 = row + 2 * wstep, nrow = n0 < hi ? n0 : lo;
            s0 = cand[nrow * C + hc0];
            s1 = cand[nrow * C + hc1];
            s2 = cand[nrow * C + hc2];
            id = gidx[nrow * K + hk];
            dd = gd2[nrow * K + hk];
            fl = gflag[nrow * K + hk];
        }
        slid[seg][hl] = lid;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        int nc = 0;
        for (int c0 = 0; c0 < C; c0 += 32) {
            uint64_t key = kEmptyCand;
            if (rv && c0 + hl < C) {
                unsigned long long* p = &cand[row * C + c0 + hl];
                key = c0 == 0 ? f0 : (c0 == 32 ? f1 : (c0 == 64 ? f2 : *p));
                if (key != kEmptyCand) *p = kEmptyCand;
            }
            if (!ballot(key != kEmptyCand)) continue;
            const uint32_t sid = key_idx(key);
            bool dup = sid == (uint32_t)row;
#pragma unroll
            for (int r = 0; r < 32; r += 4) {
                const uint4 x = *(const uint4*)&slid[seg][r];
                dup = dup || x.x == sid || x.y == sid || x.z == sid || x.w == sid;
            }
            const bool keep = key != kEmptyCand && !dup;
            const uint64_t km = ballot(keep);
            const uint64_t hm = hf ? (km >> 32) : (km & 0xFFFFFFFFull);
            if (keep) sbuf[nc + __popcll(hm & below)] = key;
            nc += __popcll(hm);
        }
        if (!Smp && !ballot(nc > 0)) continue;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // the sampling may have turned entries old since the list was
        // sorted, which can reorder equal distances: re-sort if needed
        const uint64_t nxt = shfl_u64(cur, lane + 1 < 64 ? lane + 1 : lane);
        if (ballot(hl < 31 && cur > nxt)) cur = seg_sort<32>(cur);
        const uint64_t orig = cur;   // the row's list before the insertions
        if (!ballot(nc > 8)) {
            // a few candidates: each is inserted into its half's sorted list;
            // lanes whose entry exceeds it move up one place and the first
            // of them takes it (the same 32 smallest as the bitonic route)
            const int from = hl == 0 ? lane : lane - 1;
            for (int i = 0; ballot(i < nc); ++i) {
                const uint64_t x = i < nc ? sbuf[i] : kEmptyCand;
                const bool gt = cur > x;
                const uint64_t gm = ballot(gt);
                const bool pgt = hl != 0 && ((gm >> ((lane - 1) & 63)) & 1ull);
                const uint64_t prev = shfl_u64(cur, from);
                cur = gt ? (pgt ? prev : x) : cur;
            }
        } else {
            for (int b0 = 0; ballot(b0 < nc); b0 += 32) {
                uint64_t x = b0 + hl < nc ? sbuf[b0 + hl] : kEmptyCand;
                x = seg_sort<32>(x);
                cur = seg_merge_sorted<32>(cur, x);
            }
        }
        const uint32_t w = key_idx(cur);
        const uint32_t cidx = w & ~kWasOld;
        const bool sv = key_valid(cur) && key_d2(cur) < __builtin_inff();
        // insertions = valid entries of the new list minus the old valid
        // entries it kept; keys are unique, so an old entry was kept iff its
        // key is at most the new K-th key
        const uint64_t kth = shfl_u64(cur, (lane & 32) + K - 1);
        const bool osv = hl < K && key_valid(orig) && key_d2(orig) < __builtin_inff();
        upd += (unsigned long long)popc64(ballot(hl < K && nc > 0 && sv)) -
               (unsigned long long)popc64(ballot(nc > 0 && osv && orig <= kth));
        if (!Smp) {
            if (nc > 0 && hl < K) {
                gidx[row * K + hl] = sv ? (int32_t)cidx : -1;
                gd2[row * K + hl] = sv ? key_d2(cur) : __builtin_inff();
                gflag[row * K + hl] = sv ? (uint8_t)((w & kWasOld) ? 0 : 1) : 0;
                if (hl == K - 1) worst[row * wstride] = sv ? key_d2(cur) : __builtin_inff();
            }
        } else {
            // the next iteration's sampling of the merged row: every row is
            // written (its list may have been re-sorted), picks marked old
            const bool inl = rv && hl < K && sv;
            const bool isnew = inl && !(w & kWasOld), isold = inl && (w & kWasOld);
            const bool pick = sample_row(row, rv, K, sa.s, sa.R, (int32_t)cidx, isnew, isold, sa.newf, sa.oldf,
                                         sa.revnew, sa.revold, sa.seed, sa.iter);
            if (rv && hl < K) {
                gidx[row * K + hl] = sv ? (int32_t)cidx : -1;
                gd2[row * K + hl] = sv ? key_d2(cur) : __builtin_inff();
                gflag[row * K + hl] = isnew && !pick ? 1 : 0;
                if (hl == K - 1) worst[row * wstride] = sv ? key_d2(cur) : __builtin_inff();
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0 && upd) atomicAdd(&counters[0], upd);
}

// --------------------------------------------------------------- finalize

// One wave per processing-order row i: canonical FP32 direct-difference
// distances of the K list entries (on the staged rows, whose values are the
// input's), sorted by (distance, input index); the first k are written to
// input row perm[i] with input indices; optionally the working lists too.
__global__ __launch_bounds__(256) void nnd_finalize_kernel(
    int64_t n, int K, int k, const float* __restrict__ Xs, int64_t ldp, int d,
    const int32_t* __restrict__ gidx, const float* __restrict__ gd2, const uint8_t* __restrict__ gflag,
    int out_kind, int32_t* __restrict__ out_idx, float* __restrict__ out_dist,
    int32_t* __restrict__ st_idx, float* __restrict__ st_d2, uint8_t* __restrict__ st_fl,
    const uint32_t* __restrict__ perm)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int64_t orow = perm[row];
    const int32_t id = lane < K ? gidx[row * K + lane] : -1;
    const int32_t oid = id >= 0 ? (int32_t)perm[id] : -1;
    if (lane < K) {
        if (st_idx) st_idx[orow * K + lane] = oid;
        if (st_d2) st_d2[orow * K + lane] = gd2[row * K + lane];
        if (st_fl) st_fl[orow * K + lane] = gflag[row * K + lane];
    }
    // distances of the K <= 32 entries (16-lane groups, passes batched)
    const float mine = dist_batch16<KNN_F32, 8>(Xs, ldp, row, (uint32_t)id, lane < K && id >= 0, d);
    uint64_t key = (lane < K && id >= 0) ? make_key(mine, (uint32_t)oid) : kEmptyCand;
    key = seg_sort<64>(key);
    if (lane < k) {
        const bool sv = key_valid(key);
        const float d2 = sv ? key_d2(key) : __builtin_inff();
        out_idx[orow * k + lane] = sv ? (int32_t)key_idx(key) : -1;
        out_dist[orow * k + lane] = out_kind == KNN_OUT_L2 ? sqrtf(d2) : d2;
    }
}

// ------------------------------------------------------------------ host

// Encoder seeding: the 2wP window entries (index, squared distance in Xd's
// precision) of every point in processing order, n x 2wP each, ranked by
// the init kernel.
knn_status encoder_seed(const knn_encoder* enc, const knn_matrix& X, const knn_matrix& Xd, int precision, int P,
                        int D, int w, uint64_t seed, Workspace& ws, int32_t** seed_idx, float** seed_d2,
                        hipStream_t st);

int encoder_dim(const knn_encoder* enc);

namespace {

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer()
    {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer()
    {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

template <typename F>
static void launch_by_dtype(int dt, F&& f)
{
    if (dt == KNN_F32) f(std::integral_constant<int, KNN_F32>());
    else if (dt == KNN_BF16) f(std::integral_constant<int, KNN_BF16>());
    else f(std::integral_constant<int, KNN_F16>());
}

}  // namespace

static knn_status nnd_run(const knn_matrix& X, const knn_nnd_params* p, const int32_t* init_idx,
                          const float* init_dist, const uint8_t* init_flags, int32_t init_k,
                          int32_t iter_offset, int32_t* out_idx, float* out_dist,
                          int32_t* state_idx, float* state_dist, uint8_t* state_flags,
                          knn_nnd_stats* stats, hipStream_t st)
{
    knn_status r = check_matrix(X, "X");
    if (r != KNN_OK) return r;
    if (!p) return fail(KNN_EINVAL, "params is null");
    if (!out_idx || !out_dist) return fail(KNN_EINVAL, "null output pointer");
    const int64_t n = X.n;
    if (n < 2) return fail(KNN_EINVAL, "X.n must be >= 2");
    if (p->k < 1 || (int64_t)p->k > n - 1) return fail(KNN_EINVAL, "k must satisfy 1 <= k <= n-1");
    if (p->precision != KNN_PREC_FP32 && p->precision != KNN_PREC_BF16 && p->precision != KNN_PREC_FP16)
        return fail(KNN_EINVAL, "unknown precision");
    if (p->out_kind != KNN_OUT_L2 && p->out_kind != KNN_OUT_SQL2)
        return fail(KNN_EINVAL, "unknown out_kind");
    if (p->init_kind != KNN_INIT_RANDOM && p->init_kind != KNN_INIT_ENCODER)
        return fail(KNN_EINVAL, "unknown init_kind");
    if (!(p->sample_rate > 0.0f && p->sample_rate <= 1.0f))
        return fail(KNN_EINVAL, "sample_rate must be in (0, 1]");
    if (!(p->delta >= 0.0f)) return fail(KNN_EINVAL, "delta must be >= 0");
    if (p->max_iters < 0) return fail(KNN_EINVAL, "max_iters must be >= 0");
    if (iter_offset < 0) return fail(KNN_EINVAL, "iter_offset must be >= 0");
    if (init_idx && (init_k < 1 || init_k > 64)) return fail(KNN_EINVAL, "init_k must be in [1, 64]");
    // the 16-bit MFMA forms (BF16, FP16) and their staged element type
    const bool bf = p->precision != KNN_PREC_FP32;
    const int kind = p->precision == KNN_PREC_BF16 ? KNN_BF16 : (p->precision == KNN_PREC_FP16 ? KNN_F16 : KNN_F32);
    int K = p->build_k;
    if (K == 0) K = bf ? (2 * p->k < KNN_MAX_K ? 2 * p->k : KNN_MAX_K) : p->k;
    if (K < p->k) return fail(KNN_EINVAL, "build_k must be >= k");
    if (K > KNN_MAX_K) return fail(KNN_ENOTSUP, "build_k above 32 is not supported");
    if ((int64_t)K > n - 1) K = (int)(n - 1);
    if (p->init_kind == KNN_INIT_ENCODER) {
        if (!p->encoder) return fail(KNN_EINVAL, "encoder init needs an encoder");
        if (encoder_dim(p->encoder) != X.d) return fail(KNN_EINVAL, "encoder input width != X.d");
    }
    const int s = (int)ceilf(p->sample_rate * (float)K);
    JoinCfg cfg;
    cfg.s = s;
    cfg.R = s;
    // reverse edges are scattered into a table of T >= s hashed slots per
    // row and list; before each join the s filled slots with the least codes
    // are kept (an s-sample of the reverse edges, as the forward lists are
    // s-samples), so a larger table loses fewer edges to slot collisions
    if (p->rev_slots != 0 && (p->rev_slots < s || p->rev_slots > 64))
        return fail(KNN_EINVAL, "rev_slots must satisfy s <= rev_slots <= 64");
    const int T = p->rev_slots != 0 ? p->rev_slots : (4 * s < 64 ? 4 * s : 64);
    // a table of s slots is its own sample: the join reads and empties it
    cfg.reset = T == s ? 1 : 0;
    cfg.K = K;
    // default: 8 candidate slots per list entry (at most 256), which keeps
    // slot collisions rare; the benchmark forms pass smaller tables, chosen
    // by time at equal recall
    cfg.C = p->cand_slots > 0 ? p->cand_slots : (8 * K < 256 ? 8 * K : 256);
    if (cfg.C > 256) return fail(KNN_ENOTSUP, "cand_slots above 256 is not supported");
    cfg.J = p->join_cap > 0 ? p->join_cap : 4;
    if (cfg.J > kJMax) cfg.J = kJMax;
    cfg.ncap = cfg.s + cfg.R;
    cfg.lcap = cfg.s + cfg.R + cfg.K + cfg.R;
    if (cfg.lcap > 64) cfg.lcap = 64;
    if (cfg.ncap > 64) cfg.ncap = 64;

    Timer t_all, t_init, t_fin;
    (void)hipEventRecord(t_all.a, st);
    Workspace ws(st, p->workspace_limit_bytes);
    // processing order: Z-order curve of X (see morton_order); every staged
    // copy and every list below is indexed in that order
    uint32_t *perm = nullptr, *inv = nullptr;
    r = morton_order(X, 8, p->seed, ws, &perm, &inv, st);
    if (r != KNN_OK) return r;
    void* Xs = nullptr;
    float* norms = nullptr;
    int ldp = 0;
    r = stage_matrix(ws, X, KNN_F32, &Xs, &ldp, &norms, nullptr, st, perm, 1);
    if (r != KNN_OK) return r;
    void* Xb = nullptr;
    float* nb = nullptr;
    int ldb = 0;
    if (bf) {
        r = stage_matrix(ws, X, kind, &Xb, &ldb, &nb, nullptr, st, perm, 1);
        if (r != KNN_OK) return r;
    }
    // the copy the join reads, and its per-row worst-distance word
    const uint8_t* Xr = (const uint8_t*)(bf ? Xb : Xs);
    const int64_t rowbytes = bf ? (int64_t)ldb * 2 : (int64_t)ldp * 4;
    const int np = (int)ceil_div((int64_t)X.d * (bf ? 2 : 4), 32);
    float* worst = (float*)(Xr + rowbytes - 4);
    const int64_t wstride = rowbytes / 4;
    const knn_matrix Xp = {Xs, X.n, X.d, ldp, KNN_F32};   // input values in processing order
    int32_t *gidx, *newf, *oldf;
    float* gd2;
    uint8_t* gflag;
    uint32_t *revnew, *revold, *sampnew, *sampold;
    unsigned long long *cand, *counters;
    if ((r = ws.alloc(&gidx, (size_t)n * K)) != KNN_OK) return r;
    if ((r = ws.alloc(&gd2, (size_t)n * K)) != KNN_OK) return r;
    if ((r = ws.alloc(&gflag, (size_t)n * K)) != KNN_OK) return r;
    if ((r = ws.alloc(&newf, (size_t)n * s)) != KNN_OK) return r;
    if ((r = ws.alloc(&oldf, (size_t)n * K)) != KNN_OK) return r;
    if ((r = ws.alloc(&revnew, (size_t)n * T)) != KNN_OK) return r;
    if ((r = ws.alloc(&revold, (size_t)n * T)) != KNN_OK) return r;
    if (!cfg.reset) {
        if ((r = ws.alloc(&sampnew, (size_t)n * s)) != KNN_OK) return r;
        if ((r = ws.alloc(&sampold, (size_t)n * s)) != KNN_OK) return r;
    } else {
        sampnew = revnew;
        sampold = revold;
    }
    if ((r = ws.alloc(&cand, (size_t)n * cfg.C)) != KNN_OK) return r;
    if ((r = ws.alloc(&counters, 8)) != KNN_OK) return r;
    KNN_HIP(hipMemsetAsync(revnew, 0xFF, (size_t)n * T * 4, st));
    KNN_HIP(hipMemsetAsync(revold, 0xFF, (size_t)n * T * 4, st));

    // ---- init
    (void)hipEventRecord(t_init.a, st);
    const int32_t* seed_idx = init_idx;
    const float* seed_d2 = init_dist;
    const uint8_t* seed_fl = init_flags;
    int seed_k = init_k;
    if (!init_idx && p->init_kind == KNN_INIT_ENCODER) {
        int32_t* si = nullptr;
        float* sd = nullptr;
        const int P = p->proj_count > 0 ? p->proj_count : 4;
        const int w = p->proj_window > 0 ? p->proj_window : 8;
        const int D = p->proj_dims > 0 ? p->proj_dims : 8;
        // seed distances in the form's precision (the BF16 copy's values)
        const knn_matrix Xd = bf ? knn_matrix{Xb, X.n, X.d, ldb, kind} : Xp;
        // the encoder embeds in FP32 or in its BF16 mode (the 16-bit forms)
        r = encoder_seed(p->encoder, Xp, Xd, bf ? KNN_PREC_BF16 : KNN_PREC_FP32, P, D, w, p->seed, ws, &si, &sd, st);
        if (r != KNN_OK) return r;
        seed_idx = si;
        seed_d2 = sd;
        seed_fl = nullptr;
        seed_k = 2 * w * P;
    }
    {
        dim3 grid((unsigned)ceil_div(n, 4));
        // canonical FP32 direct-difference distances on the staged input values;
        // caller lists are in input order, encoder seeds already in processing order
        const int sk = seed_idx ? seed_k : 0;
        const bool given = init_idx != nullptr;
        // the first iteration (if any) is sampled by the init kernel
        const SampleArgs sa = {s, T, newf, oldf, revnew, revold, p->seed, iter_offset};
        nnd_init_kernel<KNN_F32><<<grid, 256, 0, st>>>(n, K, Xs, ldp, X.d, seed_idx, seed_d2, seed_fl, sk, p->seed,
                                                       gidx, gd2, gflag, given ? perm : nullptr,
                                                       given ? inv : nullptr, worst, wstride, sa,
                                                       p->max_iters > 0, cand, cfg.C);
        KNN_HIP(hipGetLastError());
    }
    (void)hipEventRecord(t_init.b, st);

    // ---- iterations
    unsigned long long* host_cnt = pinned_counters();
    if (!host_cnt) return fail(KNN_EDEVICE, "pinned host allocation failed");
    const double stop = (double)p->delta * (double)n * (double)K;
    const size_t merge_lds = (size_t)8 * cfg.C * 8;
    int dev = 0;
    KNN_HIP(hipGetDevice(&dev));
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    int jpc = 0;
    KNN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &jpc, (const void*)nnd_join_mfma_kernel<KNN_BF16>, 64, 0));
    if (jpc < 1) jpc = 1;
    // a multiple of 8: the join splits its grid into 8 contiguous point ranges
    const unsigned join_grid = (unsigned)round_up((int64_t)ncu * jpc, 8);
    // grid-stride kernels get exactly the resident block count (a partial
    // second round of blocks would run on an otherwise idle chip), rounded to
    // a multiple of 8: they split their grids into 8 contiguous row ranges
    int mpc = 0;
    KNN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&mpc, (const void*)nnd_merge_kernel<true>, 256,
                                                         merge_lds));
    if (mpc < 1) mpc = 1;
    const unsigned merge_grid = (unsigned)round_up(std::min<int64_t>(ceil_div(n, 8), (int64_t)ncu * mpc), 8);
    int iters = 0;
    double ms_join = 0, ms_merge = 0, ms_sample = 0;
    uint64_t gathered = 0, pairs_joined = 0;
    Timer tj, tm, ts;
    for (int it = 0; it < p->max_iters; ++it) {
        const int iter = iter_offset + it;
        KNN_HIP(hipMemsetAsync(counters, 0, 64, st));
        // iteration `iter` was sampled by the init kernel or the previous merge
        (void)hipEventRecord(ts.a, st);
        if (!cfg.reset)
            nnd_revsample_kernel<<<(unsigned)ceil_div(n, 4), 256, 0, st>>>(n, s, T, revnew, revold, sampnew,
                                                                           sampold);
        (void)hipEventRecord(ts.b, st);
        (void)hipEventRecord(tj.a, st);
        if (kind == KNN_F16)
            nnd_join_mfma_kernel<KNN_F16><<<join_grid, 64, 0, st>>>(n, cfg, Xr, rowbytes, np, newf, sampnew, oldf,
                                                                    sampold, cand, p->seed, iter, counters);
        else if (kind == KNN_BF16)
            nnd_join_mfma_kernel<KNN_BF16><<<join_grid, 64, 0, st>>>(n, cfg, Xr, rowbytes, np, newf, sampnew, oldf,
                                                                     sampold, cand, p->seed, iter, counters);
        else
            nnd_join_mfma_kernel<KNN_F32><<<join_grid, 64, 0, st>>>(n, cfg, Xr, rowbytes, np, newf, sampnew, oldf,
                                                                    sampold, cand, p->seed, iter, counters);
        KNN_HIP(hipGetLastError());
        (void)hipEventRecord(tj.b, st);
        // the merge samples the next iteration unless this is the last one
        // allowed; if the stop rule ends the run instead, that sampling's
        // flag changes are undone below
        const bool smp = it + 1 < p->max_iters;
        const SampleArgs sa = {s, T, newf, oldf, revnew, revold, p->seed, iter + 1};
        (void)hipEventRecord(tm.a, st);
        if (smp)
            nnd_merge_kernel<true><<<merge_grid, 256, merge_lds, st>>>(n, K, cfg.C, gidx, gd2, gflag, cand,
                                                                       counters, worst, wstride, sa);
        else
            nnd_merge_kernel<false><<<merge_grid, 256, merge_lds, st>>>(n, K, cfg.C, gidx, gd2, gflag, cand,
                                                                        counters, worst, wstride, sa);
        KNN_HIP(hipGetLastError());
        (void)hipEventRecord(tm.b, st);
        KNN_HIP(hipMemcpyAsync(host_cnt, counters, 64, hipMemcpyDeviceToHost, st));
        KNN_HIP(hipStreamSynchronize(st));
        float ms = 0;
        (void)hipEventElapsedTime(&ms, tj.a, tj.b);
        ms_join += ms;
        if (stats && it < KNN_MAX_ITERS_LOGGED) stats->ms_join_iter[it] = ms;
        (void)hipEventElapsedTime(&ms, tm.a, tm.b);
        ms_merge += ms;
        (void)hipEventElapsedTime(&ms, ts.a, ts.b);
        ms_sample += ms;
        gathered += host_cnt[2];
        pairs_joined += host_cnt[5];
        if (stats && it < KNN_MAX_ITERS_LOGGED) {
            stats->updates[it] = (int64_t)host_cnt[0];
            stats->emitted[it] = (int64_t)host_cnt[1];
            stats->slot_collisions[it] = (int64_t)host_cnt[3];
            stats->list_dropped[it] = (int64_t)host_cnt[4];
        }
        ++iters;
        if ((double)host_cnt[0] < stop) {
            // the flags are seen only through the returned state
            if (smp && state_flags) {
                nnd_unsample_kernel<<<(unsigned)ceil_div(n, 8), 256, 0, st>>>(n, K, s, gidx, gflag, newf);
                KNN_HIP(hipGetLastError());
            }
            break;
        }
    }

    // ---- finalize
    (void)hipEventRecord(t_fin.a, st);
    {
        dim3 grid((unsigned)ceil_div(n, 4));
        const int k = p->k;
        nnd_finalize_kernel<<<grid, 256, 0, st>>>(n, K, k, (const float*)Xs, ldp, X.d, gidx, gd2, gflag,
                                                  p->out_kind, out_idx, out_dist, state_idx, state_dist,
                                                  state_flags, perm);
        KNN_HIP(hipGetLastError());
    }
    (void)hipEventRecord(t_fin.b, st);
    (void)hipEventRecord(t_all.b, st);
    KNN_HIP(hipStreamSynchronize(st));
    if (stats) {
        stats->iters = iters;
        stats->build_k = K;
        for (int i = iters; i < KNN_MAX_ITERS_LOGGED; ++i) {
            stats->updates[i] = stats->emitted[i] = stats->slot_collisions[i] = stats->list_dropped[i] = 0;
            stats->ms_join_iter[i] = 0.0f;
        }
        const int rb = bf ? 2 : 4;
        stats->bytes_gathered = gathered * (uint64_t)X.d * (uint64_t)rb;
        stats->pairs_joined = pairs_joined;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, t_all.a, t_all.b);
        stats->ms_total = ms;
        (void)hipEventElapsedTime(&ms, t_init.a, t_init.b);
        stats->ms_init = ms;
        (void)hipEventElapsedTime(&ms, t_fin.a, t_fin.b);
        stats->ms_final = ms;
        stats->ms_sample = ms_sample;   // the reverse-sample passes (forward sampling runs in init / merge)
        stats->ms_join = ms_join;
        stats->ms_merge = ms_merge;
    }
    return KNN_OK;
}

}  // namespace knn

using namespace knn;

extern "C" void knn_nnd_default_params(int32_t k, knn_nnd_params* p)
{
    if (!p) return;
    p->k = k;
    p->build_k = 0;
    p->max_iters = 20;
    p->sample_rate = 0.5f;
    p->delta = 0.015f;
    p->seed = 0;
    p->precision = KNN_PREC_FP32;
    p->out_kind = KNN_OUT_L2;
    p->init_kind = KNN_INIT_RANDOM;
    p->encoder = nullptr;
    p->proj_count = 0;
    p->proj_window = 0;
    p->proj_dims = 0;
    p->cand_slots = 0;
    p->join_cap = 0;
    p->workspace_limit_bytes = 0;
    p->rev_slots = 0;
    p->ensemble = 0;
}

namespace knn {

// Row r of the union: the K entries of list a then those of list b, every
// flag new (the init kernel drops repeats and keeps the best K).
__global__ __launch_bounds__(256) void nnd_union_kernel(int64_t n, int K, const int32_t* __restrict__ ai,
                                                        const float* __restrict__ ad, const int32_t* __restrict__ bi,
                                                        const float* __restrict__ bd, int32_t* __restrict__ ci,
                                                        float* __restrict__ cd, uint8_t* __restrict__ cf)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * 2 * K) return;
    const int64_t r = e / (2 * K);
    const int j = (int)(e % (2 * K));
    ci[e] = j < K ? ai[r * K + j] : bi[r * K + j - K];
    cd[e] = j < K ? ad[r * K + j] : bd[r * K + j - K];
    cf[e] = 1;
}

static void stats_add(knn_nnd_stats* acc, const knn_nnd_stats& s)
{
    for (int i = 0; i < s.iters && acc->iters + i < KNN_MAX_ITERS_LOGGED; ++i) {
        const int j = acc->iters + i;
        acc->updates[j] = s.updates[i];
        acc->emitted[j] = s.emitted[i];
        acc->ms_join_iter[j] = s.ms_join_iter[i];
        acc->slot_collisions[j] = s.slot_collisions[i];
        acc->list_dropped[j] = s.list_dropped[i];
    }
    acc->iters += s.iters;
    acc->build_k = s.build_k;
    acc->bytes_gathered += s.bytes_gathered;
    acc->pairs_joined += s.pairs_joined;
    acc->ms_total += s.ms_total;
    acc->ms_init += s.ms_init;
    acc->ms_sample += s.ms_sample;
    acc->ms_join += s.ms_join;
    acc->ms_merge += s.ms_merge;
    acc->ms_final += s.ms_final;
}

// E independent runs joined into one graph: run 0, then for each further run
// the union of its lists with the lists so far seeds a continuation (every
// entry new, so every pair in the union is joined once more).  Independent
// runs miss different neighbours: at 10M points two runs at K_b = 32 reach a
// recall one run cannot reach at any supported K_b.
static knn_status nnd_ensemble(const knn_matrix& X, const knn_nnd_params* p, int E, int32_t* out_idx,
                               float* out_dist, int32_t* state_idx, float* state_dist, uint8_t* state_flags,
                               knn_nnd_stats* stats, hipStream_t st)
{
    knn_status r = check_matrix(X, "X");
    if (r != KNN_OK) return r;
    const int64_t n = X.n;
    int K = p->build_k;
    if (K == 0) K = p->precision != KNN_PREC_FP32 ? std::min(2 * p->k, KNN_MAX_K) : p->k;
    if ((int64_t)K > n - 1) K = (int)(n - 1);
    if (K < 1) return fail(KNN_EINVAL, "build_k");
    if (2 * K > 64) return fail(KNN_ENOTSUP, "ensemble needs 2 K_b <= 64");
    const size_t nk = (size_t)n * K;
    int32_t *ai = nullptr, *bi = nullptr, *ci = nullptr, *ti = nullptr;
    float *ad = nullptr, *bd = nullptr, *cd = nullptr, *td = nullptr;
    uint8_t* cf = nullptr;
    void* bufs[9];
    const size_t sizes[9] = {nk * 4, nk * 4, nk * 4, nk * 4, 2 * nk * 4, 2 * nk * 4, 2 * nk, (size_t)n * p->k * 4,
                             (size_t)n * p->k * 4};
    for (int i = 0; i < 9; ++i) {
        if (hipMallocAsync(&bufs[i], sizes[i] ? sizes[i] : 4, st) != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < i; ++j) (void)hipFreeAsync(bufs[j], st);
            return fail(KNN_ENOMEM, "ensemble buffers");
        }
    }
    ai = (int32_t*)bufs[0];
    ad = (float*)bufs[1];
    bi = (int32_t*)bufs[2];
    bd = (float*)bufs[3];
    ci = (int32_t*)bufs[4];
    cd = (float*)bufs[5];
    cf = (uint8_t*)bufs[6];
    ti = (int32_t*)bufs[7];
    td = (float*)bufs[8];
    knn_nnd_stats acc = {};
    knn_nnd_stats one;
    knn_nnd_params q = *p;
    q.ensemble = 1;
    q.build_k = K;
    r = nnd_run(X, &q, nullptr, nullptr, nullptr, 0, 0, ti, td, ai, ad, nullptr, &one, st);
    if (r == KNN_OK) stats_add(&acc, one);
    for (int e = 1; e < E && r == KNN_OK; ++e) {
        knn_nnd_params qe = q;
        qe.seed = p->seed + (uint64_t)e * 0x9E3779B97F4A7C15ull;
        r = nnd_run(X, &qe, nullptr, nullptr, nullptr, 0, 0, ti, td, bi, bd, nullptr, &one, st);
        if (r != KNN_OK) break;
        stats_add(&acc, one);
        nnd_union_kernel<<<(unsigned)ceil_div((int64_t)(2 * nk), 256), 256, 0, st>>>(n, K, ai, ad, bi, bd, ci, cd,
                                                                                  cf);
        KNN_HIP(hipGetLastError());
        knn_nnd_params qr = qe;
        qr.init_kind = KNN_INIT_RANDOM;
        qr.encoder = nullptr;
        const bool last = e == E - 1;
        r = nnd_run(X, &qr, ci, cd, cf, 2 * K, 4096 * e, last ? out_idx : ti, last ? out_dist : td,
                    last ? state_idx : ai, last ? state_dist : ad, last ? state_flags : nullptr, &one, st);
        if (r == KNN_OK) stats_add(&acc, one);
    }
    for (int i = 0; i < 9; ++i) (void)hipFreeAsync(bufs[i], st);
    if (r == KNN_OK) KNN_HIP(hipStreamSynchronize(st));
    if (r == KNN_OK && stats) *stats = acc;
    return r;
}

}  // namespace knn

extern "C" knn_status nndescent_build(knn_matrix X, const knn_nnd_params* p, int32_t* out_idx,
                                      float* out_dist, int32_t* state_idx, float* state_dist,
                                      uint8_t* state_flags, knn_nnd_stats* stats, void* stream)
{
    try {
        if (!p) return fail(KNN_EINVAL, "params are null");
        if (p->ensemble < 0 || p->ensemble > 8) return fail(KNN_EINVAL, "ensemble must be in [0, 8]");
        if (p->ensemble > 1)
            return nnd_ensemble(X, p, p->ensemble, out_idx, out_dist, state_idx, state_dist, state_flags, stats,
                                (hipStream_t)stream);
        return nnd_run(X, p, nullptr, nullptr, nullptr, 0, 0, out_idx, out_dist, state_idx,
                       state_dist, state_flags, stats, (hipStream_t)stream);
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}

extern "C" knn_status nndescent_refine(knn_matrix X, const knn_nnd_params* p,
                                       const int32_t* init_idx, const float* init_dist,
                                       const uint8_t* init_flags, int32_t init_k,
                                       int32_t iter_offset, int32_t* out_idx, float* out_dist,
                                       int32_t* state_idx, float* state_dist,
                                       uint8_t* state_flags, knn_nnd_stats* stats, void* stream)
{
    try {
        if (!init_idx) return fail(KNN_EINVAL, "init_idx is null");
        return nnd_run(X, p, init_idx, init_dist, init_flags, init_k, iter_offset, out_idx,
                       out_dist, state_idx, state_dist, state_flags, stats, (hipStream_t)stream);
    } catch (...) {
        return fail(KNN_EDEVICE, "unexpected exception");
    }
}
