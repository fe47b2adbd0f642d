/*
 * knn.h -- C ABI of the MI355X (gfx950) k-nearest-neighbour graph library.
 *
 * The library builds k-NN graphs of an n x d point set resident in device
 * memory: an exact brute-force path (tiled distance GEMM + top-k) and
 * NNDescent (random or encoder-seeded init, sampled new/old local joins,
 * bounded sorted list merges, stop on update count).  It is the graph stage
 * the paper's dimensionality-reduction methods share (paper, section
 * "GPU-Native k-NN via NNDescent"; the exact ranks of the embedding-quality
 * section), with the steps next to it: PCA before the graph, the UMAP fuzzy
 * graph and the embedding-quality metrics after it.
 *
 * Conventions for every entry point:
 *  - Pointers named as device pointers must point to device memory of the
 *    current HIP device; host pointers are marked "host".  The caller owns
 *    every buffer passed in.  Scratch (staged copies, working lists, slots)
 *    is carved from a per-device arena that the library owns and keeps
 *    between calls: it grows when a call needs more and is never returned
 *    before the process ends, and calls on one device take turns on it.
 *    knn_exact_noalloc takes its scratch from a fixed static device array
 *    instead; nndescent_build with ensemble > 1 also takes the runs' lists
 *    from stream-ordered allocations freed before it returns.  knn_encoder
 *    objects are library-owned until destroyed.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Every call is
 *    blocking: the stream is synchronised before return.
 *  - Errors are returned as knn_status (never thrown).  On error the outputs
 *    are unspecified; knn_last_error() gives a thread-local message.
 *  - Results: each output row is sorted by (squared distance, index)
 *    ascending and never contains its own row index.  Duplicate points are
 *    kept at distance 0.  Distances are ranked on squared Euclidean distance
 *    and returned as Euclidean (KNN_OUT_L2) or squared (KNN_OUT_SQL2).
 *  - Inputs holding NaN or Inf give unspecified results.
 *  - Index arrays are int32: n must be below 2^31.
 */
#ifndef KNN_H_
#define KNN_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t knn_status;
enum {
    KNN_OK = 0,
    KNN_EINVAL = -1,   /* bad argument (size, pointer, enum) */
    KNN_ENOMEM = -2,   /* device allocation failed or workspace limit exceeded */
    KNN_EDEVICE = -3,  /* a HIP runtime call failed */
    KNN_ENOTSUP = -4   /* valid request outside what is implemented (e.g. k, re-rank
                          width or K_b above KNN_MAX_K) */
};

/* element type of an input matrix */
enum { KNN_F32 = 0, KNN_BF16 = 1, KNN_F16 = 2 };
/* distance precision: FP32 throughout, or 16-bit MFMA candidates (inputs
 * rounded to BF16, or to FP16 -- exact for FP16-stored data, finite below
 * 65504 in magnitude) with FP32 accumulation + FP32 re-rank */
enum { KNN_PREC_FP32 = 0, KNN_PREC_BF16 = 1, KNN_PREC_FP16 = 2 };
/* returned distance kind */
enum { KNN_OUT_L2 = 0, KNN_OUT_SQL2 = 1 };
/* NNDescent initial lists */
enum { KNN_INIT_RANDOM = 0, KNN_INIT_ENCODER = 1 };

/* Largest k / re-rank width / working list size the kernels support. */
#define KNN_MAX_K 32

/* A row-major n x d matrix in device memory; row r starts at data + r*ld
 * elements of `dtype`.  Requires n >= 1, d >= 1, ld >= d. */
typedef struct {
    const void* data;
    int64_t n;
    int32_t d;
    int64_t ld;
    int32_t dtype;
} knn_matrix;

const char* knn_status_str(knn_status s);
/* Message of the last failing call on this thread ("" if none). */
const char* knn_last_error(void);

/*
 * Exact k nearest neighbours of every row of X among the other rows of X
 * (the exact pairwise-distance ranking of the paper's embedding-quality
 * section, computed by tiled GEMM with the norm expansion of the paper's
 * k-NN section, then re-ranked by direct differences).
 *
 *  precision  KNN_PREC_FP32: FP32 MFMA distances; KNN_PREC_BF16: BF16 MFMA
 *             distances with FP32 accumulation.  Either way the best
 *             `rerank_k` candidates per row are re-ranked with FP32
 *             direct-difference distances, and FP32 rows whose candidate
 *             set cannot be certified are recomputed exhaustively.  With
 *             KNN_PREC_FP32 and d <= 16 no GEMM is run: every pair's
 *             direct-difference distance is formed (the same lists).
 *  rerank_k   candidates kept per row before the re-rank, k <= rerank_k <=
 *             KNN_MAX_K (0 = min(2k, KNN_MAX_K)).
 *  out_idx    device, n x k int32.   out_dist  device, n x k float.
 * Errors: KNN_EINVAL if n < 2, k < 1, k > n-1, d < 1, ld < d, n >= 2^31,
 * a null pointer or an unknown enum; KNN_ENOTSUP if rerank_k > KNN_MAX_K.
 */
knn_status knn_exact(knn_matrix X, int32_t k, int32_t precision, int32_t rerank_k,
                     int32_t out_kind, int32_t* out_idx, float* out_dist, void* stream);

/*
 * Exact k nearest rows of R for each row of Q (Q.d == R.d, same dtype).
 * q_self (device, nullable, Q.n int32): row of R that query i must not
 * return (-1: none).  out_idx / out_dist: device, Q.n x k.
 * Errors as knn_exact, with k > R.n (or R.n - 1 when q_self is given)
 * rejected.
 */
knn_status knn_exact_query(knn_matrix Q, knn_matrix R, const int32_t* q_self, int32_t k,
                           int32_t precision, int32_t rerank_k, int32_t out_kind,
                           int32_t* out_idx, float* out_dist, void* stream);

/*
 * knn_exact_query with a bound on its scratch: the queries are processed in
 * chunks (multiples of 128 rows) small enough that the staged reference
 * set plus one chunk's staged rows and candidate lists fit in
 * workspace_limit_bytes; every chunk is a pass over R, so a smaller limit
 * trades time for memory (the paper's chunked pairwise-distance evaluation,
 * section "Scaling Behavior").  0 = no limit (one chunk).  Results are those
 * of knn_exact_query.  Errors as knn_exact_query, plus KNN_ENOMEM when the
 * staged reference set and a single 128-query chunk exceed the limit, and
 * KNN_EINVAL for a negative limit.  (FP32 with d <= 16 stages nothing: a
 * chunk is a multiple of 256 rows, each needing S * 256 bytes of split
 * lists, S <= 16 reference splits.)
 */
knn_status knn_exact_query_limited(knn_matrix Q, knn_matrix R, const int32_t* q_self, int32_t k,
                                   int32_t precision, int32_t rerank_k, int32_t out_kind,
                                   int64_t workspace_limit_bytes, int32_t* out_idx, float* out_dist,
                                   void* stream);

/* Size of the static device array knn_exact_noalloc works in (64 MiB). */
#define KNN_NOALLOC_SCRATCH_BYTES (64ll << 20)

/*
 * knn_exact for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same results as knn_exact, with every scratch buffer carved from a
 * file-scope static device array of KNN_NOALLOC_SCRATCH_BYTES that each
 * device holds from the library's first use on it until the process ends.
 * The call makes no hipMalloc, hipFree or other allocation; queries are
 * chunked to fit the array.  The caller passes inputs and outputs as for
 * knn_exact.  Limit: the staged copy of X (n * roundup(d, 32) * 4 bytes in
 * FP32, n * roundup(d, 64) * 2 in BF16) plus n * 4 bytes of norms and one
 * 128-query chunk (about 140 KB) must fit, e.g. n <= 240,000 at d = 50 FP32
 * (FP32 with d <= 16 stages nothing and fits any n); larger inputs get
 * KNN_ENOMEM with the sizes in the message.  Every call on
 * a device shares that device's array and leaves it holding its last
 * contents: calls that overlap on one device (other threads or streams)
 * race and must be serialised by the caller.  Other errors as knn_exact.
 */
knn_status knn_exact_noalloc(knn_matrix X, int32_t k, int32_t precision, int32_t rerank_k,
                             int32_t out_kind, int32_t* out_idx, float* out_dist, void* stream);

typedef struct knn_encoder knn_encoder;

/* NNDescent parameters (Dong, Charikar & Li 2011; the paper fixes the
 * early-termination rate delta = 0.015). */
typedef struct {
    int32_t k;            /* neighbours returned, 1 <= k <= n-1 */
    int32_t build_k;      /* working list size K_b, k <= K_b <= KNN_MAX_K (0: k, or 2k for BF16) */
    int32_t max_iters;    /* iteration cap, >= 0 */
    float sample_rate;    /* rho in (0, 1]: s = ceil(rho * K_b) new entries sampled per row */
    float delta;          /* stop when updates < delta * n * K_b; >= 0 */
    uint64_t seed;        /* all random choices are a function of (seed, iteration, row, slot) */
    int32_t precision;    /* KNN_PREC_FP32, or KNN_PREC_BF16 / KNN_PREC_FP16 (join on MFMA, FP32 re-rank at the end) */
    int32_t out_kind;     /* KNN_OUT_L2 / KNN_OUT_SQL2 */
    int32_t init_kind;    /* KNN_INIT_RANDOM or KNN_INIT_ENCODER */
    const knn_encoder* encoder;  /* required for KNN_INIT_ENCODER */
    int32_t proj_count;   /* encoder init: number of sorted orders P (0: 4) */
    int32_t proj_window;  /* encoder init: neighbours taken on each side per order (0: 8) */
    int32_t proj_dims;    /* encoder init: projections per order key D in {1,2,4,8} (0: 8) */
    int32_t cand_slots;   /* hashed candidate slots per row and iteration, <= 256 (0: min(8 K_b, 256)) */
    int32_t join_cap;     /* max candidates one join list sends to one member, <= 4 (0: 4) */
    int64_t workspace_limit_bytes; /* 0: no limit; else KNN_ENOMEM when scratch exceeds it */
    int32_t rev_slots;    /* hashed reverse-edge slots per row and list, s <= rev_slots <= 64; the join
                           * takes the s filled slots with the least codes (0: min(4 s, 64)) */
    int32_t ensemble;     /* nndescent_build only: E independent runs (seeds seed + e * 0x9E3779B97F4A7C15),
                           * each after the first joined to the lists so far by a continuation seeded
                           * with their union (all entries new); 0 or 1: one run; at most 8, and
                           * 2 K_b <= 64.  The E runs' buffers beyond the arena's are stream-ordered
                           * allocations freed before return. */
} knn_nnd_params;

/* Fills the defaults: build_k 0, max_iters 20, rho 0.5, delta 0.015, seed 0,
 * FP32, L2, random init, other knobs 0 (= library choice). */
void knn_nnd_default_params(int32_t k, knn_nnd_params* p);

#define KNN_MAX_ITERS_LOGGED 64
typedef struct {
    int32_t iters;                            /* iterations run in this call */
    int32_t build_k;                          /* K_b actually used */
    int64_t updates[KNN_MAX_ITERS_LOGGED];    /* list insertions per iteration */
    int64_t emitted[KNN_MAX_ITERS_LOGGED];    /* candidates sent to the slot buffers */
    uint64_t bytes_gathered;                  /* algorithmic row bytes gathered by local joins */
    /* wall times (ms) of the phases; new/old sampling and the scatter of
     * reverse edges run inside the init kernel (first iteration) and the
     * merges (later ones) and are counted there; ms_sample is the passes
     * that reduce each row's reverse-slot table to its s-sample */
    double ms_total, ms_init, ms_sample, ms_join, ms_merge, ms_final;
    float ms_join_iter[KNN_MAX_ITERS_LOGGED]; /* local-join kernel time per iteration */
    /* offers that found their hashed candidate slot holding another source's
     * key (one of the two is lost), per iteration; seen by each offer's slot
     * read, so offers racing for one slot are not counted */
    int64_t slot_collisions[KNN_MAX_ITERS_LOGGED];
    /* join-list members not joined because the list exceeded 64 members
     * (old members are cut first), per iteration */
    int64_t list_dropped[KNN_MAX_ITERS_LOGGED];
    /* member pairs whose distance the local joins evaluated (new x new once,
     * new x old), over all iterations: the Gram work, 2 d flops each */
    uint64_t pairs_joined;
} knn_nnd_stats;

/*
 * Approximate k-NN graph of X by NNDescent.
 *  out_idx, out_dist  device, n x p->k.
 *  state_idx, state_dist, state_flags  device, nullable, n x K_b each
 *       (int32 / float squared distance / uint8 1 = new): the working lists
 *       after the last iteration, which nndescent_refine can continue.
 *  stats  host, nullable.
 * Errors: KNN_EINVAL for bad sizes/params (k, K_b, rho, delta, max_iters,
 * null pointers, encoder missing for KNN_INIT_ENCODER or of another d);
 * KNN_ENOTSUP if K_b > KNN_MAX_K or cand_slots > 256; KNN_ENOMEM as above.
 * Scratch (about n * (13 K_b + 12 s + 8 T + 8 C) bytes, T = rev_slots and
 * C = cand_slots as used, plus staged copies of X) comes from a per-device
 * arena the library keeps between calls; calls on one device take turns on
 * it.
 */
knn_status nndescent_build(knn_matrix X, const knn_nnd_params* p,
                           int32_t* out_idx, float* out_dist,
                           int32_t* state_idx, float* state_dist, uint8_t* state_flags,
                           knn_nnd_stats* stats, void* stream);

/*
 * Continue NNDescent from given lists.
 *  init_idx    device, n x init_k int32; entries that are -1, out of range,
 *              equal to their row or repeated are replaced by random fill.
 *  init_dist   device, nullable, n x init_k squared distances of those
 *              entries (recomputed when NULL).
 *  init_flags  device, nullable, n x init_k (1 = new; NULL = all new).
 *  iter_offset first iteration number: the random stream continues there, so
 *              build(a iters) then refine(b iters, iter_offset = a) from its
 *              state reproduces build(a + b iters) bit for bit.
 * init_k may differ from K_b (extra columns are dropped after sorting,
 * missing ones are filled at random); 1 <= init_k <= 64, else KNN_EINVAL.
 * Outputs as nndescent_build.
 */
knn_status nndescent_refine(knn_matrix X, const knn_nnd_params* p,
                            const int32_t* init_idx, const float* init_dist,
                            const uint8_t* init_flags, int32_t init_k, int32_t iter_offset,
                            int32_t* out_idx, float* out_dist,
                            int32_t* state_idx, float* state_dist, uint8_t* state_flags,
                            knn_nnd_stats* stats, void* stream);

/* ----------------------------------------------------------------------
 * Learned seeding: an MLP encoder d -> 64 -> 32 (ReLU hidden layer) whose
 * embedding is projected on P seeded directions; the sorted orders give
 * each point its window neighbours as initial candidates for NNDescent.
 * The paper has no encoder: this learned-initialisation form is an addition
 * that replaces the random k-neighbour init of NNDescent (paper, section
 * "GPU-Native k-NN via NNDescent"), which stays the default and fallback.
 * The activation, loss and optimiser are this library's choices: ReLU,
 * triplet loss with a margin, Adam (Kingma & Ba 2015).
 * ---------------------------------------------------------------------- */
#define KNN_ENC_H1 64
#define KNN_ENC_H2 32

/* Creates an encoder for inputs of width d with He-uniform weights drawn
 * from `seed` (W1: d x 64, b1: 64, W2: 64 x 32, b2: 32, row-major FP32). */
knn_status knn_encoder_create(int32_t d, uint64_t seed, knn_encoder** enc);
void knn_encoder_destroy(knn_encoder* enc);
/* Copy the FP32 weights in / out (host buffers of the sizes above). */
knn_status knn_encoder_set_weights(knn_encoder* enc, const float* W1, const float* b1,
                                   const float* W2, const float* b2);
knn_status knn_encoder_get_weights(const knn_encoder* enc, float* W1, float* b1,
                                   float* W2, float* b2);

/* Z = W2^T relu(W1^T x + b1) + b2 for every row of X; Z: device, n x 32 float.
 * precision KNN_PREC_FP32 (FP32 FMA) or KNN_PREC_BF16 (BF16 MFMA, FP32
 * accumulate: x, W1, the hidden layer and W2 rounded to BF16; biases FP32).
 * The NNDescent BF16 form seeds through the BF16 embedding. */
knn_status knn_encoder_embed(const knn_encoder* enc, knn_matrix X, int32_t precision,
                             float* Z, void* stream);

/*
 * One triplet-loss forward/backward pass without updating the weights.
 * rows: device, 3B int32 = [anchors; positives; negatives] (rows of X).
 * loss = (1/B) sum max(0, margin + |za-zp|^2 - |za-zn|^2).
 * precision: KNN_PREC_FP32, or KNN_PREC_BF16: the factors of every product
 *   (inputs, weights, hidden values, output gradients) are rounded to BF16
 *   and accumulated in FP32; bias terms and bias gradients stay FP32.
 * grads: device, nullable, d*64 + 64 + 64*32 + 32 floats (gW1, gb1, gW2, gb2).
 * loss_out: host.
 */
knn_status knn_encoder_grads(knn_encoder* enc, knn_matrix X, const int32_t* rows, int32_t B,
                             float margin, int32_t precision, float* loss_out, float* grads,
                             void* stream);

/* Adam settings for knn_encoder_train. */
typedef struct {
    int32_t steps;        /* optimisation steps */
    int32_t batch;        /* triplets per step */
    float lr, beta1, beta2, eps, margin;
    uint64_t seed;        /* triplet sampling */
    int32_t precision;    /* forward / backward products: KNN_PREC_FP32 or KNN_PREC_BF16 (FP32 weights) */
} knn_train_params;

void knn_train_default_params(knn_train_params* t);

/*
 * Train the encoder on X with its k-NN graph knn_idx (device, X.n x k):
 * each triplet takes a uniform anchor, a uniform positive among its k
 * neighbours and a uniform negative row; Adam on FP32 weights.
 * loss_log: host, nullable, t->steps floats.
 */
knn_status knn_encoder_train(knn_encoder* enc, knn_matrix X, const int32_t* knn_idx, int32_t k,
                             const knn_train_params* t, float* loss_log, void* stream);

/*
 * The triplets training step `step` (0-based, counted over the encoder's
 * life) of knn_encoder_train draws: rows (device, 3B int32) = [anchors;
 * positives; negatives].  Anchor b and negative b are uniform rows of
 * [0, n); positive b is knn_idx[anchor * k + j] for a uniform j < k (the
 * anchor itself if that entry is out of range).  Each is a function of
 * (seed, step, b).  knn_idx: device, n x k.
 */
knn_status knn_encoder_triplets(int64_t n, const int32_t* knn_idx, int32_t k, int32_t B,
                                uint64_t seed, int32_t step, int32_t* rows, void* stream);

/*
 * One optimisation step on caller-given triplets: the gradient of
 * knn_encoder_grads on rows (device, 3B int32) at the current weights, then
 * Adam step t + 1 (t = steps taken so far) with t's settings (steps, batch
 * and seed are not used).  knn_encoder_train's step s is this step on
 * knn_encoder_triplets(seed = t->seed, step = steps taken before it).
 * loss_out: host, nullable (the batch loss before the update).
 */
knn_status knn_encoder_step(knn_encoder* enc, knn_matrix X, const int32_t* rows, int32_t B,
                            const knn_train_params* t, float* loss_out, void* stream);

/* Adam state: first and second moments (host, as many floats as weights)
 * and the number of steps taken. */
knn_status knn_encoder_get_adam(const knn_encoder* enc, float* m, float* v, int32_t* t);

/*
 * Seed lists from sorted projections of an embedding Z.  Order p uses the D
 * directions dirs[p*D .. p*D+D): the projections Z . r are FP32 sums in
 * coordinate order; D = 1 sorts by the projection itself, D > 1 by the
 * Z-order code of the D projections, each quantised to 32/D bits over its
 * range across all points.  Points are sorted by (key, index) with a stable
 * radix sort; each point takes the w predecessors and successors in every
 * order; candidates (self removed, repeats merged) are ranked by canonical
 * FP32 squared input distance and the best K kept, sorted by (distance,
 * index); rows with fewer than K candidates are padded with -1 / +inf.
 *  Z     device, n x m float (m <= 64).   dirs  device, (P*D) x m float.
 *  D in {1, 2, 4, 8};  2*w*P <= 64;  K <= 64.
 *  out_idx / out_dist  device, n x K (squared distances).
 */
knn_status knn_proj_seed(knn_matrix X, const float* Z, int32_t m, const float* dirs,
                         int32_t P, int32_t D, int32_t w, int32_t K, int32_t* out_idx,
                         float* out_dist, void* stream);

/*
 * Principal components of the rows of X and the projection onto the first p
 * (the PCA preprocessing to pca_dim the paper runs before the k-NN stage,
 * sections "Reproducibility" and "Scaling Behavior"), in FP64: mean mu,
 * covariance C = (X - mu)^T (X - mu) / (n - 1), the p largest eigenvalues
 * (descending) and their eigenvectors, each with its entry of largest
 * magnitude positive, and Z = (X - mu) V rounded to FP32.
 *  p       1 <= p <= min(d, 64).
 *  iters   subspace iterations (0: 200); the eigenvectors come from an
 *          m = min(d, 80, max(2p, p + 16))-column subspace iteration with a
 *          final Rayleigh-Ritz step (exact when m = d), so their error falls
 *          as (lambda_{m+1} / lambda_p)^iters.
 *  Z       device, n x p float.   components  device, nullable, d x p
 *          double (row-major).   eigenvalues  device, nullable, p double.
 *  mean    device, nullable, d double.
 * Errors: KNN_EINVAL for a bad matrix, n < 2, p out of range, iters < 0,
 * or X of rank below the subspace width; KNN_ENOTSUP for p > 64 or
 * d > 16384.
 */
knn_status knn_pca(knn_matrix X, int32_t p, int32_t iters, float* Z, double* components,
                   double* eigenvalues, double* mean, void* stream);

/*
 * Embedding quality as the paper's section "Embedding Quality" measures it
 * (Venna & Kaski 2006), from exact ranks in both spaces: X (n x d, the
 * input) and Y (n x e, an embedding of the same rows).  r(i,j) = rank of j
 * among the other rows by distance from i in X (1 = nearest), r'(i,j) in Y;
 * N(i) / L(i) = the k nearest in X / Y.  Ranks break distance ties by the
 * smaller index and are taken on canonical FP32 direct-difference squared
 * distances (the order knn_exact returns); the X-space distances come from
 * an FP32 MFMA Gram with every comparison inside its error bound re-decided
 * in the canonical precision.  Above 16 dimensions the same Gram pass also
 * yields X's exact k-NN (knn_exact's merge, re-rank and certificate); the
 * embedding's k-NN and ranks use direct differences when e <= 16.
 *  metrics  host, 3 doubles: k-NN preservation sum_i |N(i) & L(i)| / (n k);
 *           trustworthiness 1 - 2 / (n k (2n - 3k - 1)) sum_i sum_{j in
 *           L(i) \ N(i)} (r(i,j) - k); continuity, the same with N, L and r,
 *           r' swapped.
 *  hits, trust, cont  device, nullable, n each: the per-row terms
 *           (|N(i) & L(i)| int32, the two rank sums int64).
 * Errors: KNN_EINVAL for bad matrices, X.n != Y.n, k < 1 or 3k >= 2n - 1;
 * KNN_ENOTSUP for k > 16.
 */
knn_status knn_quality(knn_matrix X, knn_matrix Y, int32_t k, int32_t* hits, int64_t* trust,
                       int64_t* cont, double* metrics, void* stream);

/* ----------------------------------------------------------------------
 * The fuzzy graph UMAP-family methods build from the k-NN graph (UMAP of
 * McInnes, Healy & Melville 2018; the paper's sections "Architecture" and
 * "Method Implementations": every method starts from the shared k-NN stage).
 * ---------------------------------------------------------------------- */

/*
 * Membership strengths of the graph's edges and their fuzzy union.
 *  knn_idx, knn_dist  device, n x k: each row's neighbours (distinct, in
 *      [0, n), not the row itself) and their Euclidean distances.
 *  For row i: rho_i = smallest positive distance (0 if none); sigma_i > 0
 *  solves sum_r exp(-max(0, d_ir - rho_i) / sigma_i) = log2(k), found in
 *  double; rows where #{r : d_ir <= rho_i} >= log2(k) have no root and get
 *  sigma_i = 0 with weights 1 where d_ir <= rho_i and 0 elsewhere (the
 *  limit); w_ir = exp(-max(0, d_ir - rho_i) / sigma_i).
 *  rho, sigma   device, nullable, n floats.
 *  weights      device, nullable, n x k floats: w_ir.
 *  The symmetric graph W = A + A^T - A o A^T (A[i][idx_ir] = w_ir) is
 *  returned in CSR form: row_ptr (device, n + 1 int64), col (device, int32)
 *  and val (device, float), each row's columns ascending; the pattern is the
 *  union of the lists and their transpose (entries of value 0 are kept).
 *  col and val must hold 2 n k entries; *nnz (host) receives the count.
 * Errors: KNN_EINVAL for null pointers, n < 2, k < 1 or k > n - 1, or an
 * entry of knn_idx out of range, equal to its row or repeated in its row
 * (detected after the work; outputs unspecified); KNN_ENOTSUP for
 * k > KNN_MAX_K or 2 n k >= 2^32.
 */
knn_status knn_fuzzy_graph(const int32_t* knn_idx, const float* knn_dist, int64_t n, int32_t k,
                           float* rho, float* sigma, float* weights, int64_t* row_ptr,
                           int32_t* col, float* val, int64_t* nnz, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* KNN_H_ */
