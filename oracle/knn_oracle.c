/*
 * CPU oracle for the kNN-graph path.  TEST INFRASTRUCTURE ONLY: it is called
 * by the test-suite, by the smoke check and by the benchmark's CPU-baseline
 * leg, never by the library.  It shares no code with the HIP path.
 *
 * Everything is plain, slow and sequential in the order the definitions are
 * written, in double precision, so that it can be checked against the paper
 * and the NNDescent paper by eye:
 *
 *  - exact kNN: the paper's quality section ranks neighbours by exact pairwise
 *    Euclidean distances; here D(i,j) = sum_t (x_it - x_jt)^2 in fp64, sorted
 *    by (D, j) ascending, self excluded.
 *  - NNDescent: Dong, Charikar & Li (WWW 2011), the algorithm the paper's
 *    GPU-native k-NN section builds on: random init, sampled new/old lists,
 *    reverse lists, local join, update counting, stop when the count falls
 *    below delta * n * K (the paper fixes delta = 0.015).
 *  - round-to-nearest-even FP32 -> BF16 by its bit definition.
 *  - the seeding encoder: a d -> 64 -> 32 ReLU MLP, triplet loss, analytic
 *    backward pass, and Adam (Kingma & Ba 2015).
 *  - sorted-projection seeding of initial neighbour lists.
 *
 * Parity of the NNDescent trajectory with the GPU is not defined (each side
 * draws its own random numbers and the GPU updates in batches); the GPU graph
 * is judged by recall against oracle_exact_query.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- helpers */

static double sqdist(const double* a, const double* b, int d)
{
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double e = a[t] - b[t];
        s += e * e;
    }
    return s;
}

/* (da, ja) < (db, jb) lexicographically: distance first, then index. */
static int pair_less(double da, int64_t ja, double db, int64_t jb)
{
    return da < db || (da == db && ja < jb);
}

/* splitmix64 (Steele, Lea & Flood, OOPSLA 2014): a sequential generator. */
static uint64_t rng_next(uint64_t* s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform integer in [0, m); modulo bias below 2^-40 for m < 2^24. */
static int64_t rng_below(uint64_t* s, int64_t m)
{
    return (int64_t)(rng_next(s) % (uint64_t)m);
}

/* ------------------------------------------------------------- exact kNN */

/*
 * For each query q_i (row i of Q) the k reference rows j with the smallest
 * (D(q_i, r_j), j), ascending.  q_self (nullable) names a reference row to
 * exclude for each query (-1: none).  Returns 0, or -1 on bad arguments.
 */
int oracle_exact_query(const double* R, int64_t nr, int64_t ldr, int d,
                       const double* Q, int64_t nq, int64_t ldq,
                       const int64_t* q_self, int k,
                       int64_t* out_idx, double* out_d2)
{
    if (k < 1 || d < 1 || nr < 1 || nq < 0) return -1;
    if (k > nr - (q_self ? 1 : 0)) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < nq; ++i) {
        int64_t* I = out_idx + i * k;
        double* D = out_d2 + i * k;
        int cnt = 0;
        const double* q = Q + i * ldq;
        for (int64_t j = 0; j < nr; ++j) {
            if (q_self && q_self[i] == j) continue;
            double dj = sqdist(q, R + j * ldr, d);
            if (cnt == k && !pair_less(dj, j, D[k - 1], I[k - 1])) continue;
            int p = (cnt < k) ? cnt++ : k - 1;
            while (p > 0 && pair_less(dj, j, D[p - 1], I[p - 1])) {
                D[p] = D[p - 1];
                I[p] = I[p - 1];
                --p;
            }
            D[p] = dj;
            I[p] = j;
        }
        if (cnt < k) bad = 1;
    }
    return bad ? -1 : 0;
}

/* Squared distances of given (row, col) pairs of X: out[e] = D(a[e], b[e]). */
void oracle_pair_d2(const double* X, int64_t ld, int d, const int64_t* a,
                    const int64_t* b, int64_t m, double* out)
{
    for (int64_t e = 0; e < m; ++e) out[e] = sqdist(X + a[e] * ld, X + b[e] * ld, d);
}

/* ------------------------------------------------------------- NNDescent */

typedef struct {
    int64_t* idx;   /* n x K */
    double* dist;   /* n x K, squared */
    uint8_t* isnew; /* n x K */
    int K;
} heaps_t;

/*
 * Update of Dong et al.: try to put w (at squared distance l) into u's list.
 * Returns 1 if the list changed.  The list stays sorted by (dist, idx); the
 * entry that enters is flagged new.
 */
static int heap_update(heaps_t* H, int64_t u, int64_t w, double l)
{
    const int K = H->K;
    int64_t* I = H->idx + u * K;
    double* D = H->dist + u * K;
    uint8_t* F = H->isnew + u * K;
    if (w == u) return 0;
    for (int r = 0; r < K; ++r)
        if (I[r] == w) return 0;
    if (!pair_less(l, w, D[K - 1], I[K - 1])) return 0;
    int p = K - 1;
    while (p > 0 && pair_less(l, w, D[p - 1], I[p - 1])) {
        D[p] = D[p - 1];
        I[p] = I[p - 1];
        F[p] = F[p - 1];
        --p;
    }
    D[p] = l;
    I[p] = w;
    F[p] = 1;
    return 1;
}

/* Sorted random init: K distinct uniform u != v, true distances, all new. */
static void nnd_random_init(const double* X, int64_t n, int64_t ld, int d,
                            heaps_t* H, uint64_t* rs)
{
    const int K = H->K;
    for (int64_t v = 0; v < n; ++v) {
        int64_t* I = H->idx + v * K;
        double* D = H->dist + v * K;
        uint8_t* F = H->isnew + v * K;
        int cnt = 0;
        while (cnt < K) {
            int64_t u = rng_below(rs, n);
            if (u == v) continue;
            int dup = 0;
            for (int r = 0; r < cnt; ++r)
                if (I[r] == u) dup = 1;
            if (dup) continue;
            double l = sqdist(X + v * ld, X + u * ld, d);
            int p = cnt++;
            while (p > 0 && pair_less(l, u, D[p - 1], I[p - 1])) {
                D[p] = D[p - 1];
                I[p] = I[p - 1];
                --p;
            }
            D[p] = l;
            I[p] = u;
        }
        for (int r = 0; r < K; ++r) F[r] = 1;
    }
}

/* Append u to list[v] (capacity cap) unless already there. */
static void set_add(int64_t* list, int* cnt, int cap, int64_t u)
{
    for (int r = 0; r < *cnt; ++r)
        if (list[r] == u) return;
    if (*cnt < cap) list[(*cnt)++] = u;
}

/* Uniform sample of min(s, m) items of a[0..m) without replacement
 * (partial Fisher-Yates on a scratch copy); writes them to out, returns count. */
static int sample_wo_repl(const int64_t* a, int m, int s, int64_t* out,
                          int64_t* scratch, uint64_t* rs)
{
    memcpy(scratch, a, sizeof(int64_t) * (size_t)m);
    int take = m < s ? m : s;
    for (int r = 0; r < take; ++r) {
        int64_t j = r + rng_below(rs, m - r);
        int64_t t = scratch[r];
        scratch[r] = scratch[j];
        scratch[j] = t;
        out[r] = scratch[r];
    }
    return take;
}

/*
 * Sequential NNDescent (Dong, Charikar & Li 2011, Algorithm 2 with sampling).
 *
 * K = working list size, rho = sample rate, S = ceil(rho*K) samples,
 * delta = early-termination rate.  init_idx (nullable, n x K, -1 = empty)
 * seeds the lists instead of random init; missing/invalid entries are
 * completed with random distinct indices.  On return out_idx / out_d2 hold
 * the n x K lists sorted by (dist, idx); iters_out the iterations run;
 * updates_out[t] (capacity max_iters) the update count of iteration t.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
/*
 * Optional trace of the first trace_iters iterations (every pointer NULL or
 * all set), for checking the sample / reverse steps against hand-worked
 * cases.  For iteration t and point v (-1 pads every list):
 *   tr_lidx / tr_lflag  [t][v][0..K)     v's list and new-flags as the
 *                                        iteration starts (before sampling);
 *   tr_newf [t][v][0..S)                 the forward new sample new[v];
 *   tr_oldf [t][v][0..K)                 the forward old list old[v];
 *   tr_new  [t][v][0..2S)                new[v] after the reverse union;
 *   tr_old  [t][v][0..K+S)               old[v] after the reverse union.
 */
int oracle_nndescent_traced(const double* X, int64_t n, int64_t ld, int d, int K,
                            int max_iters, double rho, double delta, uint64_t seed,
                            const int64_t* init_idx,
                            int64_t* out_idx, double* out_d2, int* iters_out,
                            int64_t* updates_out, int trace_iters,
                            int64_t* tr_lidx, uint8_t* tr_lflag, int64_t* tr_newf,
                            int64_t* tr_oldf, int64_t* tr_new, int64_t* tr_old)
{
    if (n < 2 || K < 1 || K > n - 1 || d < 1 || rho <= 0.0 || rho > 1.0 ||
        delta < 0.0 || max_iters < 0)
        return -1;
    const int S = (int)ceil(rho * K);
    heaps_t H;
    H.K = K;
    H.idx = out_idx;
    H.dist = out_d2;
    H.isnew = (uint8_t*)malloc((size_t)n * K);
    const int cap_new = 2 * S, cap_old = K + S;
    int64_t* newl = (int64_t*)malloc(sizeof(int64_t) * (size_t)n * cap_new);
    int64_t* oldl = (int64_t*)malloc(sizeof(int64_t) * (size_t)n * cap_old);
    int* nnew = (int*)malloc(sizeof(int) * (size_t)n);
    int* nold = (int*)malloc(sizeof(int) * (size_t)n);
    int64_t* rcnt_new = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* rcnt_old = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* rev_new = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n * S + 1));
    int64_t* rev_old = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n * K + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t* pick = (int64_t*)malloc(sizeof(int64_t) * (size_t)(K + 1));
    int64_t* scratch = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t* samp = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!H.isnew || !newl || !oldl || !nnew || !nold || !rcnt_new || !rcnt_old ||
        !rev_new || !rev_old || !fill || !pick || !scratch || !samp) {
        free(H.isnew); free(newl); free(oldl); free(nnew); free(nold);
        free(rcnt_new); free(rcnt_old); free(rev_new); free(rev_old);
        free(fill); free(pick); free(scratch); free(samp);
        return -1;
    }
    uint64_t rs = seed * 0xD1B54A32D192ED03ull + 1;

    /* step 1: init */
    if (!init_idx) {
        nnd_random_init(X, n, ld, d, &H, &rs);
    } else {
        for (int64_t v = 0; v < n; ++v) {
            int64_t* I = H.idx + v * K;
            double* D = H.dist + v * K;
            int cnt = 0;
            for (int r = 0; r < K; ++r) {
                int64_t u = init_idx[v * K + r];
                if (u < 0 || u >= n || u == v) continue;
                int dup = 0;
                for (int q = 0; q < cnt; ++q)
                    if (I[q] == u) dup = 1;
                if (!dup) I[cnt++] = u;
            }
            while (cnt < K) {
                int64_t u = rng_below(&rs, n);
                if (u == v) continue;
                int dup = 0;
                for (int q = 0; q < cnt; ++q)
                    if (I[q] == u) dup = 1;
                if (!dup) I[cnt++] = u;
            }
            for (int r = 0; r < K; ++r) D[r] = sqdist(X + v * ld, X + I[r] * ld, d);
            for (int r = 1; r < K; ++r) { /* insertion sort by (D, idx) */
                double dl = D[r];
                int64_t il = I[r];
                int p = r;
                while (p > 0 && pair_less(dl, il, D[p - 1], I[p - 1])) {
                    D[p] = D[p - 1];
                    I[p] = I[p - 1];
                    --p;
                }
                D[p] = dl;
                I[p] = il;
            }
            for (int r = 0; r < K; ++r) H.isnew[v * K + r] = 1;
        }
    }

    int it = 0;
    for (; it < max_iters; ++it) {
        const int tr = trace_iters > it && tr_lidx && tr_lflag && tr_newf && tr_oldf && tr_new && tr_old;
        if (tr) {
            memcpy(tr_lidx + (size_t)it * n * K, H.idx, sizeof(int64_t) * (size_t)n * K);
            memcpy(tr_lflag + (size_t)it * n * K, H.isnew, (size_t)n * K);
        }
        /* step 2: sample -- old = entries flagged old; new = S of the new ones */
        for (int64_t v = 0; v < n; ++v) {
            int64_t* I = H.idx + v * K;
            uint8_t* F = H.isnew + v * K;
            nold[v] = 0;
            nnew[v] = 0;
            int m = 0;
            for (int r = 0; r < K; ++r) {
                if (F[r]) pick[m++] = r;
                else oldl[v * cap_old + nold[v]++] = I[r];
            }
            int take = sample_wo_repl(pick, m, S, samp, scratch, &rs);
            for (int r = 0; r < take; ++r) {
                newl[v * cap_new + nnew[v]++] = I[samp[r]];
                F[samp[r]] = 0;
            }
        }
        if (tr) {
            for (int64_t v = 0; v < n; ++v) {
                int64_t* a = tr_newf + ((size_t)it * n + v) * S;
                int64_t* b = tr_oldf + ((size_t)it * n + v) * K;
                for (int r = 0; r < S; ++r) a[r] = r < nnew[v] ? newl[v * cap_new + r] : -1;
                for (int r = 0; r < K; ++r) b[r] = r < nold[v] ? oldl[v * cap_old + r] : -1;
            }
        }
        /* step 3: reverse lists (CSR, rows in increasing source order) */
        memset(rcnt_new, 0, sizeof(int64_t) * ((size_t)n + 1));
        memset(rcnt_old, 0, sizeof(int64_t) * ((size_t)n + 1));
        for (int64_t v = 0; v < n; ++v) {
            for (int r = 0; r < nnew[v]; ++r) rcnt_new[newl[v * cap_new + r] + 1]++;
            for (int r = 0; r < nold[v]; ++r) rcnt_old[oldl[v * cap_old + r] + 1]++;
        }
        for (int64_t u = 0; u < n; ++u) {
            rcnt_new[u + 1] += rcnt_new[u];
            rcnt_old[u + 1] += rcnt_old[u];
        }
        memcpy(fill, rcnt_new, sizeof(int64_t) * (size_t)n);
        for (int64_t v = 0; v < n; ++v)
            for (int r = 0; r < nnew[v]; ++r) {
                int64_t u = newl[v * cap_new + r];
                rev_new[fill[u]++] = v;
            }
        memcpy(fill, rcnt_old, sizeof(int64_t) * (size_t)n);
        for (int64_t v = 0; v < n; ++v)
            for (int r = 0; r < nold[v]; ++r) {
                int64_t u = oldl[v * cap_old + r];
                rev_old[fill[u]++] = v;
            }
        for (int64_t v = 0; v < n; ++v) {
            int m = (int)(rcnt_new[v + 1] - rcnt_new[v]);
            int take = sample_wo_repl(rev_new + rcnt_new[v], m, S, samp, scratch, &rs);
            for (int r = 0; r < take; ++r) set_add(newl + v * cap_new, &nnew[v], cap_new, samp[r]);
            m = (int)(rcnt_old[v + 1] - rcnt_old[v]);
            take = sample_wo_repl(rev_old + rcnt_old[v], m, S, samp, scratch, &rs);
            for (int r = 0; r < take; ++r) set_add(oldl + v * cap_old, &nold[v], cap_old, samp[r]);
        }
        if (tr) {
            for (int64_t v = 0; v < n; ++v) {
                int64_t* a = tr_new + ((size_t)it * n + v) * cap_new;
                int64_t* b = tr_old + ((size_t)it * n + v) * cap_old;
                for (int r = 0; r < cap_new; ++r) a[r] = r < nnew[v] ? newl[v * cap_new + r] : -1;
                for (int r = 0; r < cap_old; ++r) b[r] = r < nold[v] ? oldl[v * cap_old + r] : -1;
            }
        }
        /* step 4: local join, updates applied immediately */
        int64_t c = 0;
        for (int64_t v = 0; v < n; ++v) {
            const int64_t* nw = newl + v * cap_new;
            const int64_t* od = oldl + v * cap_old;
            for (int a = 0; a < nnew[v]; ++a) {
                int64_t u1 = nw[a];
                for (int b = a + 1; b < nnew[v]; ++b) {
                    int64_t u2 = nw[b];
                    if (u1 == u2) continue;
                    double l = sqdist(X + u1 * ld, X + u2 * ld, d);
                    c += heap_update(&H, u1, u2, l);
                    c += heap_update(&H, u2, u1, l);
                }
                for (int b = 0; b < nold[v]; ++b) {
                    int64_t u2 = od[b];
                    if (u1 == u2) continue;
                    double l = sqdist(X + u1 * ld, X + u2 * ld, d);
                    c += heap_update(&H, u1, u2, l);
                    c += heap_update(&H, u2, u1, l);
                }
            }
        }
        if (updates_out) updates_out[it] = c;
        /* step 6: early termination */
        if ((double)c < delta * (double)n * (double)K) {
            ++it;
            break;
        }
    }
    if (iters_out) *iters_out = it;
    free(H.isnew); free(newl); free(oldl); free(nnew); free(nold);
    free(rcnt_new); free(rcnt_old); free(rev_new); free(rev_old);
    free(fill); free(pick); free(scratch); free(samp);
    return 0;
}

/* The same without a trace. */
int oracle_nndescent(const double* X, int64_t n, int64_t ld, int d, int K,
                     int max_iters, double rho, double delta, uint64_t seed,
                     const int64_t* init_idx,
                     int64_t* out_idx, double* out_d2, int* iters_out,
                     int64_t* updates_out)
{
    return oracle_nndescent_traced(X, n, ld, d, K, max_iters, rho, delta, seed, init_idx,
                                   out_idx, out_d2, iters_out, updates_out, 0,
                                   NULL, NULL, NULL, NULL, NULL, NULL);
}

/* ------------------------------------------------------------- rounding */

/* FP32 -> BF16, round to nearest, ties to even, by the bit definition:
 * add 0x7FFF plus the lowest kept bit, keep the top 16 bits; NaN stays NaN. */
void oracle_round_bf16(const float* in, uint16_t* out, int64_t m)
{
    for (int64_t e = 0; e < m; ++e) {
        uint32_t u;
        memcpy(&u, &in[e], 4);
        if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
            out[e] = (uint16_t)((u >> 16) | 0x0040u);
            continue;
        }
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7FFFu + lsb;
        out[e] = (uint16_t)(u >> 16);
    }
}

/* ------------------------------------------------------- seeding encoder */

/*
 * Encoder z = W2^T relu(W1^T x + b1) + b2 with W1: d x h1 (row-major),
 * W2: h1 x h2.  H (nullable) receives the post-ReLU hidden layer (m x h1).
 */
void oracle_mlp_forward(const double* X, int64_t m, int64_t ld, int d,
                        const double* W1, const double* b1, int h1,
                        const double* W2, const double* b2, int h2,
                        double* H, double* Z)
{
    double* hid = (double*)malloc(sizeof(double) * (size_t)h1);
    for (int64_t i = 0; i < m; ++i) {
        const double* x = X + i * ld;
        for (int j = 0; j < h1; ++j) {
            double s = b1[j];
            for (int t = 0; t < d; ++t) s += x[t] * W1[t * h1 + j];
            hid[j] = s > 0.0 ? s : 0.0;
            if (H) H[i * h1 + j] = hid[j];
        }
        for (int o = 0; o < h2; ++o) {
            double s = b2[o];
            for (int j = 0; j < h1; ++j) s += hid[j] * W2[j * h2 + o];
            Z[i * h2 + o] = s;
        }
    }
    free(hid);
}

/*
 * Triplet loss over B triplets whose embeddings are the rows of Z laid out as
 * [anchors (B rows); positives (B rows); negatives (B rows)], width h2:
 *   loss = (1/B) sum_b max(0, margin + |za-zp|^2 - |za-zn|^2).
 * dZ (nullable, 3B x h2) receives d loss / d Z.  Returns the loss.
 */
double oracle_triplet_loss(const double* Z, int64_t B, int h2, double margin, double* dZ)
{
    double loss = 0.0;
    if (dZ) memset(dZ, 0, sizeof(double) * (size_t)(3 * B * h2));
    for (int64_t b = 0; b < B; ++b) {
        const double* za = Z + b * h2;
        const double* zp = Z + (B + b) * h2;
        const double* zn = Z + (2 * B + b) * h2;
        double dp = 0.0, dn = 0.0;
        for (int o = 0; o < h2; ++o) {
            dp += (za[o] - zp[o]) * (za[o] - zp[o]);
            dn += (za[o] - zn[o]) * (za[o] - zn[o]);
        }
        double g = margin + dp - dn;
        if (g <= 0.0) continue;
        loss += g;
        if (dZ) {
            double s = 2.0 / (double)B;
            for (int o = 0; o < h2; ++o) {
                dZ[b * h2 + o] += s * (zn[o] - zp[o]);
                dZ[(B + b) * h2 + o] += s * (zp[o] - za[o]);
                dZ[(2 * B + b) * h2 + o] += s * (za[o] - zn[o]);
            }
        }
    }
    return loss / (double)B;
}

/*
 * Backward pass of the encoder for rows X (m x d) given dZ (m x h2):
 * gW1 = X^T (dH .* [pre > 0]), gb1 = column sums of that, gW2 = H^T dZ,
 * gb2 = column sums of dZ, with dH = dZ W2^T.  Gradients are overwritten.
 */
void oracle_mlp_backward(const double* X, int64_t m, int64_t ld, int d,
                         const double* W1, const double* b1, int h1,
                         const double* W2, int h2, const double* dZ,
                         double* gW1, double* gb1, double* gW2, double* gb2)
{
    memset(gW1, 0, sizeof(double) * (size_t)d * h1);
    memset(gb1, 0, sizeof(double) * (size_t)h1);
    memset(gW2, 0, sizeof(double) * (size_t)h1 * h2);
    memset(gb2, 0, sizeof(double) * (size_t)h2);
    double* pre = (double*)malloc(sizeof(double) * (size_t)h1);
    double* dh = (double*)malloc(sizeof(double) * (size_t)h1);
    for (int64_t i = 0; i < m; ++i) {
        const double* x = X + i * ld;
        const double* dz = dZ + i * h2;
        for (int j = 0; j < h1; ++j) {
            double s = b1[j];
            for (int t = 0; t < d; ++t) s += x[t] * W1[t * h1 + j];
            pre[j] = s;
        }
        for (int o = 0; o < h2; ++o) gb2[o] += dz[o];
        for (int j = 0; j < h1; ++j) {
            double hj = pre[j] > 0.0 ? pre[j] : 0.0;
            double acc = 0.0;
            for (int o = 0; o < h2; ++o) {
                gW2[j * h2 + o] += hj * dz[o];
                acc += dz[o] * W2[j * h2 + o];
            }
            dh[j] = pre[j] > 0.0 ? acc : 0.0;
        }
        for (int j = 0; j < h1; ++j) {
            gb1[j] += dh[j];
            for (int t = 0; t < d; ++t) gW1[t * h1 + j] += x[t] * dh[j];
        }
    }
    free(pre);
    free(dh);
}

/* One Adam step (Kingma & Ba 2015) on m parameters; t is the 1-based step. */
void oracle_adam_step(double* w, const double* g, double* mom, double* vel, int64_t m,
                      double lr, double beta1, double beta2, double eps, int t)
{
    double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t e = 0; e < m; ++e) {
        mom[e] = beta1 * mom[e] + (1.0 - beta1) * g[e];
        vel[e] = beta2 * vel[e] + (1.0 - beta2) * g[e] * g[e];
        double mh = mom[e] / c1, vh = vel[e] / c2;
        w[e] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ---------------------------------------------- sorted-projection seeding */

typedef struct {
    uint32_t key;
    int64_t idx;
} keyed_t;

static int keyed_cmp(const void* a, const void* b)
{
    const keyed_t* x = (const keyed_t*)a;
    const keyed_t* y = (const keyed_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Order-preserving map of an FP32 value to uint32 (both zeros map alike). */
static uint32_t f32_order(float f)
{
    uint32_t u;
    if (f == 0.0f) return 0x80000000u;
    memcpy(&u, &f, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

/*
 * Seed lists from sorted projections of an embedding Z (n x m).
 *
 * Curve p (0 <= p < P) uses the D directions dirs[p*D .. p*D+D) (each of
 * length m).  Projections are FP32 sums of products taken in coordinate
 * order with fused multiply-adds, because the order they decide must be the
 * one the kernel decides.  D = 1: the key is the projection itself (order-
 * preserving uint32).  D > 1: each projection is quantised to b = 32 / D bits
 * over its range [lo, hi] across all points, q = min(floor((y - lo) * s),
 * 2^b - 1) with s = 2^b / (hi - lo) in FP32, and the key interleaves the bits
 * of q_0..q_{D-1} from the most significant level down (a Z-order code).
 * Points are sorted by (key, index).  Each point's candidates are the w
 * predecessors and w successors in every order; self and repeats are
 * removed; candidates are ranked by exact squared input distance D and the
 * best K kept, sorted by (D, idx).  Rows with fewer than K candidates are
 * padded with -1 / +inf.
 */
/*
 * Order keys of one curve (see below): directions r_0..r_{D-1} (rows of dirs,
 * length m).  y is scratch of n*D floats.  Returns 0, or -1 on bad D.
 */
int oracle_proj_keys(const float* Z, int64_t n, int m, const float* dirs, int Dk,
                     uint32_t* keys, float* y)
{
    if (Dk < 1 || 32 % Dk != 0) return -1;
    const int bits = 32 / Dk;
    for (int j = 0; j < Dk; ++j) {
        const float* r = dirs + (size_t)j * m;
        for (int64_t i = 0; i < n; ++i) {
            float s = 0.0f;
            for (int t = 0; t < m; ++t) s = fmaf(Z[i * m + t], r[t], s);
            y[(size_t)j * n + i] = s;
        }
    }
    if (Dk == 1) {
        for (int64_t i = 0; i < n; ++i) keys[i] = f32_order(y[i]);
        return 0;
    }
    for (int j = 0; j < Dk; ++j) {
        float lo = y[(size_t)j * n], hi = lo;
        for (int64_t i = 1; i < n; ++i) {
            float v = y[(size_t)j * n + i];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        const float sc = hi > lo ? (float)(1u << bits) / (hi - lo) : 0.0f;
        const uint32_t qmax = (1u << bits) - 1u;
        for (int64_t i = 0; i < n; ++i) {
            float f = floorf((y[(size_t)j * n + i] - lo) * sc);
            uint32_t q = f <= 0.0f ? 0u : (uint32_t)f;
            y[(size_t)j * n + i] = (float)(q < qmax ? q : qmax);   /* reuse as the code */
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        uint32_t key = 0;
        for (int l = bits - 1; l >= 0; --l)
            for (int j = 0; j < Dk; ++j)
                key = (key << 1) | (((uint32_t)y[(size_t)j * n + i] >> l) & 1u);
        keys[i] = key;
    }
    return 0;
}

int oracle_proj_seed(const double* X, int64_t n, int64_t ld, int d,
                     const float* Z, int m, const float* dirs, int P, int Dk, int w, int K,
                     int64_t* out_idx, double* out_d2)
{
    if (n < 2 || K < 1 || w < 1 || P < 1 || Dk < 1 || 32 % Dk != 0) return -1;
    keyed_t* ord = (keyed_t*)malloc(sizeof(keyed_t) * (size_t)n * P);
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)n * P);
    float* y = (float*)malloc(sizeof(float) * (size_t)n * Dk);
    uint32_t* keys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    int cap = 2 * w * P;
    int64_t* cand = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    if (!ord || !pos || !y || !keys || !cand) {
        free(ord); free(pos); free(y); free(keys); free(cand);
        return -1;
    }
    for (int p = 0; p < P; ++p) {
        keyed_t* o = ord + (size_t)p * n;
        oracle_proj_keys(Z, n, m, dirs + (size_t)p * Dk * m, Dk, keys, y);
        for (int64_t i = 0; i < n; ++i) {
            o[i].idx = i;
            o[i].key = keys[i];
        }
        qsort(o, (size_t)n, sizeof(keyed_t), keyed_cmp);
        for (int64_t r = 0; r < n; ++r) pos[(size_t)p * n + o[r].idx] = r;
    }
    for (int64_t i = 0; i < n; ++i) {
        int nc = 0;
        for (int p = 0; p < P; ++p) {
            const keyed_t* o = ord + (size_t)p * n;
            int64_t r0 = pos[(size_t)p * n + i];
            for (int64_t r = r0 - w; r <= r0 + w; ++r) {
                if (r < 0 || r >= n || r == r0) continue;
                int64_t u = o[r].idx;
                int dup = 0;
                for (int q = 0; q < nc; ++q)
                    if (cand[q] == u) dup = 1;
                if (!dup) cand[nc++] = u;
            }
        }
        int64_t* I = out_idx + i * K;
        double* Dd = out_d2 + i * K;
        int cnt = 0;
        for (int q = 0; q < nc; ++q) {
            int64_t u = cand[q];
            double l = sqdist(X + i * ld, X + u * ld, d);
            if (cnt == K && !pair_less(l, u, Dd[K - 1], I[K - 1])) continue;
            int pp = (cnt < K) ? cnt++ : K - 1;
            while (pp > 0 && pair_less(l, u, Dd[pp - 1], I[pp - 1])) {
                Dd[pp] = Dd[pp - 1];
                I[pp] = I[pp - 1];
                --pp;
            }
            Dd[pp] = l;
            I[pp] = u;
        }
        for (int r = cnt; r < K; ++r) {
            I[r] = -1;
            Dd[r] = INFINITY;
        }
    }
    free(ord);
    free(pos);
    free(y);
    free(keys);
    free(cand);
    return 0;
}

/* ------------------------------------------- fuzzy graph (UMAP weights) */

/*
 * Membership strengths of each point's k-NN edges, as UMAP defines them
 * (McInnes, Healy & Melville 2018; the graph every UMAP-family method of the
 * paper builds from the shared k-NN stage).  For row i with neighbour
 * distances d_1..d_k (Euclidean, self excluded):
 *   rho_i   = the smallest positive d_r (0 if none is positive);
 *   sigma_i > 0 solves  sum_r exp(-max(0, d_r - rho_i) / sigma_i) = log2(k);
 *   w_ir    = exp(-max(0, d_r - rho_i) / sigma_i).
 * The sum falls from k (sigma -> inf) to c_i = #{r : d_r <= rho_i}
 * (sigma -> 0), so a root exists iff c_i < log2(k).  Otherwise sigma_i = 0
 * and the weights are the limit: 1 where d_r <= rho_i, else 0.
 * sigma is found by bisection in double: a bracket [0, hi] whose hi doubles
 * from max(d_r - rho_i) until the sum reaches log2(k), halved until no
 * double lies strictly inside.
 */
static double fuzzy_sum(const double* x, int k, double sigma)
{
    double s = 0.0;
    for (int r = 0; r < k; ++r) s += exp(-x[r] / sigma);
    return s;
}

void oracle_fuzzy_rows(const double* dist, int64_t n, int k, double* rho, double* sigma, double* w)
{
    double* x = (double*)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    const double target = log2((double)k);
    for (int64_t i = 0; i < n; ++i) {
        const double* d = dist + i * k;
        double p = 0.0;
        for (int r = 0; r < k; ++r)
            if (d[r] > 0.0 && (p == 0.0 || d[r] < p)) p = d[r];
        int cnt = 0;
        double xmax = 0.0;
        for (int r = 0; r < k; ++r) {
            x[r] = d[r] - p > 0.0 ? d[r] - p : 0.0;
            if (x[r] == 0.0) ++cnt;
            if (x[r] > xmax) xmax = x[r];
        }
        rho[i] = p;
        if ((double)cnt >= target) {
            sigma[i] = 0.0;
            for (int r = 0; r < k; ++r) w[i * k + r] = x[r] == 0.0 ? 1.0 : 0.0;
            continue;
        }
        double lo = 0.0, hi = xmax;
        while (fuzzy_sum(x, k, hi) < target) hi *= 2.0;
        for (;;) {
            const double mid = 0.5 * (lo + hi);
            if (!(mid > lo && mid < hi)) break;
            if (fuzzy_sum(x, k, mid) < target) lo = mid;
            else hi = mid;
        }
        sigma[i] = hi;
        for (int r = 0; r < k; ++r) w[i * k + r] = exp(-x[r] / hi);
    }
    free(x);
}

/* -------------------------------------------- embedding-quality metrics */

/*
 * Canonical FP32 squared distance of two rows given as doubles holding FP32
 * values: coordinate t goes to partial sum t mod 16 (fused multiply-add of
 * the FP32 difference, in coordinate order), then the 16 partial sums are
 * added pairwise at strides 8, 4, 2, 1.  This is the precision in which the
 * GPU path ranks points (its exact k-NN re-rank and its rank counts), so
 * rank decisions compared bit for bit are taken in it on both sides.
 */
static double sqdist_f32c(const double* a, const double* b, int d)
{
    float s[16];
    for (int g = 0; g < 16; ++g) s[g] = 0.0f;
    for (int t = 0; t < d; ++t) {
        float e = (float)a[t] - (float)b[t];
        s[t & 15] = fmaf(e, e, s[t & 15]);
    }
    for (int j = 8; j > 0; j >>= 1) {
        float u[16];
        for (int g = 0; g < 16; ++g) u[g] = s[g] + s[g ^ j];
        for (int g = 0; g < 16; ++g) s[g] = u[g];
    }
    return (double)s[0];
}

typedef struct {
    double d;
    int64_t j;
} dj_t;

static int dj_cmp(const void* x, const void* y)
{
    const dj_t* a = (const dj_t*)x;
    const dj_t* b = (const dj_t*)y;
    if (a->d != b->d) return a->d < b->d ? -1 : 1;
    return (a->j > b->j) - (a->j < b->j);
}

/* rank[j] (1 = nearest) of every j != i by (distance, index) from row i of
 * A (n x w); rank[i] = 0.  scratch holds n entries. */
static void ranks_from(const double* A, int64_t n, int w, int64_t i, int canonical, dj_t* scratch,
                       int64_t* rank)
{
    int64_t m = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        scratch[m].d = canonical ? sqdist_f32c(A + i * w, A + j * w, w) : sqdist(A + i * w, A + j * w, w);
        scratch[m].j = j;
        ++m;
    }
    qsort(scratch, (size_t)m, sizeof(dj_t), dj_cmp);
    rank[i] = 0;
    for (int64_t r = 0; r < m; ++r) rank[scratch[r].j] = r + 1;
}

/*
 * Per-row terms of k-NN preservation, trustworthiness and continuity
 * (Venna & Kaski 2006; the paper's section "Embedding Quality") for the
 * rows listed in `rows`: with r(i,j) the rank of j from i among all other
 * points by high-dimensional distance (rows of X, n x d) and r'(i,j) by
 * embedding distance (rows of Y, n x e), N(i) = {j : r(i,j) <= k} and
 * L(i) = {j : r'(i,j) <= k}:
 *   hits[q]  = |N(i) intersect L(i)|,
 *   trust[q] = sum over j in L(i) \ N(i) of (r(i,j) - k),
 *   cont[q]  = sum over j in N(i) \ L(i) of (r'(i,j) - k).
 * Ranks break distance ties by the smaller index.  canonical = 0 ranks by
 * FP64 direct differences, 1 by the canonical FP32 distance above.
 */
int oracle_quality_rows(const double* X, int d, const double* Y, int e, int64_t n, int k,
                        const int64_t* rows, int64_t nrows, int canonical,
                        int64_t* hits, int64_t* trust, int64_t* cont)
{
    if (k < 1 || k >= n || d < 1 || e < 1) return -1;
    int bad = 0;
#pragma omp parallel
    {
        dj_t* scratch = (dj_t*)malloc(sizeof(dj_t) * (size_t)n);
        int64_t* rx = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        int64_t* ry = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        if (!scratch || !rx || !ry) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int64_t q = 0; q < nrows; ++q) {
                const int64_t i = rows[q];
                ranks_from(X, n, d, i, canonical, scratch, rx);
                ranks_from(Y, n, e, i, canonical, scratch, ry);
                int64_t h = 0, t = 0, c = 0;
                for (int64_t j = 0; j < n; ++j) {
                    if (j == i) continue;
                    const int inN = rx[j] <= k, inL = ry[j] <= k;
                    if (inN && inL) ++h;
                    if (inL && !inN) t += rx[j] - k;
                    if (inN && !inL) c += ry[j] - k;
                }
                hits[q] = h;
                trust[q] = t;
                cont[q] = c;
            }
        }
        free(scratch);
        free(rx);
        free(ry);
    }
    return bad ? -1 : 0;
}
