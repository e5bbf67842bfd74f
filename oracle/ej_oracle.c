/*
 * ej_oracle.c -- plain, slow CPU oracle for EmbedJoin (Zhang & Zhang,
 * "EmbedJoin: Efficient Edit Similarity Joins via Embeddings").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * GPU path.
 *
 * Everything is computed the direct way, one string and one table at a time,
 * in the order the paper states it:
 *   - Algorithm 1 (CGK embedding) materialises every one of the L output
 *     symbols of the walk, then the LSH coordinates are read from it;
 *   - Section 4 "two-level hashing": a signature u in {1..|S|+1}^m is hashed
 *     to <u, v> mod P with 128-bit intermediates;
 *   - Algorithm 3 (EmbedJoin) keeps one chained hash table per (seed, LSH
 *     function), visits the strings in length order, probes, applies the
 *     length test / eviction, inserts, and de-duplicates the pairs found in
 *     each iteration;
 *   - Section 3.3 (Ukkonen): threshold edit distance on the 2K+1 diagonals
 *     with an early exit once a whole row of the band exceeds K.
 *
 * Randomness (the paper only says "random string" and "random hash
 * function"): every random word is W(key, c) = Mix64(key + (c+1)*GAMMA),
 * i.e. the (c+1)-th output of a SplitMix64 generator seeded with `key`
 * (Steele, Lea, Flood, OOPSLA 2014).  Stream keys are W(seed, tag<<32|idx)
 * with tag 0 = the CGK random string R of seed l (idx = l), tag 1 = LSH
 * coordinates of table (l, j) (idx = l*z + j), tag 2 = the second-level hash
 * vector of table (l, j).
 *   R bit b          = bit (b mod 64) of W(key_R, b / 64)
 *   coordinate k     = floor(W(key_POS, k) * L / 2^64)       (with replacement)
 *   v_k              = (W(key_V, k) >> 3) mod P,   P = 2^61 - 1
 * Symbol codes: the alphabet is the sorted set of distinct input bytes, code
 * of the k-th smallest byte is k-1, and the padding symbol (bottom) is |S|.
 * A sampled symbol c maps to u = c + 1, so bottom maps to |S| + 1.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EJO_P ((1ULL << 61) - 1ULL)
#define EJO_GAMMA 0x9E3779B97F4A7C15ULL

/* ---------------------------------------------------------------- RNG -- */

uint64_t ejo_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Plain sequential SplitMix64: the state advances by GAMMA per draw. */
void ejo_splitmix64_stream(uint64_t seed, uint64_t count, uint64_t *out) {
    uint64_t s = seed;
    for (uint64_t i = 0; i < count; i++) {
        s += EJO_GAMMA;
        out[i] = ejo_mix64(s);
    }
}

/* The c-th word (0-based) of the stream seeded with `key`.  The generator's
 * state after c+1 draws is key + (c+1)*GAMMA (a Weyl sequence), so the word
 * is the output function applied to that state. */
uint64_t ejo_word(uint64_t key, uint64_t c) {
    return ejo_mix64(key + (c + 1ULL) * EJO_GAMMA);
}

uint64_t ejo_stream_key(uint64_t seed, uint32_t tag, uint32_t idx) {
    return ejo_word(seed, ((uint64_t)tag << 32) | (uint64_t)idx);
}

/* Draws the randomness of one run.
 *   Rbits[l][b]  for b < L*sigma : the first L*|S| bits of R^l as 0/1 bytes
 *   pos[l][j][k] in [0, L)        : coordinate k of LSH function f_j^l
 *   v[l][j][k]   in [0, P)        : second-level vector of table (l, j)     */
void ejo_draw(uint64_t seed, uint32_t r, uint32_t z, uint32_t m, uint32_t L,
              uint32_t sigma, uint8_t *Rbits, uint32_t *pos, uint64_t *v) {
    uint64_t nbits = (uint64_t)L * sigma;
    for (uint32_t l = 0; l < r; l++) {
        uint64_t key = ejo_stream_key(seed, 0, l);
        uint64_t nwords = (nbits + 63) / 64;
        uint64_t *words = (uint64_t *)malloc(sizeof(uint64_t) * (nwords ? nwords : 1));
        ejo_splitmix64_stream(key, nwords, words);
        for (uint64_t b = 0; b < nbits; b++)
            Rbits[l * nbits + b] = (uint8_t)((words[b / 64] >> (b % 64)) & 1ULL);
        free(words);
    }
    for (uint32_t l = 0; l < r; l++) {
        for (uint32_t j = 0; j < z; j++) {
            uint64_t kp = ejo_stream_key(seed, 1, l * z + j);
            uint64_t kv = ejo_stream_key(seed, 2, l * z + j);
            uint64_t *wp = (uint64_t *)malloc(sizeof(uint64_t) * m);
            uint64_t *wv = (uint64_t *)malloc(sizeof(uint64_t) * m);
            ejo_splitmix64_stream(kp, m, wp);
            ejo_splitmix64_stream(kv, m, wv);
            for (uint32_t k = 0; k < m; k++) {
                unsigned __int128 prod = (unsigned __int128)wp[k] * (unsigned __int128)L;
                pos[((uint64_t)l * z + j) * m + k] = (uint32_t)(prod >> 64);
                v[((uint64_t)l * z + j) * m + k] = (wv[k] >> 3) % EJO_P;
            }
            free(wp);
            free(wv);
        }
    }
}

/* ----------------------------------------------------------- alphabet -- */

/* Sorted distinct bytes; lut[b] = code or -1.  Returns |S|. */
int ejo_alphabet(const uint8_t *chars, uint64_t total, int32_t *lut) {
    int present[256];
    memset(present, 0, sizeof(present));
    for (uint64_t i = 0; i < total; i++) present[chars[i]] = 1;
    int sigma = 0;
    for (int b = 0; b < 256; b++) lut[b] = present[b] ? sigma++ : -1;
    return sigma;
}

/* ------------------------------------------------- Algorithm 1 (CGK) -- */

/* Embeds x (symbol codes, length len) with random bits Rbits (0/1 bytes,
 * pi_j(sigma_k) = Rbits[(j-1)*sigma + (k-1)] in the paper's 1-based terms)
 * into out[0..L).  Pointer i starts at the first character; at every step
 * the current character is emitted and i moves on iff pi_j(x[i]) = 1; once i
 * is past the end the padding symbol `sigma` is emitted. */
void ejo_cgk_embed(const uint8_t *x, uint32_t len, const uint8_t *Rbits,
                   uint32_t sigma, uint32_t L, uint8_t *out) {
    uint64_t i = 0;
    for (uint64_t j = 0; j < L; j++) {
        if (i < len) {
            out[j] = x[i];
            i += Rbits[j * sigma + x[i]];
        } else {
            out[j] = (uint8_t)sigma;
        }
    }
}

/* Section 4, two-level hashing: <u, v> mod P with u_k = t[pos_k] + 1. */
uint64_t ejo_key(const uint8_t *t, const uint32_t *pos, const uint64_t *v, uint32_t m) {
    unsigned __int128 acc = 0;
    for (uint32_t k = 0; k < m; k++) {
        uint64_t u = (uint64_t)t[pos[k]] + 1ULL;
        acc += (unsigned __int128)u * (unsigned __int128)v[k];
        acc %= EJO_P;
    }
    return (uint64_t)acc;
}

/* ------------------------------------------------ edit distance (3.3) -- */

/* Textbook Wagner-Fischer, full table, two rows. */
uint32_t ejo_ed_full(const uint8_t *x, uint32_t lx, const uint8_t *y, uint32_t ly) {
    uint32_t *prev = (uint32_t *)malloc(sizeof(uint32_t) * (ly + 1));
    uint32_t *cur = (uint32_t *)malloc(sizeof(uint32_t) * (ly + 1));
    for (uint32_t j = 0; j <= ly; j++) prev[j] = j;
    for (uint32_t i = 1; i <= lx; i++) {
        cur[0] = i;
        for (uint32_t j = 1; j <= ly; j++) {
            uint32_t best = prev[j - 1] + (x[i - 1] != y[j - 1]);
            if (prev[j] + 1 < best) best = prev[j] + 1;
            if (cur[j - 1] + 1 < best) best = cur[j - 1] + 1;
            cur[j] = best;
        }
        uint32_t *t = prev; prev = cur; cur = t;
    }
    uint32_t d = prev[ly];
    free(prev);
    free(cur);
    return d;
}

/* Ukkonen's threshold algorithm: only cells with |i - j| <= K are filled
 * (cells outside the band count as infinite); a row whose band cells all
 * exceed K ends the computation.  Returns ED(x, y) if it is <= K, else K+1. */
uint32_t ejo_ed_banded(const uint8_t *x, uint32_t lx, const uint8_t *y, uint32_t ly,
                       uint32_t K) {
    const uint32_t INF = 0xFFFFFFF0u;
    uint32_t diff = lx > ly ? lx - ly : ly - lx;
    if (diff > K) return K + 1;
    uint32_t *prev = (uint32_t *)malloc(sizeof(uint32_t) * (ly + 1));
    uint32_t *cur = (uint32_t *)malloc(sizeof(uint32_t) * (ly + 1));
    for (uint32_t j = 0; j <= ly; j++) prev[j] = (j <= K) ? j : INF;
    uint32_t result = K + 1;
    int done = 0;
    for (uint32_t i = 1; i <= lx && !done; i++) {
        uint32_t jlo = (i > K) ? i - K : 0;
        uint32_t jhi = (i + K < ly) ? i + K : ly;
        /* the cells just outside the band are infinite */
        if (jlo >= 1) cur[jlo - 1] = INF;
        if (jhi + 1 <= ly) cur[jhi + 1] = INF;
        uint32_t rowmin = INF;
        for (uint32_t j = jlo; j <= jhi; j++) {
            uint32_t best;
            if (j == 0) {
                best = i;
            } else {
                best = prev[j - 1] + (x[i - 1] != y[j - 1]);
                if (prev[j] != INF && prev[j] + 1 < best) best = prev[j] + 1;
                if (cur[j - 1] != INF && cur[j - 1] + 1 < best) best = cur[j - 1] + 1;
            }
            if (best > INF) best = INF;
            cur[j] = best;
            if (best < rowmin) rowmin = best;
        }
        if (rowmin > K) done = 1;
        uint32_t *t = prev; prev = cur; cur = t;
    }
    if (!done && prev[ly] <= K) result = prev[ly];
    free(prev);
    free(cur);
    return result;
}

/* -------------------------------------------------- Algorithm 2 + 3 ----- */

typedef struct {
    uint64_t key;
    uint32_t *ids;
    uint32_t count, cap;
    int used;
} ejo_bucket;

typedef struct {
    ejo_bucket *slots;
    uint64_t nslots; /* power of two */
} ejo_table;

static void table_init(ejo_table *t, uint64_t nslots) {
    t->nslots = nslots;
    t->slots = (ejo_bucket *)calloc(nslots, sizeof(ejo_bucket));
}

static void table_free(ejo_table *t) {
    for (uint64_t s = 0; s < t->nslots; s++) free(t->slots[s].ids);
    free(t->slots);
}

/* Linear probing on the key; returns the bucket holding `key`, creating it. */
static ejo_bucket *table_bucket(ejo_table *t, uint64_t key) {
    uint64_t h = ejo_mix64(key) & (t->nslots - 1);
    while (t->slots[h].used && t->slots[h].key != key) h = (h + 1) & (t->nslots - 1);
    if (!t->slots[h].used) {
        t->slots[h].used = 1;
        t->slots[h].key = key;
    }
    return &t->slots[h];
}

static void bucket_push(ejo_bucket *b, uint32_t id) {
    if (b->count == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 4;
        b->ids = (uint32_t *)realloc(b->ids, sizeof(uint32_t) * b->cap);
    }
    b->ids[b->count++] = id;
}

/* Sort order of Algorithm 2: length, then bytes, then original position. */
static const uint8_t *g_chars;
static const uint64_t *g_offsets;
static int cmp_len_alpha(const void *pa, const void *pb) {
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    uint64_t la = g_offsets[a + 1] - g_offsets[a], lb = g_offsets[b + 1] - g_offsets[b];
    if (la != lb) return la < lb ? -1 : 1;
    int c = memcmp(g_chars + g_offsets[a], g_chars + g_offsets[b], la);
    if (c) return c < 0 ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static int cmp_u64(const void *pa, const void *pb) {
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Result of one join.  All indices are positions in the input.  Arrays are
 * malloc'ed here and released with ejo_result_free. */
typedef struct {
    uint32_t sigma, L;
    uint64_t n_raw;      /* pairs found by the tables before de-duplication */
    uint64_t n_cand;
    uint64_t *cand;      /* (i << 32) | j, i < j, sorted */
    uint32_t *cand_dist; /* min(ED, K+1) per candidate */
    uint64_t n_out;
    uint64_t *out;       /* (i << 32) | j, i < j, ED <= K, sorted */
    uint32_t *out_dist;
    uint64_t *keys;      /* [r*z][n], table-major, input order */
    uint8_t *sig;        /* [n][r][z][m] sampled symbols (codes), input order */
} ejo_result;

void ejo_result_free(ejo_result *res) {
    free(res->cand);
    free(res->cand_dist);
    free(res->out);
    free(res->out_dist);
    free(res->keys);
    free(res->sig);
    memset(res, 0, sizeof(*res));
}

/* Truncation length actually used: L_req, or ceil(average length) when 0,
 * never more than 3N (the full output length of Algorithm 1) and at least 1. */
uint32_t ejo_effective_L(const uint64_t *offsets, uint32_t n, uint32_t L_req) {
    uint64_t total = n ? offsets[n] - offsets[0] : 0, N = 0;
    for (uint32_t i = 0; i < n; i++) {
        uint64_t li = offsets[i + 1] - offsets[i];
        if (li > N) N = li;
    }
    uint64_t L = L_req;
    if (L == 0) L = n ? (total + n - 1) / n : 1;
    if (L > 3 * N) L = 3 * N;
    if (L == 0) L = 1;
    return (uint32_t)L;
}

/* Options of ejo_join_opts.  They only leave work out; none changes a value
 * that is computed. */
#define EJO_STOP_AFTER_CANDIDATES 1u /* the candidate set C only: no verification */
#define EJO_NO_SIG 2u                /* do not keep the sampled symbols */

/* EmbedJoin (Algorithm 3 with Algorithm 2 as preprocessing).
 * explicit_R (r * L * sigma 0/1 bytes), explicit_pos and explicit_v replace
 * the drawn randomness when non-NULL (used to replay the paper's running
 * example).  Returns 0 on success, -1 for r, z or m of 0, -2 when all 256
 * byte values occur (the padding symbol needs a code of its own). */
int ejo_join_opts(const uint8_t *chars, const uint64_t *offsets, uint32_t n, uint32_t K,
                  uint32_t r, uint32_t z, uint32_t m, uint32_t L_req, uint64_t seed,
                  const uint8_t *explicit_R, const uint32_t *explicit_pos,
                  const uint64_t *explicit_v, uint32_t opts, ejo_result *res) {
    memset(res, 0, sizeof(*res));
    if (r == 0 || z == 0 || m == 0) return -1;
    uint64_t total = n ? offsets[n] - offsets[0] : 0;
    int32_t lut[256];
    int sigma = ejo_alphabet(chars + (n ? offsets[0] : 0), total, lut);
    if (sigma > 255) return -2;
    uint32_t L = ejo_effective_L(offsets, n, L_req);
    res->sigma = (uint32_t)sigma;
    res->L = L;
    uint32_t T = r * z;

    /* symbol codes of every string */
    uint8_t *codes = (uint8_t *)malloc(total ? total : 1);
    for (uint64_t i = 0; i < total; i++) codes[i] = (uint8_t)lut[chars[offsets[0] + i]];

    /* randomness */
    uint64_t rb = (uint64_t)L * (uint64_t)sigma;
    uint8_t *Rbits = (uint8_t *)malloc(r * rb + 1);
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * T * m);
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * T * m);
    ejo_draw(seed, r, z, m, L, (uint32_t)sigma, Rbits, pos, v);
    if (explicit_R) memcpy(Rbits, explicit_R, r * rb);
    if (explicit_pos) memcpy(pos, explicit_pos, sizeof(uint32_t) * T * m);
    if (explicit_v) memcpy(v, explicit_v, sizeof(uint64_t) * T * m);

    /* Algorithm 2: sort, then embed every string r times; keep only the
     * sampled symbols (Section 4) and the resulting bucket keys. */
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    for (uint32_t i = 0; i < n; i++) order[i] = i;
    g_chars = chars;
    g_offsets = offsets;
    qsort(order, n, sizeof(uint32_t), cmp_len_alpha);

    res->keys = (uint64_t *)malloc(sizeof(uint64_t) * T * (n ? n : 1));
    res->sig = (opts & EJO_NO_SIG) ? NULL : (uint8_t *)malloc((uint64_t)n * T * m + 1);
    uint8_t *t = (uint8_t *)malloc(L);
    uint8_t *u = (uint8_t *)malloc(m);
    for (uint32_t l = 0; l < r; l++) {
        for (uint32_t oi = 0; oi < n; oi++) {
            uint32_t i = order[oi];
            uint32_t len = (uint32_t)(offsets[i + 1] - offsets[i]);
            ejo_cgk_embed(codes + (offsets[i] - offsets[0]), len, Rbits + l * rb,
                          (uint32_t)sigma, L, t);
            for (uint32_t j = 0; j < z; j++) {
                const uint32_t *pj = pos + ((uint64_t)l * z + j) * m;
                const uint64_t *vj = v + ((uint64_t)l * z + j) * m;
                for (uint32_t k = 0; k < m; k++) u[k] = t[pj[k]];
                if (res->sig) memcpy(res->sig + (((uint64_t)i * r + l) * z + j) * m, u, m);
                res->keys[((uint64_t)l * z + j) * n + i] = ejo_key(t, pj, vj, m);
            }
        }
    }
    free(t);
    free(u);

    /* Algorithm 3: one hash table per (l, j); strings in sorted order. */
    ejo_table *tables = (ejo_table *)malloc(sizeof(ejo_table) * T);
    uint64_t nslots = 16;
    while (nslots < 2ULL * n) nslots <<= 1;
    for (uint32_t q = 0; q < T; q++) table_init(&tables[q], nslots);
    uint64_t cap = 1024, cnt = 0;
    uint64_t *cand = (uint64_t *)malloc(sizeof(uint64_t) * cap);
    uint64_t icap = 64;
    uint64_t *iter_pairs = (uint64_t *)malloc(sizeof(uint64_t) * icap);
    for (uint32_t oi = 0; oi < n; oi++) {
        uint32_t si = order[oi];
        uint64_t len_i = offsets[si + 1] - offsets[si];
        uint64_t icnt = 0;
        for (uint32_t l = 0; l < r; l++) {
            for (uint32_t j = 0; j < z; j++) {
                uint32_t q = l * z + j;
                ejo_bucket *b = table_bucket(&tables[q], res->keys[(uint64_t)q * n + si]);
                uint32_t keep = 0;
                for (uint32_t e = 0; e < b->count; e++) {
                    uint32_t s = b->ids[e];
                    uint64_t len_s = offsets[s + 1] - offsets[s];
                    if (len_i - len_s <= K) {
                        uint32_t a = s < si ? s : si, c = s < si ? si : s;
                        if (icnt == icap) {
                            icap *= 2;
                            iter_pairs = (uint64_t *)realloc(iter_pairs, sizeof(uint64_t) * icap);
                        }
                        iter_pairs[icnt++] = ((uint64_t)a << 32) | c;
                        b->ids[keep++] = s;
                    }
                    /* else: evicted (not kept) */
                }
                b->count = keep;
                bucket_push(b, si);
            }
        }
        /* remove duplicate pairs found in this iteration; pairs from
         * different iterations differ in their later element */
        res->n_raw += icnt;
        qsort(iter_pairs, icnt, sizeof(uint64_t), cmp_u64);
        for (uint64_t e = 0; e < icnt; e++) {
            if (e > 0 && iter_pairs[e] == iter_pairs[e - 1]) continue;
            if (cnt == cap) {
                cap *= 2;
                cand = (uint64_t *)realloc(cand, sizeof(uint64_t) * cap);
            }
            cand[cnt++] = iter_pairs[e];
        }
    }
    free(iter_pairs);
    for (uint32_t q = 0; q < T; q++) table_free(&tables[q]);
    free(tables);
    qsort(cand, cnt, sizeof(uint64_t), cmp_u64);

    res->n_cand = cnt;
    res->cand = cand;
    if (opts & EJO_STOP_AFTER_CANDIDATES) {
        free(order);
        free(codes);
        free(Rbits);
        free(pos);
        free(v);
        return 0;
    }

    /* verification */
    res->cand_dist = (uint32_t *)malloc(sizeof(uint32_t) * (cnt ? cnt : 1));
    res->out = (uint64_t *)malloc(sizeof(uint64_t) * (cnt ? cnt : 1));
    res->out_dist = (uint32_t *)malloc(sizeof(uint32_t) * (cnt ? cnt : 1));
    uint64_t nout = 0;
    for (uint64_t e = 0; e < cnt; e++) {
        uint32_t a = (uint32_t)(cand[e] >> 32), c = (uint32_t)(cand[e] & 0xFFFFFFFFu);
        uint32_t d = ejo_ed_banded(chars + offsets[a], (uint32_t)(offsets[a + 1] - offsets[a]),
                                   chars + offsets[c], (uint32_t)(offsets[c + 1] - offsets[c]), K);
        res->cand_dist[e] = d;
        if (d <= K) {
            res->out[nout] = cand[e];
            res->out_dist[nout] = d;
            nout++;
        }
    }
    res->n_out = nout;
    free(order);
    free(codes);
    free(Rbits);
    free(pos);
    free(v);
    return 0;
}

int ejo_join(const uint8_t *chars, const uint64_t *offsets, uint32_t n, uint32_t K,
             uint32_t r, uint32_t z, uint32_t m, uint32_t L_req, uint64_t seed,
             const uint8_t *explicit_R, const uint32_t *explicit_pos,
             const uint64_t *explicit_v, ejo_result *res) {
    return ejo_join_opts(chars, offsets, n, K, r, z, m, L_req, seed, explicit_R, explicit_pos,
                         explicit_v, 0u, res);
}

/* ---------------------------------------------- Algorithms 4-5 (plus) -- */

/* Number of suffixes per string, ceil(K / delta), at least 1. */
uint32_t ejo_plus_kappa(uint32_t K, uint32_t delta) {
    uint32_t k = delta ? (K + delta - 1) / delta : 1;
    return k ? k : 1;
}

/* The threshold T of Section 5 when the caller leaves it open: 2 when each
 * string has more than one suffix, else 1. */
uint32_t ejo_plus_default_T(uint32_t K, uint32_t delta) {
    return ejo_plus_kappa(K, delta) > 1 ? 2u : 1u;
}

typedef struct {
    uint32_t x, y, kx, ky; /* x stored earlier in the sorted order, y the probing string */
} ejo_tuple;

static int cmp_tuple(const void *pa, const void *pb) {
    const ejo_tuple *a = (const ejo_tuple *)pa, *b = (const ejo_tuple *)pb;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    if (a->kx != b->kx) return a->kx < b->kx ? -1 : 1;
    if (a->ky != b->ky) return a->ky < b->ky ? -1 : 1;
    return 0;
}

/* EmbedJoin+ (Algorithm 5 with Algorithm 4 as preprocessing).  Every string
 * s_i contributes kappa = ceil(K/delta) suffixes s_{i,k} = s_i[(k-1)delta ..]
 * (0-based here; a suffix past the end is empty), each embedded with the
 * seed's random string and truncated to L; a table bucket stores (string,
 * suffix index) tuples.  Strings are visited in the sorted order; for each
 * seed l, function j and suffix k, the bucket of s_{i,k} is probed: every
 * stored tuple (s, k') of another string with |s_i| - |s| <= K adds the
 * tuple (s, s_i, k', k) to the collection C (a multiset), the others are
 * evicted; then (s_i, k) is stored.  A pair is a candidate when one of its
 * tuples occurs at least T times in C; candidates are verified exactly.
 * The result has the same layout as ejo_join's; keys are [r*z][n*kappa]
 * (suffix (i, k) at column i*kappa + k) and sig is not kept.  Returns 0, -1
 * for invalid sizes, -2 for a 256-symbol alphabet. */
int ejo_join_plus(const uint8_t *chars, const uint64_t *offsets, uint32_t n, uint32_t K,
                  uint32_t r, uint32_t z, uint32_t m, uint32_t L_req, uint64_t seed,
                  uint32_t delta, uint32_t T, uint32_t opts, ejo_result *res) {
    memset(res, 0, sizeof(*res));
    if (r == 0 || z == 0 || m == 0 || delta == 0 || T == 0) return -1;
    const uint32_t kappa = ejo_plus_kappa(K, delta);
    if ((uint64_t)n * kappa >= 0xFFFFFFFFull) return -1;
    uint64_t total = n ? offsets[n] - offsets[0] : 0;
    int32_t lut[256];
    int sigma = ejo_alphabet(chars + (n ? offsets[0] : 0), total, lut);
    if (sigma > 255) return -2;
    uint32_t L = ejo_effective_L(offsets, n, L_req);
    res->sigma = (uint32_t)sigma;
    res->L = L;
    const uint32_t Tn = r * z;
    const uint64_t ns = (uint64_t)n * kappa;

    uint8_t *codes = (uint8_t *)malloc(total ? total : 1);
    for (uint64_t i = 0; i < total; i++) codes[i] = (uint8_t)lut[chars[offsets[0] + i]];
    uint64_t rb = (uint64_t)L * (uint64_t)sigma;
    uint8_t *Rbits = (uint8_t *)malloc(r * rb + 1);
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * Tn * m);
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * Tn * m);
    ejo_draw(seed, r, z, m, L, (uint32_t)sigma, Rbits, pos, v);

    /* Algorithm 4: sort, then embed every suffix of every string r times */
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    for (uint32_t i = 0; i < n; i++) order[i] = i;
    g_chars = chars;
    g_offsets = offsets;
    qsort(order, n, sizeof(uint32_t), cmp_len_alpha);
    res->keys = (uint64_t *)malloc(sizeof(uint64_t) * Tn * (ns ? ns : 1));
    uint8_t *t = (uint8_t *)malloc(L);
    for (uint32_t l = 0; l < r; l++) {
        for (uint32_t i = 0; i < n; i++) {
            const uint32_t len = (uint32_t)(offsets[i + 1] - offsets[i]);
            for (uint32_t k = 0; k < kappa; k++) {
                const uint64_t start = (uint64_t)k * delta;
                const uint32_t skip = start < len ? (uint32_t)start : len;
                ejo_cgk_embed(codes + (offsets[i] - offsets[0]) + skip, len - skip,
                              Rbits + l * rb, (uint32_t)sigma, L, t);
                for (uint32_t j = 0; j < z; j++)
                    res->keys[((uint64_t)l * z + j) * ns + (uint64_t)i * kappa + k] =
                        ejo_key(t, pos + ((uint64_t)l * z + j) * m, v + ((uint64_t)l * z + j) * m,
                                m);
            }
        }
    }
    free(t);

    /* Algorithm 5: tables of (string, suffix) tuples, strings in sorted order */
    ejo_table *tables = (ejo_table *)malloc(sizeof(ejo_table) * Tn);
    uint64_t nslots = 16;
    while (nslots < 2ULL * ns) nslots <<= 1;
    for (uint32_t q = 0; q < Tn; q++) table_init(&tables[q], nslots);
    uint64_t ccap = 1024, ccnt = 0;
    ejo_tuple *C = (ejo_tuple *)malloc(sizeof(ejo_tuple) * ccap);
    for (uint32_t oi = 0; oi < n; oi++) {
        const uint32_t si = order[oi];
        const uint64_t len_i = offsets[si + 1] - offsets[si];
        for (uint32_t l = 0; l < r; l++) {
            for (uint32_t j = 0; j < z; j++) {
                const uint32_t q = l * z + j;
                for (uint32_t k = 0; k < kappa; k++) {
                    const uint64_t key = res->keys[(uint64_t)q * ns + (uint64_t)si * kappa + k];
                    ejo_bucket *b = table_bucket(&tables[q], key);
                    uint32_t keep = 0;
                    for (uint32_t e = 0; e < b->count; e++) {
                        const uint32_t tup = b->ids[e];
                        const uint32_t s = tup / kappa, kk = tup % kappa;
                        if (s == si) { /* the string's own earlier suffix: skipped */
                            b->ids[keep++] = tup;
                            continue;
                        }
                        const uint64_t len_s = offsets[s + 1] - offsets[s];
                        if (len_i - len_s <= K) {
                            if (ccnt == ccap) {
                                ccap *= 2;
                                C = (ejo_tuple *)realloc(C, sizeof(ejo_tuple) * ccap);
                            }
                            C[ccnt].x = s;
                            C[ccnt].y = si;
                            C[ccnt].kx = kk;
                            C[ccnt].ky = k;
                            ccnt++;
                            b->ids[keep++] = tup;
                        }
                        /* else: evicted */
                    }
                    b->count = keep;
                    bucket_push(b, si * kappa + k);
                }
            }
        }
    }
    for (uint32_t q = 0; q < Tn; q++) table_free(&tables[q]);
    free(tables);
    res->n_raw = ccnt;

    /* count each tuple; a pair with some tuple counted >= T is a candidate */
    qsort(C, ccnt, sizeof(ejo_tuple), cmp_tuple);
    uint64_t cap = 1024, cnt = 0;
    uint64_t *cand = (uint64_t *)malloc(sizeof(uint64_t) * cap);
    for (uint64_t e = 0; e < ccnt;) {
        uint64_t f = e;
        while (f < ccnt && cmp_tuple(&C[f], &C[e]) == 0) f++;
        if (f - e >= T) {
            const uint32_t a = C[e].x < C[e].y ? C[e].x : C[e].y;
            const uint32_t c = C[e].x < C[e].y ? C[e].y : C[e].x;
            if (cnt == cap) {
                cap *= 2;
                cand = (uint64_t *)realloc(cand, sizeof(uint64_t) * cap);
            }
            cand[cnt++] = ((uint64_t)a << 32) | c;
        }
        e = f;
    }
    free(C);
    qsort(cand, cnt, sizeof(uint64_t), cmp_u64);
    uint64_t u = 0;
    for (uint64_t e = 0; e < cnt; e++)
        if (e == 0 || cand[e] != cand[e - 1]) cand[u++] = cand[e];
    cnt = u;
    res->n_cand = cnt;
    res->cand = cand;
    if (!(opts & EJO_STOP_AFTER_CANDIDATES)) {
        res->cand_dist = (uint32_t *)malloc(sizeof(uint32_t) * (cnt ? cnt : 1));
        res->out = (uint64_t *)malloc(sizeof(uint64_t) * (cnt ? cnt : 1));
        res->out_dist = (uint32_t *)malloc(sizeof(uint32_t) * (cnt ? cnt : 1));
        uint64_t nout = 0;
        for (uint64_t e = 0; e < cnt; e++) {
            const uint32_t a = (uint32_t)(cand[e] >> 32), c = (uint32_t)cand[e];
            const uint32_t d =
                ejo_ed_banded(chars + offsets[a], (uint32_t)(offsets[a + 1] - offsets[a]),
                              chars + offsets[c], (uint32_t)(offsets[c + 1] - offsets[c]), K);
            res->cand_dist[e] = d;
            if (d <= K) {
                res->out[nout] = cand[e];
                res->out_dist[nout] = d;
                nout++;
            }
        }
        res->n_out = nout;
    }
    free(order);
    free(codes);
    free(Rbits);
    free(pos);
    free(v);
    return 0;
}

/* ------------------------------------------- grouping (Section 4.1) -- */

/* Group g (0-based) of the grouping alternative to truncation holds the
 * strings of length in ((g)K, (g+2)K], for g = 0 .. G-1 with
 * G = max(1, ceil(N/K) - 1); group 0 also holds the empty strings (they pair
 * with every string of length <= K).  With K = 0 there is one group per
 * length.  Every string is in at most two groups and every pair within K in
 * length shares one. */
static int in_group(uint64_t len, uint64_t g, uint32_t K) {
    if (K == 0) return len == g;
    if (g == 0 && len == 0) return 1;
    return len > g * K && len <= (g + 2) * K;
}

static uint64_t group_count(uint64_t N, uint32_t K) {
    if (K == 0) return N + 1;
    uint64_t c = (N + K - 1) / K;
    return c > 1 ? c - 1 : 1;
}

/* EmbedJoin with grouping instead of truncation: EmbedJoin (ejo_join) on each
 * group on its own -- its own alphabet, the same seed, L = 3 N_g (N_g = the
 * group's longest string; the walks are not truncated) unless L_req > 0 asks
 * for a truncation -- and the union of the groups' candidates and outputs.
 * n_raw sums the groups' raw counts.  Keys and signatures are not kept.
 * Returns 0, or the first failing group's code. */
int ejo_join_grouped(const uint8_t *chars, const uint64_t *offsets, uint32_t n, uint32_t K,
                     uint32_t r, uint32_t z, uint32_t m, uint32_t L_req, uint64_t seed,
                     ejo_result *res) {
    memset(res, 0, sizeof(*res));
    if (r == 0 || z == 0 || m == 0) return -1;
    uint64_t N = 0;
    for (uint32_t i = 0; i < n; i++)
        if (offsets[i + 1] - offsets[i] > N) N = offsets[i + 1] - offsets[i];
    const uint64_t G = group_count(N, K);
    uint64_t ccap = 1024, cc = 0, ocap = 1024, oc = 0;
    uint64_t *cand = (uint64_t *)malloc(sizeof(uint64_t) * ccap);
    uint64_t *outp = (uint64_t *)malloc(sizeof(uint64_t) * ocap);
    uint32_t *outd = (uint32_t *)malloc(sizeof(uint32_t) * ocap);
    uint32_t *ids = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t *soff = (uint64_t *)malloc(sizeof(uint64_t) * (n + 1));
    uint8_t *sub = (uint8_t *)malloc((n ? offsets[n] - offsets[0] : 0) + 1);
    int rc = 0;
    for (uint64_t g = 0; g < G && rc == 0; g++) {
        uint32_t k = 0;
        uint64_t Ng = 0, t = 0;
        soff[0] = 0;
        for (uint32_t i = 0; i < n; i++) {
            const uint64_t len = offsets[i + 1] - offsets[i];
            if (!in_group(len, g, K)) continue;
            memcpy(sub + t, chars + offsets[i], len);
            t += len;
            ids[k++] = i;
            soff[k] = t;
            if (len > Ng) Ng = len;
        }
        if (k < 2) continue;
        uint64_t Lg = L_req ? L_req : 3 * Ng;
        if (Lg == 0) Lg = 1;
        ejo_result gr;
        rc = ejo_join_opts(sub, soff, k, K, r, z, m, (uint32_t)Lg, seed, NULL, NULL, NULL,
                           EJO_NO_SIG, &gr);
        if (rc != 0) break;
        res->n_raw += gr.n_raw;
        for (uint64_t e = 0; e < gr.n_cand; e++) {
            if (cc == ccap) cand = (uint64_t *)realloc(cand, sizeof(uint64_t) * (ccap *= 2));
            cand[cc++] = ((uint64_t)ids[gr.cand[e] >> 32] << 32) | ids[gr.cand[e] & 0xFFFFFFFFu];
        }
        for (uint64_t e = 0; e < gr.n_out; e++) {
            if (oc == ocap) {
                ocap *= 2;
                outp = (uint64_t *)realloc(outp, sizeof(uint64_t) * ocap);
                outd = (uint32_t *)realloc(outd, sizeof(uint32_t) * ocap);
            }
            outp[oc] = ((uint64_t)ids[gr.out[e] >> 32] << 32) | ids[gr.out[e] & 0xFFFFFFFFu];
            outd[oc++] = gr.out_dist[e];
        }
        ejo_result_free(&gr);
    }
    free(ids);
    free(soff);
    free(sub);
    /* union: sort and keep one of each (a pair found by two groups has one
     * distance) */
    qsort(cand, cc, sizeof(uint64_t), cmp_u64);
    uint64_t u = 0;
    for (uint64_t e = 0; e < cc; e++)
        if (e == 0 || cand[e] != cand[e - 1]) cand[u++] = cand[e];
    res->n_cand = u;
    res->cand = cand;
    /* sort the outputs with their distances; keep one of each pair (a pair
     * found by two groups has one distance) */
    ejo_tuple *od = (ejo_tuple *)malloc(sizeof(ejo_tuple) * (oc ? oc : 1));
    for (uint64_t e = 0; e < oc; e++) {
        od[e].x = (uint32_t)(outp[e] >> 32);
        od[e].y = (uint32_t)outp[e];
        od[e].kx = outd[e];
        od[e].ky = 0;
    }
    qsort(od, oc, sizeof(ejo_tuple), cmp_tuple);
    res->out = (uint64_t *)malloc(sizeof(uint64_t) * (oc ? oc : 1));
    res->out_dist = (uint32_t *)malloc(sizeof(uint32_t) * (oc ? oc : 1));
    uint64_t no = 0;
    for (uint64_t e = 0; e < oc; e++) {
        const uint64_t code = ((uint64_t)od[e].x << 32) | od[e].y;
        if (no && res->out[no - 1] == code) continue;
        res->out[no] = code;
        res->out_dist[no] = od[e].kx;
        no++;
    }
    res->n_out = no;
    free(od);
    free(outp);
    free(outd);
    return rc;
}

/* --------------------------------------------- exhaustive short strings -- */

/* Short strings.  The paper observes that LSH filtering suits long strings and
 * that short ones may call for another filter; with a threshold K that is large
 * next to a string's length, random strings of such lengths are within K of
 * each other by chance and no embedding brings them together.  This pass adds,
 * for S > 0, every pair (i, j), i < j, whose strings are both no longer than S
 * and whose lengths differ by at most K (the length filter: ED >= the length
 * difference) to the candidates of `res` -- a result of the EmbedJoin,
 * EmbedJoin+ or grouping join over the same strings -- verifies the union
 * (Section 3.3, Ukkonen's band) and replaces res's candidates, their distances
 * and its output.  n_raw keeps the tables' count.  S = 0 leaves res as it is.
 * Returns 0, or -1 when an allocation fails. */
int ejo_exact_short(const uint8_t *chars, const uint64_t *offsets, uint32_t n, uint32_t K,
                    uint32_t S, ejo_result *res) {
    if (S == 0) return 0;
    uint32_t *sid = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!sid) return -1;
    uint32_t ns = 0;
    for (uint32_t i = 0; i < n; i++)
        if (offsets[i + 1] - offsets[i] <= S) sid[ns++] = i;
    uint64_t extra = 0;
    for (uint32_t a = 0; a < ns; a++)
        for (uint32_t b = a + 1; b < ns; b++) {
            const uint64_t la = offsets[sid[a] + 1] - offsets[sid[a]];
            const uint64_t lb = offsets[sid[b] + 1] - offsets[sid[b]];
            if ((la > lb ? la - lb : lb - la) <= K) extra++;
        }
    const uint64_t tot = res->n_cand + extra;
    uint64_t *u = (uint64_t *)malloc(sizeof(uint64_t) * (tot ? tot : 1));
    if (!u) {
        free(sid);
        return -1;
    }
    uint64_t t = 0;
    for (uint64_t e = 0; e < res->n_cand; e++) u[t++] = res->cand[e];
    for (uint32_t a = 0; a < ns; a++)
        for (uint32_t b = a + 1; b < ns; b++) {
            const uint64_t la = offsets[sid[a] + 1] - offsets[sid[a]];
            const uint64_t lb = offsets[sid[b] + 1] - offsets[sid[b]];
            if ((la > lb ? la - lb : lb - la) <= K) u[t++] = ((uint64_t)sid[a] << 32) | sid[b];
        }
    free(sid);
    qsort(u, tot, sizeof(uint64_t), cmp_u64);
    uint64_t nu = 0;
    for (uint64_t e = 0; e < tot; e++)
        if (e == 0 || u[e] != u[e - 1]) u[nu++] = u[e];
    uint32_t *cd = (uint32_t *)malloc(sizeof(uint32_t) * (nu ? nu : 1));
    uint64_t *op = (uint64_t *)malloc(sizeof(uint64_t) * (nu ? nu : 1));
    uint32_t *od = (uint32_t *)malloc(sizeof(uint32_t) * (nu ? nu : 1));
    if (!cd || !op || !od) {
        free(u);
        free(cd);
        free(op);
        free(od);
        return -1;
    }
    uint64_t no = 0;
    for (uint64_t e = 0; e < nu; e++) {
        const uint32_t a = (uint32_t)(u[e] >> 32), b = (uint32_t)u[e];
        cd[e] = ejo_ed_banded(chars + offsets[a], (uint32_t)(offsets[a + 1] - offsets[a]),
                              chars + offsets[b], (uint32_t)(offsets[b + 1] - offsets[b]), K);
        if (cd[e] <= K) {
            op[no] = u[e];
            od[no++] = cd[e];
        }
    }
    free(res->cand);
    free(res->cand_dist);
    free(res->out);
    free(res->out_dist);
    res->cand = u;
    res->n_cand = nu;
    res->cand_dist = cd;
    res->out = op;
    res->out_dist = od;
    res->n_out = no;
    return 0;
}

/* ------------------------------------------- distortion diagnostics ---- */

/* Section 3.1 (distortion of the CGK embedding) and Section 6 (normalised
 * Hamming distance under truncation): for each pair (a, b) and seed l < r,
 * the Hamming distance between the first L symbols of the two strings'
 * embeddings under R^l.  With delta > 0 every string contributes
 * kappa = ceil(K / delta) suffixes (as in EmbedJoin+) and the distance is the
 * minimum over the kappa^2 suffix pairs.  ham[pair * r + l].  The alphabet and
 * L (0 = ceil(average length), at most 3N) come from the whole set.  Returns
 * 0, -1 for invalid sizes, -2 for a 256-symbol alphabet. */
int ejo_embed_hamming(const uint8_t *chars, const uint64_t *offsets, uint32_t n, uint32_t r,
                      uint32_t L_req, uint64_t seed, uint32_t K, uint32_t delta,
                      const uint64_t *pairs, uint64_t count, uint32_t *ham) {
    if (r == 0) return -1;
    uint64_t total = n ? offsets[n] - offsets[0] : 0;
    int32_t lut[256];
    int sigma = ejo_alphabet(chars + (n ? offsets[0] : 0), total, lut);
    if (sigma > 255) return -2;
    const uint32_t L = ejo_effective_L(offsets, n, L_req);
    const uint32_t kappa = delta ? ejo_plus_kappa(K, delta) : 1;
    uint8_t *codes = (uint8_t *)malloc(total ? total : 1);
    for (uint64_t i = 0; i < total; i++) codes[i] = (uint8_t)lut[chars[offsets[0] + i]];
    const uint64_t rb = (uint64_t)L * (uint64_t)sigma;
    uint8_t *Rbits = (uint8_t *)malloc(r * rb + 1);
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * r);
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * r);
    ejo_draw(seed, r, 1, 1, L, (uint32_t)sigma, Rbits, pos, v);
    uint8_t *ta = (uint8_t *)malloc(L), *tb = (uint8_t *)malloc(L);
    for (uint64_t e = 0; e < count; e++) {
        const uint32_t a = (uint32_t)(pairs[e] >> 32), b = (uint32_t)pairs[e];
        const uint32_t la = (uint32_t)(offsets[a + 1] - offsets[a]);
        const uint32_t lb = (uint32_t)(offsets[b + 1] - offsets[b]);
        for (uint32_t l = 0; l < r; l++) {
            uint32_t best = 0xFFFFFFFFu;
            for (uint32_t ka = 0; ka < kappa; ka++) {
                const uint64_t sa64 = (uint64_t)ka * delta;
                const uint32_t sa = sa64 < la ? (uint32_t)sa64 : la;
                ejo_cgk_embed(codes + (offsets[a] - offsets[0]) + sa, la - sa, Rbits + l * rb,
                              (uint32_t)sigma, L, ta);
                for (uint32_t kb = 0; kb < kappa; kb++) {
                    const uint64_t sb64 = (uint64_t)kb * delta;
                    const uint32_t sb = sb64 < lb ? (uint32_t)sb64 : lb;
                    ejo_cgk_embed(codes + (offsets[b] - offsets[0]) + sb, lb - sb,
                                  Rbits + l * rb, (uint32_t)sigma, L, tb);
                    uint32_t h = 0;
                    for (uint32_t j = 0; j < L; j++) h += ta[j] != tb[j];
                    if (h < best) best = h;
                }
            }
            ham[e * r + l] = best;
        }
    }
    free(codes);
    free(Rbits);
    free(pos);
    free(v);
    free(ta);
    free(tb);
    return 0;
}

/* ------------------------------------------------------------- serving --
 * Serving is a systems layer on the method, not a step of the paper: an
 * index fixes the alphabet (its sorted distinct bytes), the truncation L and
 * the random streams; query q's result is every index string s that shares
 * the key of some table (l, j) with q, whose length differs from |q| by at
 * most K_q and whose edit distance to q is at most K_q, in increasing
 * position order.  Written as a plain double loop over (query, index
 * string), with the keys from the same embedding and key functions as the
 * join.  Returns the number of results (entries beyond cap are not
 * written), -1 for invalid sizes, -2 if a query byte is outside the index
 * alphabet, -3 when all 256 byte values occur in the index. */
static void string_keys(const uint8_t *codes, uint32_t len, const uint8_t *Rbits, uint64_t rb,
                        uint32_t sigma, uint32_t L, const uint32_t *pos, const uint64_t *v,
                        uint32_t r, uint32_t z, uint32_t m, uint8_t *t, uint64_t *keys) {
    for (uint32_t l = 0; l < r; l++) {
        ejo_cgk_embed(codes, len, Rbits + l * rb, sigma, L, t);
        for (uint32_t j = 0; j < z; j++)
            keys[l * z + j] = ejo_key(t, pos + ((uint64_t)l * z + j) * m,
                                      v + ((uint64_t)l * z + j) * m, m);
    }
}

int64_t ejo_query(const uint8_t *ichars, const uint64_t *ioff, uint32_t n, const uint8_t *qchars,
                  const uint64_t *qoff, uint32_t nq, const uint32_t *Kq, uint32_t r, uint32_t z,
                  uint32_t m, uint32_t L_req, uint64_t seed, uint64_t *res_off,
                  uint32_t *res_ids, uint32_t *res_dist, uint64_t cap) {
    if (r == 0 || z == 0 || m == 0) return -1;
    uint64_t itotal = n ? ioff[n] - ioff[0] : 0;
    int32_t lut[256];
    int sigma = ejo_alphabet(ichars + (n ? ioff[0] : 0), itotal, lut);
    if (sigma > 255) return -3;
    uint32_t L = ejo_effective_L(ioff, n, L_req);
    uint32_t T = r * z;
    uint64_t qtotal = nq ? qoff[nq] - qoff[0] : 0;
    for (uint64_t i = 0; i < qtotal; i++)
        if (lut[qchars[qoff[0] + i]] < 0) return -2;
    uint8_t *icodes = (uint8_t *)malloc(itotal + 1);
    uint8_t *qcodes = (uint8_t *)malloc(qtotal + 1);
    for (uint64_t i = 0; i < itotal; i++) icodes[i] = (uint8_t)lut[ichars[ioff[0] + i]];
    for (uint64_t i = 0; i < qtotal; i++) qcodes[i] = (uint8_t)lut[qchars[qoff[0] + i]];
    uint64_t rb = (uint64_t)L * (uint64_t)sigma;
    uint8_t *Rbits = (uint8_t *)malloc(r * rb + 1);
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * T * m);
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * T * m);
    ejo_draw(seed, r, z, m, L, (uint32_t)sigma, Rbits, pos, v);
    uint8_t *t = (uint8_t *)malloc(L);
    uint64_t *ikeys = (uint64_t *)malloc(sizeof(uint64_t) * T * (n ? n : 1));
    uint64_t *qk = (uint64_t *)malloc(sizeof(uint64_t) * T);
    for (uint32_t s = 0; s < n; s++)
        string_keys(icodes + (ioff[s] - ioff[0]), (uint32_t)(ioff[s + 1] - ioff[s]), Rbits, rb,
                    (uint32_t)sigma, L, pos, v, r, z, m, t, ikeys + (uint64_t)s * T);
    uint64_t cnt = 0;
    res_off[0] = 0;
    for (uint32_t q = 0; q < nq; q++) {
        const uint8_t *xq = qcodes + (qoff[q] - qoff[0]);
        uint32_t lq = (uint32_t)(qoff[q + 1] - qoff[q]);
        string_keys(xq, lq, Rbits, rb, (uint32_t)sigma, L, pos, v, r, z, m, t, qk);
        for (uint32_t s = 0; s < n; s++) {
            uint32_t ls = (uint32_t)(ioff[s + 1] - ioff[s]);
            uint32_t gap = ls > lq ? ls - lq : lq - ls;
            if (gap > Kq[q]) continue;
            int hit = 0;
            for (uint32_t e = 0; e < T && !hit; e++) hit = ikeys[(uint64_t)s * T + e] == qk[e];
            if (!hit) continue;
            uint32_t d = ejo_ed_banded(icodes + (ioff[s] - ioff[0]), ls, xq, lq, Kq[q]);
            if (d > Kq[q]) continue;
            if (cnt < cap) {
                res_ids[cnt] = s;
                res_dist[cnt] = d;
            }
            cnt++;
        }
        res_off[q + 1] = cnt;
    }
    free(icodes);
    free(qcodes);
    free(Rbits);
    free(pos);
    free(v);
    free(t);
    free(ikeys);
    free(qk);
    return (int64_t)cnt;
}

/* Bucket keys of every string of a set x under the alphabet, truncation and
 * random streams that the set s (ichars/ioff, n strings) fixes -- the keys the
 * serving definition compares (x = s gives the join's keys).  keys[i][q] for
 * table q = l*z + j.  Returns 0, -1 for invalid sizes, -2 if a byte of x is
 * outside the alphabet of s, -3 when all 256 byte values occur in s. */
int ejo_keys(const uint8_t *ichars, const uint64_t *ioff, uint32_t n, const uint8_t *xchars,
             const uint64_t *xoff, uint32_t nx, uint32_t r, uint32_t z, uint32_t m,
             uint32_t L_req, uint64_t seed, uint64_t *keys) {
    if (r == 0 || z == 0 || m == 0) return -1;
    uint64_t itotal = n ? ioff[n] - ioff[0] : 0;
    int32_t lut[256];
    int sigma = ejo_alphabet(ichars + (n ? ioff[0] : 0), itotal, lut);
    if (sigma > 255) return -3;
    uint32_t L = ejo_effective_L(ioff, n, L_req);
    uint32_t T = r * z;
    uint64_t xtotal = nx ? xoff[nx] - xoff[0] : 0;
    for (uint64_t i = 0; i < xtotal; i++)
        if (lut[xchars[xoff[0] + i]] < 0) return -2;
    uint8_t *xcodes = (uint8_t *)malloc(xtotal + 1);
    for (uint64_t i = 0; i < xtotal; i++) xcodes[i] = (uint8_t)lut[xchars[xoff[0] + i]];
    uint64_t rb = (uint64_t)L * (uint64_t)sigma;
    uint8_t *Rbits = (uint8_t *)malloc(r * rb + 1);
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * T * m);
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * T * m);
    ejo_draw(seed, r, z, m, L, (uint32_t)sigma, Rbits, pos, v);
    uint8_t *t = (uint8_t *)malloc(L);
    for (uint32_t i = 0; i < nx; i++)
        string_keys(xcodes + (xoff[i] - xoff[0]), (uint32_t)(xoff[i + 1] - xoff[i]), Rbits, rb,
                    (uint32_t)sigma, L, pos, v, r, z, m, t, keys + (uint64_t)i * T);
    free(xcodes);
    free(Rbits);
    free(pos);
    free(v);
    free(t);
    return 0;
}

/* Verification only: min(ED, K+1) for each pair (a_k, b_k). */
void ejo_verify_pairs(const uint8_t *chars, const uint64_t *offsets, const uint64_t *pairs,
                      uint64_t count, uint32_t K, uint32_t *dist) {
    for (uint64_t e = 0; e < count; e++) {
        uint32_t a = (uint32_t)(pairs[e] >> 32), c = (uint32_t)(pairs[e] & 0xFFFFFFFFu);
        dist[e] = ejo_ed_banded(chars + offsets[a], (uint32_t)(offsets[a + 1] - offsets[a]),
                                chars + offsets[c], (uint32_t)(offsets[c + 1] - offsets[c]), K);
    }
}

/* Exact join by brute force: every pair; full Wagner-Fischer when `full` is
 * set, else Ukkonen's threshold DP (same answer for ED <= K).  Writes at most
 * `cap` pairs, returns the total count. */
uint64_t ejo_brute_join(const uint8_t *chars, const uint64_t *offsets, uint32_t n, uint32_t K,
                        uint64_t *out, uint32_t *dist, uint64_t cap, int full) {
    uint64_t cnt = 0;
    for (uint32_t a = 0; a < n; a++) {
        for (uint32_t c = a + 1; c < n; c++) {
            const uint8_t *xa = chars + offsets[a], *xc = chars + offsets[c];
            uint32_t la = (uint32_t)(offsets[a + 1] - offsets[a]);
            uint32_t lc = (uint32_t)(offsets[c + 1] - offsets[c]);
            uint32_t d = full ? ejo_ed_full(xa, la, xc, lc) : ejo_ed_banded(xa, la, xc, lc, K);
            if (d <= K) {
                if (cnt < cap) {
                    out[cnt] = ((uint64_t)a << 32) | c;
                    dist[cnt] = d;
                }
                cnt++;
            }
        }
    }
    return cnt;
}
