/*
 * Drives every entry point of the CPU oracle on small random inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (see
 * test_oracle_sanitizers.py).  Includes the oracle's source so that the whole
 * oracle is one translation unit under the sanitizers.  Exits non-zero if an
 * invariant fails; the sanitizers abort on any memory or undefined-behaviour
 * error.
 */
#include <stdio.h>

#include "../oracle/ej_oracle.c"

static uint64_t lcg_state = 88172645463325252ULL;
static uint32_t rnd(uint32_t bound) {
    lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return bound ? (uint32_t)((lcg_state >> 33) % bound) : 0;
}

/* n strings over `sigma` letters starting at 'A', lengths in [0, maxlen],
 * half of them mutated copies of an earlier string. */
static void make_set(uint32_t n, uint32_t maxlen, uint32_t sigma, uint8_t **chars,
                     uint64_t *offsets) {
    uint8_t *c = (uint8_t *)malloc((uint64_t)n * (maxlen + 4) + 1);
    uint64_t t = 0;
    offsets[0] = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (i > 0 && rnd(2)) {
            uint32_t src = rnd(i);
            uint64_t a = offsets[src], b = offsets[src + 1];
            for (uint64_t k = a; k < b; k++) {
                uint32_t op = rnd(20);
                if (op == 0) continue;                          /* deletion */
                if (op == 1) c[t++] = (uint8_t)('A' + rnd(sigma)); /* insertion */
                c[t++] = op == 2 ? (uint8_t)('A' + rnd(sigma)) : c[k];
            }
        } else {
            uint32_t len = rnd(maxlen + 1);
            for (uint32_t k = 0; k < len; k++) c[t++] = (uint8_t)('A' + rnd(sigma));
        }
        offsets[i + 1] = t;
    }
    *chars = c;
}

static int check_join(uint32_t n, uint32_t maxlen, uint32_t sigma, uint32_t K, uint32_t r,
                      uint32_t z, uint32_t m, uint32_t L, uint64_t seed) {
    uint8_t *chars = NULL;
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * (n + 1));
    make_set(n, maxlen, sigma, &chars, off);
    ejo_result res;
    if (ejo_join(chars, off, n, K, r, z, m, L, seed, NULL, NULL, NULL, &res) != 0) return 1;
    uint64_t cap = (uint64_t)n * n + 1;
    uint64_t *bp = (uint64_t *)malloc(sizeof(uint64_t) * cap);
    uint32_t *bd = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    uint64_t nb = ejo_brute_join(chars, off, n, K, bp, bd, cap, 1);
    uint64_t nb2 = ejo_brute_join(chars, off, n, K, bp, bd, cap, 0);
    int bad = nb != nb2;
    /* every output pair is a true pair (both lists are sorted) */
    uint64_t j = 0;
    for (uint64_t i = 0; i < res.n_out && !bad; i++) {
        while (j < nb && bp[j] < res.out[i]) j++;
        if (j == nb || bp[j] != res.out[i] || bd[j] != res.out_dist[i]) bad = 1;
    }
    /* candidates-only mode: the same set */
    ejo_result c2;
    if (ejo_join_opts(chars, off, n, K, r, z, m, L, seed, NULL, NULL, NULL,
                      EJO_STOP_AFTER_CANDIDATES | EJO_NO_SIG, &c2) != 0)
        bad = 1;
    if (c2.n_cand != res.n_cand || c2.n_raw != res.n_raw) bad = 1;
    for (uint64_t i = 0; i < c2.n_cand && !bad; i++) bad = c2.cand[i] != res.cand[i];
    /* verification alone agrees with the join's distances */
    uint32_t *vd = (uint32_t *)malloc(sizeof(uint32_t) * (res.n_cand + 1));
    ejo_verify_pairs(chars, off, res.cand, res.n_cand, K, vd);
    for (uint64_t i = 0; i < res.n_cand && !bad; i++) bad = vd[i] != res.cand_dist[i];
    /* the query definition over the set itself */
    uint32_t *Kq = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    for (uint32_t i = 0; i < n; i++) Kq[i] = K;
    uint64_t *qoff = (uint64_t *)malloc(sizeof(uint64_t) * (n + 1));
    uint32_t *qid = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    uint32_t *qd = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    if (ejo_query(chars, off, n, chars, off, n, Kq, r, z, m, L, seed, qoff, qid, qd, cap) < 0)
        bad = 1;
    /* every string short: the exact join */
    ejo_result c3;
    if (ejo_join(chars, off, n, K, r, z, m, L, seed, NULL, NULL, NULL, &c3) != 0 ||
        ejo_exact_short(chars, off, n, K, 0xFFFFFFFFu, &c3) != 0 || c3.n_out != nb)
        bad = 1;
    ejo_brute_join(chars, off, n, K, bp, bd, cap, 0);
    for (uint64_t i = 0; i < c3.n_out && !bad; i++)
        bad = c3.out[i] != bp[i] || c3.out_dist[i] != bd[i];
    ejo_result_free(&c3);
    /* EmbedJoin+ and grouping, each with the short-string pass */
    ejo_result c4, c5;
    if (ejo_join_plus(chars, off, n, K, r, z, m, L, seed, 3, ejo_plus_default_T(K, 3), 0, &c4) != 0 ||
        ejo_exact_short(chars, off, n, K, 5, &c4) != 0)
        bad = 1;
    ejo_result_free(&c4);
    if (ejo_join_grouped(chars, off, n, K, r, z, m, L, seed, &c5) != 0 ||
        ejo_exact_short(chars, off, n, K, 7, &c5) != 0)
        bad = 1;
    ejo_result_free(&c5);
    /* embedding Hamming distances of the candidates, and keys of the set */
    uint32_t *ham = (uint32_t *)malloc(sizeof(uint32_t) * (res.n_cand * r + 1));
    if (ejo_embed_hamming(chars, off, n, r, L, seed, K, 4, res.cand, res.n_cand, ham) != 0)
        bad = 1;
    free(ham);
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * ((uint64_t)r * z * n + 1));
    if (ejo_keys(chars, off, n, chars, off, n, r, z, m, L, seed, keys) != 0) bad = 1;
    free(keys);
    free(vd);
    free(Kq);
    free(qoff);
    free(qid);
    free(qd);
    free(bp);
    free(bd);
    ejo_result_free(&res);
    ejo_result_free(&c2);
    free(chars);
    free(off);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= check_join(40, 30, 4, 5, 3, 4, 3, 0, 1);
    bad |= check_join(30, 60, 20, 12, 2, 5, 2, 50, 2);
    bad |= check_join(25, 8, 2, 0, 4, 3, 1, 0, 3);       /* K = 0, short strings */
    bad |= check_join(20, 0, 4, 3, 2, 2, 2, 0, 4);       /* all strings empty */
    bad |= check_join(1, 10, 4, 3, 2, 2, 2, 0, 5);       /* one string */
    bad |= check_join(35, 40, 4, 100, 3, 3, 4, 200, 6); /* K above every length */
    /* randomness draws of odd sizes, and the banded distance at extreme K */
    uint8_t *R = (uint8_t *)malloc(3 * 7 * 5);
    uint32_t *pos = (uint32_t *)malloc(sizeof(uint32_t) * 3 * 2 * 5);
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * 3 * 2 * 5);
    ejo_draw(9, 3, 2, 5, 7, 5, R, pos, v);
    for (int i = 0; i < 30; i++) bad |= pos[i] >= 7 || v[i] >= EJO_P;
    const uint8_t x[] = {0, 1, 2, 3, 0, 1}, y[] = {1, 2, 3, 0};
    bad |= ejo_ed_banded(x, 6, y, 4, 0) != 1;
    bad |= ejo_ed_banded(x, 6, y, 4, 1000) != ejo_ed_full(x, 6, y, 4);
    bad |= ejo_ed_banded(x, 0, y, 0, 0) != 0;
    free(R);
    free(pos);
    free(v);
    if (bad) printf("oracle invariant failed\n");
    else printf("oracle ok\n");
    return bad;
}
