/*
 * embedjoin.h -- C ABI of libembedjoin.so, an MI355X (gfx950) implementation
 * of the data-parallel hot path of EmbedJoin (H. Zhang, Q. Zhang, "EmbedJoin:
 * Efficient Edit Similarity Joins via Embeddings").
 *
 * Problem (Section 1): given strings s_1..s_n and a threshold K, report the
 * pairs (s_i, s_j), i != j, with ED(s_i, s_j) <= K.  EmbedJoin (Algorithms 1-3)
 * finds candidate pairs by embedding every string r times into Hamming space
 * with the CGK walk (Algorithm 1), hashing each embedding with z bit-sampling
 * LSH functions of m coordinates (Section 3.2, two-level hashing of Section
 * 4), keeping pairs that share a bucket in some table and differ in length by
 * at most K (Algorithm 3), and verifying every candidate with exact
 * threshold edit distance (Section 3.3).  The output is therefore exact in
 * precision and may miss pairs (recall < 1), fully determined by the inputs,
 * the parameters and the random seed.
 *
 * Conventions shared by every entry point
 *   - Strings are a byte array plus offsets: string i is
 *     chars[offsets[i] .. offsets[i+1]), offsets non-decreasing, n+1 entries.
 *     Strings may be empty.  Pairs refer to positions 0..n-1; identical
 *     strings at different positions are different strings.
 *   - Alphabet: the sorted set of distinct bytes of the input; the k-th
 *     smallest byte has code k-1 and the padding symbol (bottom) is |S|.
 *   - Randomness follows one counter-based specification (SplitMix64 words
 *     W(key, c) = Mix64(key + (c+1) * 0x9E3779B97F4A7C15)); stream keys are
 *     W(seed, tag << 32 | idx) with tag 0 for the random string R^l (idx l),
 *     tag 1 for LSH coordinates and tag 2 for the second-level hash vector of
 *     table (l, j) (idx l*z + j).  Bit b of R^l is bit b%64 of
 *     W(key_R, b/64); pi_j(sigma_k) is bit (j-1)*|S| + (k-1).  Coordinate k of
 *     table (l, j) is floor(W(key_POS, k) * L / 2^64) (drawn with
 *     replacement), and v_k = (W(key_V, k) >> 3) mod (2^61 - 1).
 *   - Bucket key of table (l, j) for a string: sum_k u_k v_k mod (2^61 - 1)
 *     with u_k = (symbol at coordinate k) + 1.
 *   - Truncation (Section 4.1): the embedding is cut to L symbols; L = 0
 *     selects ceil(average length); L is clamped to [1, 3N], N = max length.
 *   - Every call returns an ej_status.  No C++ exception crosses the ABI.
 *     On failure ej_last_error() describes the cause.
 *   - "d_" pointers are device pointers on the context's device; device work
 *     is enqueued on the context's stream.  Inputs are read-only and owned by
 *     the caller; device inputs must stay valid until the stream has
 *     finished the call.  Host inputs may be freed when the call returns.
 */
#ifndef EMBEDJOIN_H
#define EMBEDJOIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EJ_OK = 0,
    EJ_EINVAL = 1,      /* invalid argument (sizes, null pointers, offsets, r*z*m == 0 ...) */
    EJ_EALPHABET = 2,   /* byte outside the index alphabet, or a 256-symbol alphabet */
    EJ_ENOMEM = 3,      /* host or device allocation failed, or HBM admission refused */
    EJ_ECAPACITY = 4,   /* caller buffer too small; the required count was written */
    EJ_EHIP = 5,        /* a HIP runtime call failed */
    EJ_EUNSUPPORTED = 6 /* parameters outside what the kernels implement (see each call) */
} ej_status;

/* Flags of ej_params.flags */
#define EJ_FLAG_PLAIN 0u   /* one launch per stage, host-sized buffers */
#define EJ_FLAG_GRAPH 1u   /* the join after its preparation (A1-A6) sized on the device
                            and replayed from a HIP graph cached in the context per input
                            shape (buffers, sizes, alphabet, longest string, parameters,
                            knobs): the first join of a shape runs host-sized and sets the
                            candidate capacities, the second allocates every buffer at
                            them, later ones replay the graph; a count above a capacity
                            redoes the join host-sized and grows it.  With EJ_FLAG_TIMING,
                            or exact_len, only the persistent verification forms
                            ("verify_mode" 1 to 3) are captured, as a graph of their own.
                            Results are identical either way. */
#define EJ_FLAG_TIMING 2u  /* record per-stage device times in ej_result */
#define EJ_FLAG_DEVICE_OUT 4u /* leave the result in device memory: out->pairs and
                               out->dist are device pointers into the context's
                               workspace, valid until the next call on the
                               context (copy them out before it); out->on_device
                               is 1 and ej_result_free frees nothing */

typedef struct ej_ctx ej_ctx;

typedef struct {
    uint32_t K;      /* edit-distance threshold */
    uint32_t r;      /* number of CGK embeddings (seeds) per string */
    uint32_t z;      /* LSH functions per embedding */
    uint32_t m;      /* coordinates per LSH function (signature length) */
    uint32_t L;      /* truncation length, 0 = ceil(average length) */
    uint32_t flags;  /* EJ_FLAG_* */
    uint64_t seed;   /* seed of the counter-based random streams */
    uint32_t exact_len; /* 0, or S > 0: every pair of strings both no longer than S
                           whose lengths differ by at most K joins the candidates
                           as well (an exhaustive pass over the short strings, for
                           which the paper notes LSH filtering is a poor fit: with K
                           large next to their length, random short strings are
                           within K of each other by chance).  Output pairs among
                           such strings are then exact.  Applies to ej_join*,
                           ej_join_plus* and ej_join_grouped*; fails with
                           EJ_EUNSUPPORTED when the union would reach 2^32 pairs */
    uint32_t reserved; /* 0 */
} ej_params;

typedef struct {
    uint64_t count;        /* number of output pairs */
    uint32_t *pairs;       /* host (device with EJ_FLAG_DEVICE_OUT), [count][2], i < j,
                              sorted lexicographically */
    int32_t *dist;         /* host (device with EJ_FLAG_DEVICE_OUT), [count], the edit
                              distance of each pair (<= K) */
    uint64_t n_candidates; /* |C|: de-duplicated candidate pairs that were verified */
    uint64_t n_raw;        /* candidate pairs before de-duplication across tables */
    uint32_t sigma;        /* alphabet size */
    uint32_t L;            /* truncation length used */
    /* EJ_FLAG_TIMING: device time of each stage, from events on the context
     * stream: prep = A0 and the random streams, embed = the walk kernel (A1-A2),
     * bucket = A3, candidates = A4, verify = verification (A5: its kernel
     * launches and the compaction of the pairs still undecided after the first
     * pass), output = compaction and copy-out (A6). */
    float ms_prep, ms_embed, ms_bucket, ms_candidates, ms_verify, ms_output;
    /* EJ_FLAG_TIMING: work done, for rooflines.  walk_steps = CGK steps taken
     * (each walk stops after its seed's last sampled step); verify_columns =
     * text columns evaluated over all candidates (a pair stops early once its
     * distance provably exceeds K). */
    uint64_t walk_steps, verify_columns;
    /* EJ_FLAG_TIMING: summed device time of the verification kernel's own
     * launches (events right around each launch) and their number. */
    float ms_verify_kernel;
    uint32_t verify_launches;
    /* The verification form that ran: 0 two passes over groups of pairs,
     * 1 persistent groups of pairs, 2 one pair per lane, 3 several lanes per
     * pair with several band words each (2 and 3: "verify_mode" 2), 4 grouped
     * by pattern ("verify_mode" 3), 5 the two-pass form with two or four
     * band words per lane ("verify_wpl" 2 or 4). */
    uint32_t verify_form;
    /* 1 when pairs and dist are device pointers (EJ_FLAG_DEVICE_OUT) */
    uint32_t on_device;
    /* How the join ran (EJ_FLAG_GRAPH without EJ_FLAG_TIMING): 0 sized on the
     * host (stage by stage, sizes read back between stages), 1 sized on the
     * device but not captured (the run that allocates the buffers of a new
     * shape), 2 replayed as one captured graph of A1-A6. */
    uint32_t graph;
} ej_result;

/* ---------------------------------------------------------------- lifecycle */

/* Creates a context on `device`.  hip_stream (a hipStream_t) may be NULL: the
 * context then creates its own stream.  The context owns a grow-only device
 * workspace that is reused across calls. */
ej_status ej_create(ej_ctx **ctx, int device, void *hip_stream);
void ej_destroy(ej_ctx *ctx);
const char *ej_last_error(const ej_ctx *ctx);
/* Library version as major*10000 + minor*100 + patch. */
int ej_version(void);
/* Bytes of device workspace the context currently holds. */
uint64_t ej_workspace_bytes(const ej_ctx *ctx);

/* Launch-shape knobs of the context.  None of them changes any result:
 *   "verify_lds_budget"     LDS bytes per wave of the verification kernel
 *   "verify_pass1_cols"     columns of verification pass 1 (multiple of 32;
 *                           0 = a single pass)
 *   "verify_wpl"            two-pass verification: band words per lane, 1,
 *                           2 or 4 (default 2; 3 acts as 2; lowered until
 *                           the band has at least twice as many words)
 *   "verify_len_order"      two-pass verification: 1 (default) runs the
 *                           first pass in order of text length, longest
 *                           first, when some text is shorter than that pass
 *                           runs; 0 in pair order
 *   "verify_blocks_per_cu"  workgroups per CU of the verification grid (the
 *                           lane form: at most, below the occupancy limit)
 *   "verify_mode"           0: two passes over fixed groups of pairs, one
 *                           band word per lane (the first C1 columns of all,
 *                           then the survivors);
 *                           1: one persistent launch in which each pair's
 *                           lanes take the next pair from a device counter;
 *                           2: the lane form, persistent, with several band
 *                           words per lane ("verify_split" lanes per pair),
 *                           for alphabets of up to 4 symbols and bands of up
 *                           to 8 words per lane (16 with one lane per pair),
 *                           and with one lane per pair up to 32 symbols and
 *                           8 words; other inputs take form 1;
 *                           3: grouped by pattern: the pairs ordered by their
 *                           longer string and cut into chunks of at most 64
 *                           pairs of one pattern; a wave copies the pattern's
 *                           match masks into LDS once per chunk and each lane
 *                           runs one pair, its band (up to 16 words) in
 *                           registers; pairs of two string sets, and patterns
 *                           too long for LDS, take form 1
 *   "verify_split"          lane form: lanes per pair, 1, 2, 4, 8 or 16
 *                           (0 = by band width: 1 up to 4 words, 2 up to 8,
 *                           then 4)
 *   "verify_order"          joins only, two-pass and persistent forms: 0
 *                           pairs in list order, 1 most frequent pairs
 *                           (found by the most tables) first, which groups
 *                           the pairs that run to their end (the two-pass
 *                           form's first pass, within a text length) and
 *                           shortens the tail
 *   "verify_ring"           match-mask layout in LDS: 0 the whole pattern,
 *                           1 a ring of the words the band covers when it is
 *                           smaller, 2 the ring whenever the band has at
 *                           least 2 lanes
 *   "embed_lds_budget"      LDS bytes per wave of the walk kernel (0, the
 *                           default: the samples plus string windows of 16
 *                           words)
 *   "radix_bits"            digit width of the radix sorts (4..11)
 *   "bucket_key_bits"       key bits sorted when bucketing (1..32; 0 =
 *                           ceil(log2 n) + 6)
 *   "dedup_sort"            de-duplication of the candidates: 0 grouped by
 *                           the codes' top bits with an LDS hash per group
 *                           (a sort when a group is too large), 1 a sort
 *   "raw_limit"             raw candidate pairs one sort of the join may hold
 *                           (0, the default: 2^32 - 2).  A join with more
 *                           takes its candidate stage in passes over ranges
 *                           of the pairs' smaller index (same result); it
 *                           then runs host-sized, without the whole-join
 *                           graph
 * EJ_EINVAL for an unknown name or a value out of range. */
ej_status ej_tune_set(ej_ctx *ctx, const char *name, uint32_t value);
ej_status ej_tune_get(const ej_ctx *ctx, const char *name, uint32_t *value);

/* ------------------------------------------------------------- end to end */

/* EmbedJoin self-join (Algorithm 3 with Algorithm 2 as preprocessing) of the
 * host strings `strings`/`offsets` (n strings) with threshold K and
 * parameters r, z, m, the given seed and the default truncation.  The
 * library allocates out->pairs and out->dist (free with ej_result_free).
 * Errors: EJ_EINVAL (n >= 2^31, r*z*m == 0, m > 64, r*z > 4096,
 * non-monotone offsets, a string longer than 2^31 - 1), EJ_EALPHABET (all
 * 256 byte values present), EJ_EUNSUPPORTED (K > 2046), EJ_ENOMEM, EJ_EHIP. */
ej_status ej_join(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                  uint32_t K, uint32_t r, uint32_t z, uint32_t m, uint64_t seed,
                  ej_result *out);

/* As ej_join with every parameter of ej_params (L, flags). */
ej_status ej_join_ex(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                     const ej_params *p, ej_result *out);

/* As ej_join_ex with the strings already in device memory (d_offsets holds
 * n+1 absolute offsets into d_chars).  Results are still returned in host
 * memory.  This is the form whose time excludes the host-to-device copy. */
ej_status ej_join_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                         uint32_t n, const ej_params *p, ej_result *out);

/* EmbedJoin+ (Algorithms 4-5, Section 5), the variant for strings whose
 * alignments begin with a shift (a run of leading insertions).  Every string
 * s_i contributes ceil(K/delta) suffixes s_i[(k-1)*delta ..] (1-based k; a
 * suffix that starts past the end is empty), each embedded and hashed like a
 * string of its own with the same seeds, coordinates and truncation L.  A
 * table bucket holds (string, suffix) entries; two entries of different
 * strings whose lengths (of the whole strings) differ by at most K and that
 * share a bucket form a tuple (s, s', k, k').  A pair of strings is a
 * candidate when one of its tuples is found by at least T of the r*z tables;
 * candidates are verified exactly and the output has the layout of ej_join's
 * (n_raw = tuples found, with repetition).
 *   delta  suffix step; 0 selects floor(sqrt(ceil(average length))), at least 1
 *   T      tuple threshold; 0 selects 2 when ceil(K/delta) > 1, else 1 (with
 *          one suffix and T = 1 the result is exactly ej_join's)
 * Host strings; ej_join_plus_device takes device-resident ones (as
 * ej_join_device).  Errors as ej_join, plus EJ_EUNSUPPORTED when
 * r*z*n*ceil(K/delta) reaches 2^32. */
ej_status ej_join_plus(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                       const ej_params *p, uint32_t delta, uint32_t T, ej_result *out);
ej_status ej_join_plus_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                              uint32_t n, const ej_params *p, uint32_t delta, uint32_t T,
                              ej_result *out);

/* EmbedJoin with grouping instead of truncation (Section 4.1): the strings
 * are split into length groups -- group g (0-based) holds the strings of
 * length in (gK, (g+2)K], g < max(1, ceil(N/K) - 1), N the longest length;
 * group 0 also holds the empty strings; with K = 0 one group per length --
 * so every string is in at most two groups and every pair within K in
 * length shares one.  Each group is joined as a set of its own (its own
 * alphabet; walks of L = 3 x the group's longest string, untruncated, or the
 * caller's p->L; the same seed), and the result is the union: candidates are
 * the distinct pairs of all groups (a pair two groups find is verified
 * once), n_raw the sum of the groups' raw counts, out->L = p->L.  Host
 * strings; ej_join_grouped_device takes device-resident ones.  Errors as
 * ej_join. */
ej_status ej_join_grouped(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets,
                          uint32_t n, const ej_params *p, ej_result *out);
ej_status ej_join_grouped_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                                 uint32_t n, const ej_params *p, ej_result *out);

void ej_result_free(ej_result *res);

/* Autotuner of the batched form, for callers that run many joins of one
 * shape.  Joins the caller's device-resident strings (as ej_join_device)
 * repeatedly and descends one launch knob at a time (verification form,
 * first-pass columns, grid, match-mask layout, radix width), keeping in the
 * context the setting with the least wall time (best of `reps` joins per
 * trial).  No knob changes any result.  *best_ms (may be NULL) receives the
 * join time at the chosen setting.  About 15 trials; errors as
 * ej_join_device. */
ej_status ej_autotune(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                      const ej_params *p, uint32_t reps, float *best_ms);

/* --------------------------------------------------------- stage entry points
 * Each stage can be called on its own; ej_join chains the same kernels.
 * Sizes that depend on the data are returned in host memory, so these calls
 * synchronise the context stream before returning. */

/* A1-A2: CGK embedding of every string under r seeds (Algorithm 1 truncated
 * to L, Section 4.1), sampling of the z*m LSH coordinates of each seed
 * (Section 4, sparse embedding) and the two-level hash (Section 4).
 *   d_keys [r*z][n] uint64  key of string i in table l*z + j (input order)
 *   d_sig  [n][r][z][m] uint8 sampled symbol codes, or NULL
 * *L_used and *sigma receive the truncation length and alphabet size. */
ej_status ej_embed(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                   const ej_params *p, uint8_t *d_sig, uint64_t *d_keys, uint32_t *L_used,
                   uint32_t *sigma);

/* A3: bucketing (the hash tables D_j^l of Algorithm 3).  Each of the
 * `ntables` tables (keys laid out [ntables][n]) is sorted with a stable
 * on-device LSD radix sort:
 *   key_bits = 0: by (full key, string length, position); each group is
 *                 exactly one bucket D_j^l[key], its strings in length order;
 *   key_bits in 1..32: by (the top key_bits bits of the key, length,
 *                 position); a group then holds one or more whole buckets
 *                 (distinct full keys that share their top bits, rare with
 *                 enough bits), which ej_candidates tells apart by the full
 *                 key -- fewer sort passes, the form the join itself uses.
 *   d_len          [n] uint32 string lengths
 *   d_ids_sorted   [ntables][n] uint32 positions in sorted order
 *   d_group_start  capacity ntables*n + 1 uint32: index (into the
 *                  [ntables*n] sorted array) where each group starts, with
 *                  a final entry ntables*n
 *   *ngroups       number of groups */
ej_status ej_lsh_bucket(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_len, uint32_t n,
                        uint32_t ntables, uint32_t key_bits, uint32_t *d_ids_sorted,
                        uint32_t *d_group_start, uint64_t *ngroups);

/* A4: candidate pairs (Algorithm 3, with the sliding-window length test and
 * the de-duplication across tables): every pair of positions that share a
 * full key in some table and whose lengths differ by at most K, once.
 *   d_pairs   capacity `capacity` uint64 codes (i << 32) | j, i < j, sorted
 *   *count    number of candidates; if it exceeds `capacity` nothing is
 *             written to d_pairs and EJ_ECAPACITY is returned
 *   *n_raw    pairs found before de-duplication (may be NULL) */
ej_status ej_candidates(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_ids_sorted,
                        const uint32_t *d_group_start, uint64_t ngroups, const uint32_t *d_len,
                        uint32_t n, uint32_t ntables, uint32_t K, uint64_t *d_pairs,
                        uint64_t capacity, uint64_t *count, uint64_t *n_raw);

/* A5: threshold edit distance (Section 3.3) of each pair, with a
 * bit-parallel banded kernel: d_dist[k] = ED(s_a, s_b) if it is <= K_k,
 * else K_k + 1, where K_k = d_Kq[k] when d_Kq is not NULL and K otherwise.
 * Pairs are uint64 codes (a << 32) | b with a, b < n; the indexes are not
 * checked (one outside the set reads and writes outside its buffers).
 * EJ_EUNSUPPORTED if a threshold exceeds 2046. */
ej_status ej_verify(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                    const uint64_t *d_pairs, uint64_t count, uint32_t K, const uint32_t *d_Kq,
                    int32_t *d_dist);

/* ej_verify for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as ej_verify; it calls no device allocator.
 * Its workspace (symbol codes, match masks, counters) is carved from one
 * static device array of 64 MiB per GPU, which each GPU the library runs on
 * holds from the first context created on it until the process ends.  Inputs
 * whose workspace exceeds it are refused with EJ_ENOMEM before any
 * distance is written (a DNA set needs about 1.3 bytes per character plus 24
 * bytes per string; 25 letters about 4.2 bytes per character); use ej_verify
 * for those.  The two-pass verification form ("verify_mode" 0) runs as the
 * persistent form, which needs no per-pair state; no result changes.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * behind: calls that overlap on one GPU (from several host threads, or on
 * several contexts' streams without ordering between them) race, and the
 * caller must serialise them. */
ej_status ej_verify_static(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                           uint32_t n, const uint64_t *d_pairs, uint64_t count, uint32_t K,
                           const uint32_t *d_Kq, int32_t *d_dist);

/* ------------------------------------------------ diagnostics, calibration
 * Distortion of the CGK embedding (Section 3.1: Hamming distance of the
 * embeddings against edit distance, best of r embeddings) and the
 * normalised Hamming distance under truncation (Section 6), on the device.
 * d_ham [count][r] uint32: for pair e = (a << 32) | b and seed l < p->r, the
 * Hamming distance between the first L symbols (p->L; 0 = ceil(average
 * length), at most 3N) of the embeddings of s_a and s_b under R^l.  With
 * delta > 0 each string contributes ceil(p->K / delta) suffixes (as in
 * ej_join_plus) and the value is the minimum over the suffix pairs.  p->z and
 * p->m are ignored.  Errors: EJ_EINVAL (a position >= n, r = 0),
 * EJ_EUNSUPPORTED (more than 64 suffixes per string). */
ej_status ej_embed_hamming(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                           uint32_t n, const ej_params *p, uint32_t delta,
                           const uint64_t *d_pairs, uint64_t count, uint32_t *d_ham);

typedef struct {
    uint32_t K;              /* threshold of the join to calibrate */
    uint32_t delta;          /* 0: EmbedJoin; > 0: EmbedJoin+ with this suffix step */
    uint32_t T;              /* EmbedJoin+ tuple threshold (0: 2 if ceil(K/delta) > 1, else 1) */
    uint32_t r_max;          /* seeds embedded; every r in 1..r_max is scored */
    const uint32_t *z_list;  /* host arrays of the values to score */
    uint32_t nz;
    const uint32_t *m_list;  /* 1..64 each */
    uint32_t nm;
    const uint32_t *L_list;  /* truncations; 0 = ceil(average length); clamped to [1, 3N] */
    uint32_t nL;
    double target_recall;    /* the predicted recall the chosen point must reach */
    uint64_t seed;           /* the seed the join will use */
    uint32_t exact_len;      /* the join's ej_params.exact_len: a sample pair whose strings
                                are both no longer than it is a candidate with certainty
                                (in the recall, and in the false rate and work, where it
                                adds the same amount at every grid point); 0: no short pass */
    uint32_t reserved;       /* 0 */
} ej_calib_opts;

typedef struct {
    uint32_t r, z, m, L;     /* the chosen point; r = 0 if no point reaches the target */
    double recall;           /* its predicted recall over the sample pairs within K */
    double false_rate;       /* its predicted chance that a sample pair beyond K is a candidate */
    double work;             /* its predicted work per string (32-bit operations) */
    uint64_t n_similar;      /* sample pairs within K (exact distance) */
    uint64_t n_dissimilar;   /* sample pairs beyond K */
    double best_recall;      /* the highest predicted recall on the grid */
} ej_calib_result;

/* Automated choice of (r, z, m, L) for a join of these strings at threshold
 * K, from sample pairs (d_pairs, codes (a << 32) | b) that stand for the
 * similar and dissimilar pairs of the workload (say, known-similar pairs and
 * random pairs).  Each sample pair's exact distance decides whether it is
 * within K; its embeddings' Hamming distances under the first r_max seeds
 * (as ej_embed_hamming, at every L of the list) give, per grid point, the
 * probability that the join makes it a candidate: with q_l = (1 - H_l/L)^m
 * per table of seed l, 1 - prod_{l<r} (1 - q_l)^z for EmbedJoin, and for
 * EmbedJoin+ the probability that the closest suffix pair is counted in at
 * least T tables (a lower bound).  Predicted recall = the mean over pairs
 * within K; false rate = the mean over pairs beyond K.  The chosen point
 * reaches target_recall with the least predicted work per string: 3 r k L
 * (walk) + 10 r k z m (hash) + 60 r k z (bucketing) + false_rate (n-1)/2
 * 10 (K+1)/32 min(2K+64, average length) (rejecting false candidates), with
 * k = ceil(K/delta) suffixes (1 for EmbedJoin).  table (host, may be NULL)
 * receives [nL][r_max][nz][nm][3] = (recall, false rate, work) of every
 * point.  Errors as ej_verify and ej_embed_hamming, EJ_EINVAL for an empty
 * grid or r_max * z above 4096. */
ej_status ej_calibrate(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                       const uint64_t *d_pairs, uint64_t count, const ej_calib_opts *opts,
                       ej_calib_result *out, double *table);

/* Issue-rate probe for the integer-VALU roofline of verification: runs a
 * kernel of independent dependency chains (96 VALU instructions per loop
 * iteration, no memory traffic) on blocks_per_cu workgroups of 256 lanes per
 * CU for `iters` iterations and returns the achieved lane operations per
 * second and the kernel time (one untimed launch runs first).  mix selects
 * the instructions, all with register or inline-constant operands: 0
 * verification's add / 3-input logic / funnel shift in turn; 1 32-bit add;
 * 2 xor; 3 3-input logic (v_bitop3); 4 funnel shift; 5 add with the
 * carry-out to a scalar mask; 6 add with carry in and out (a carry chain);
 * 7 compare to VCC; 8 DPP one-lane shift across the wave; 9 popcount-add;
 * 10 three-input add; 11 select on a scalar mask; 12 three-input or; 13
 * and-or; 14 24-bit multiply of a selected byte.  EJ_EINVAL for iters = 0,
 * blocks_per_cu outside 1..64 or mix above 14. */
ej_status ej_probe_valu(ej_ctx *ctx, uint32_t mix, uint32_t iters, uint32_t blocks_per_cu,
                        double *lane_ops, float *ms);

/* Test hook: replace the drawn randomness of the next calls by explicit
 * values (host arrays): Rbits [r][L*sigma] 0/1 bytes (pi_j(sigma_k) at
 * (j-1)*sigma + k-1), pos [r][z][m] coordinates < L, v [r][z][m] values
 * < 2^61-1 or NULL (then v is drawn from the seed).  The values apply only
 * to calls with the same r, z, m, L and alphabet size.  Passing Rbits ==
 * NULL clears the override. */
ej_status ej_set_explicit_randomness(ej_ctx *ctx, uint32_t r, uint32_t z, uint32_t m,
                                     uint32_t L, uint32_t sigma, const uint8_t *Rbits,
                                     const uint32_t *pos, const uint64_t *v);

/* ------------------------------------------------------------------ serving
 * A device-resident LSH index over a fixed collection (the embedding and
 * bucketing stages run once at build time; queries are embedded with the
 * same random streams, truncation and alphabet).  Result of query q: the
 * index positions s that share a full key with q in some table, satisfy
 * ||q| - |s|| <= K_q and ED(q, s) <= K_q, sorted by position. */
typedef struct ej_index ej_index;

typedef struct {
    uint32_t nq;
    uint64_t *offsets;     /* host, [nq+1]: results of query q are [offsets[q], offsets[q+1]) */
    uint32_t *ids;         /* host, index positions */
    int32_t *dist;         /* host, edit distances */
    uint64_t n_candidates; /* (query, index) pairs verified */
    float ms_total;        /* device time of the batch */
    uint64_t workspace_bytes; /* the batch's admission figure: the estimate before
                                 embedding plus the candidate and verification
                                 stages' bytes once their counts were known */
} ej_qresult;

/* Builds the index from host (on_device = 0) or device (1) strings.  p->K is
 * ignored (thresholds come per query); p->L = 0 picks ceil(average length). */
ej_status ej_index_build(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                         const ej_params *p, int on_device, ej_index **index);
/* Adds n_new strings (host, or device with on_device = 1) to the index
 * (Algorithm 3 stores each string in its tables as it is visited; here a
 * batch at once).  They take positions ej_index_size() .. + n_new - 1 and are
 * embedded with the index's alphabet, truncation and random streams (fixed
 * at build: a byte outside the alphabet is EJ_EALPHABET).  The indexed
 * strings are not embedded again: each table's sorted entries are merged
 * with the new strings' (one binary search per entry), and the strings'
 * codes and match masks are extended.  Later queries answer over the grown
 * set exactly as an index built from all the strings with that alphabet,
 * truncation and seed.  On failure (EJ_ENOMEM for the grown arrays, which
 * are allocated beside the current ones) the index is unchanged. */
ej_status ej_index_insert(ej_index *index, const uint8_t *strings, const uint64_t *offsets,
                          uint32_t n_new, int on_device);
/* Answers nq queries (host strings) with per-query thresholds Kq (host).
 * Query i is q[q_offsets[i] .. q_offsets[i+1]); q_offsets[0] need not be 0,
 * so a batch can be a window of a larger buffer.
 * EJ_EALPHABET if a query byte is outside the index alphabet; EJ_ENOMEM if
 * the batch's workspace exceeds the free HBM at the call (or the admission
 * limit set with ej_index_set_hbm_limit).  Admission is checked three times,
 * each before the memory it counts is requested: with the estimate of
 * ej_query_workspace_estimate, again once the candidate count before
 * de-duplication is known, and again once the de-duplicated count (and so
 * verification's state and the query masks) is known; a refused batch
 * leaves the index usable. */
ej_status ej_query_batch(ej_index *index, const uint8_t *q, const uint64_t *q_offsets,
                         uint32_t nq, const uint32_t *Kq, ej_qresult *out);
/* Bytes of device memory the batch needs before its candidates are known
 * (the first admission check). */
uint64_t ej_query_workspace_estimate(const ej_index *index, const uint64_t *q_offsets,
                                     uint32_t nq, const uint32_t *Kq);
/* Caps the HBM the index may use for a batch (0 = free HBM reported by HIP). */
void ej_index_set_hbm_limit(ej_index *index, uint64_t bytes);
uint32_t ej_index_size(const ej_index *index);
void ej_qresult_free(ej_qresult *res);
void ej_index_free(ej_index *index);

#ifdef __cplusplus
}
#endif
#endif /* EMBEDJOIN_H */
