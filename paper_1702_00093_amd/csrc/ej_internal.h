// Internal declarations shared by the translation units of libembedjoin.so.
// Not part of the ABI (include/embedjoin.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <new>
#include <map>
#include <string>
#include <vector>

#include "embedjoin.h"

namespace ej {

// ------------------------------------------------------------------ errors --
struct Error {
    ej_status code;
    std::string msg;
};

[[noreturn]] void fail(ej_status code, const std::string &msg);

#define EJ_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::ej::fail(e_ == hipErrorOutOfMemory ? EJ_ENOMEM : EJ_EHIP,                  \
                       std::string(#call) + ": " + hipGetErrorString(e_));               \
    } while (0)

#define EJ_CHECK_LAUNCH() EJ_HIP(hipGetLastError())

// ---------------------------------------------------------------- constants --
constexpr uint64_t P61 = (1ULL << 61) - 1ULL;
constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ULL;
constexpr uint32_t TAG_R = 0, TAG_POS = 1, TAG_V = 2;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
// Word c of the SplitMix64 stream seeded with key (counter form).
__host__ __device__ inline uint64_t rng_word(uint64_t key, uint64_t c) {
    return mix64(key + (c + 1ULL) * GAMMA);
}
__host__ __device__ inline uint64_t stream_key(uint64_t seed, uint32_t tag, uint32_t idx) {
    return rng_word(seed, ((uint64_t)tag << 32) | idx);
}

// Lane broadcasts.  The builtin returns a signed int; widen through uint32_t so
// that 64-bit values (pointers, indices) are not sign-extended.
__device__ inline uint32_t readlane_u32(uint32_t v, uint32_t lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}
__device__ inline uint64_t readlane_u64(uint64_t v, uint32_t lane) {
    return ((uint64_t)readlane_u32((uint32_t)(v >> 32), lane) << 32) |
           (uint64_t)readlane_u32((uint32_t)v, lane);
}

// ---------------------------------------------------------------- context --
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Explicit {
    bool active = false;
    uint32_t r = 0, z = 0, m = 0, L = 0, sigma = 0;
    std::vector<uint32_t> Rwords;  // [r][nw] packed bits
    uint32_t nw = 0;
    std::vector<uint32_t> pos;     // [r][z][m]
    std::vector<uint64_t> v;       // [r][z][m] (empty: drawn)
};

// Workspace carved from one fixed device buffer instead of grown with
// hipMalloc (active while `base` is set): a bump allocator whose regions are
// keyed by name, so that a name asked for twice gets the same memory.
struct Arena {
    uint8_t *base = nullptr;
    size_t cap = 0, used = 0;
    std::map<std::string, std::pair<size_t, size_t>> named;  // name -> (offset, bytes)
};

struct Timers {
    hipEvent_t ev[8] = {};
    // around each launch of the verification kernel while `on`
    hipEvent_t kv[4] = {};
    int nkv = 0;
    uint32_t more = 0;  // further launches inside one pair of events
    bool on = false;
};

}  // namespace ej

namespace ej {
// Launch-shape knobs.  Defaults are set at context creation; the autotuner
// (ej_autotune) can replace them.  None of them changes a result.
struct Tuning {
    uint32_t verify_lds_budget = 48 * 1024;  // LDS per wave of the verification kernel
    uint32_t verify_pass1_cols = 1024;       // columns of verification pass 1 (0: one pass)
    uint32_t verify_blocks_per_cu = 64;      // resident-wave target of the verification grid
    uint32_t verify_order = 1;               // joins: 0 pair order, 1 by table multiplicity
    uint32_t verify_mode = 0;                // 0 two passes over pair tiles, 1 persistent pair queue
    uint32_t verify_split = 0;               // lane form: lanes per pair (0 auto, 1, 2, 4, 8, 16)
    uint32_t verify_ring = 1;                // match masks: 0 whole pattern, 1 auto, 2 ring if it fits
    uint32_t embed_lds_budget = 0;  // LDS per wave of the walk kernel (0: windows of 16 words)
    uint32_t radix_bits = 8;                 // digit width of the radix sorts
    uint32_t bucket_key_bits = 0;            // key bits sorted when bucketing, 0 = ceil(log2 n) + 6
    uint32_t dedup_sort = 0;                 // candidates: 0 grouped (sort on overflow), 1 sort
    uint32_t raw_limit = 0;  // raw pairs per sort of the candidate stage (0: 2^32 - 2)
    uint32_t verify_wpl = 2;  // two-pass verification: band words per lane (1, 2, 4)
    uint32_t verify_len_order = 1;  // two-pass: first pass in text-length order (0 off)
};
}  // namespace ej

namespace ej {
// Capacities of a join sized on the device (EJ_FLAG_GRAPH): raw and distinct
// candidate pairs; gen = the workspace generation after the last uncaptured
// run at these capacities (a capture needs every buffer to exist already);
// no_graph = the shape stays host-sized (a capture failed, or a capacity
// would reach 2^32); sort_dedup = de-duplicate by a sort (the grouped form
// overflowed, or the knob asks for it).
struct JoinCaps {
    uint64_t raw_cap = 0, cnt_cap = 0;
    uint64_t gen = ~0ull;
    bool no_graph = false;
    bool sort_dedup = false;  // de-duplicate by a sort (the grouped form overflowed)
};
}  // namespace ej

struct ej_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::map<std::string, ej::DevBuf> ws;
    ej::Explicit ex;
    int num_cu = 256;
    int lds_max = 65536;         // max dynamic LDS per workgroup
    uint64_t *pinned = nullptr;  // small pinned host buffer for size read-backs
    uint8_t *pinned_out = nullptr;  // grow-only pinned staging of join results
    size_t pinned_out_bytes = 0;
    ej::Timers timers;
    ej::Tuning tune;
    ej::Arena arena;             // set only inside ej_verify_static
    // EJ_FLAG_GRAPH: graphs of fixed launch sequences, keyed by every
    // argument of their launches (pointers included), replayed on a match
    bool graph_on = false;
    std::map<std::string, hipGraphExec_t> graphs;
    bool capturing = false;    // a graph capture is open on the stream
    bool last_dedup_sorted = false;  // the last candidates() de-duplicated by a sort
    uint64_t ws_gen = 0;       // workspace (re)allocations so far
    // joins sized on the device, per input shape: the capacities of their
    // candidate buffers and the workspace generation they were allocated in
    std::map<std::string, ej::JoinCaps> join_caps;
    uint32_t last_verify_form = 0;  // form of the last verification launched
};

namespace ej {

// Runs fn for an entry point of the C ABI: the context's device is made
// current, an Error becomes its status code and message (the stream is
// drained and the HIP error state cleared), a failed host allocation becomes
// EJ_ENOMEM.  No exception leaves.
template <typename F>
ej_status run_guarded(ej_ctx *ctx, F &&fn);

void *ws_get(ej_ctx *ctx, const std::string &name, size_t bytes);
// Size of the static scratch array of ej_verify_static (one per device).
constexpr size_t STATIC_SCRATCH_BYTES = 64ull << 20;
// Device address of the context device's static scratch array, looked up
// once per device when a context is created.
void *static_scratch(ej_ctx *ctx);
// Bytes the workspace buffer `name` holds now (0 if it does not exist).
size_t ws_capacity(ej_ctx *ctx, const std::string &name);
template <typename T>
T *ws(ej_ctx *ctx, const std::string &name, size_t count) {
    return (T *)ws_get(ctx, name, count * sizeof(T));
}
void sync(ej_ctx *ctx);
// Runs `enqueue` (kernel launches only: no allocation, synchronisation or
// memset) directly, or, with the context's graph mode on, as a captured graph
// cached under `key`, which must identify every argument of the launches.
void run_captured(ej_ctx *ctx, const std::string &key, const std::function<void()> &enqueue);
// Copies `count` u64 words from device to host through the pinned buffer.
void read_back(ej_ctx *ctx, const void *dsrc, size_t bytes, void *hdst);

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }
inline uint32_t bits_for(uint64_t v) {  // bits needed to represent values 0..v
    uint32_t b = 0;
    while (b < 64 && (v >> b) != 0) b++;
    return b;
}

// --------------------------------------------------------------- primitives --
// Exclusive prefix sum of n values (in place allowed).  *d_total (device,
// nullable) receives the sum.
void scan_exclusive_u32(ej_ctx *ctx, const uint32_t *d_in, uint32_t *d_out, uint64_t n,
                        uint64_t *d_total);
void scan_exclusive_u64(ej_ctx *ctx, const uint64_t *d_in, uint64_t *d_out, uint64_t n,
                        uint64_t *d_total);

// Stable LSD radix sort of `nseg` independent equal-length segments of
// `seglen` entries, ordered by bits [0, key_bits) of the keys.  Values
// (nullable) move with the keys.  Results end in the _out arrays; the _in
// arrays may be clobbered.  digit_bits in {4..11}.
void radix_sort_u32(ej_ctx *ctx, uint32_t *keys_in, uint32_t *vals_in, uint32_t *keys_out,
                    uint32_t *vals_out, uint32_t nseg, uint32_t seglen, uint32_t key_bits,
                    uint32_t digit_bits);
// 64-bit keys with 32-bit values, nseg segments of seglen entries sorted each
void radix_sort_u64_kv(ej_ctx *ctx, uint64_t *keys_in, uint32_t *vals_in, uint64_t *keys_out,
                       uint32_t *vals_out, uint32_t nseg, uint32_t seglen, uint32_t key_bits,
                       uint32_t digit_bits);
void radix_sort_u64(ej_ctx *ctx, uint64_t *keys_in, uint64_t *keys_out, uint64_t n,
                    uint32_t key_bits, uint32_t digit_bits);


// ------------------------------------------------------------------ stages --
struct Prep {
    uint32_t n = 0;
    uint64_t base = 0;      // offsets[0]
    uint64_t total = 0;     // total bytes
    uint32_t maxlen = 0;
    uint32_t minlen = 0;    // shortest string (0 for an empty set)
    uint32_t sigma = 0;
    uint8_t lut[256];
    uint32_t L = 0;
    uint32_t bw = 8;        // bits per packed code
    const uint64_t *d_offsets = nullptr;
    const uint8_t *d_chars = nullptr;
    uint32_t *d_len = nullptr;      // [n]
    uint8_t *d_codes = nullptr;     // [total] symbol codes, same layout as chars (base-relative)
    uint32_t *d_packed = nullptr;   // packed codes, bw bits each, base-relative
    uint32_t *d_perm = nullptr;     // [n] positions in (length, position) order
};

struct Rand {
    uint32_t r = 0, z = 0, m = 0, L = 0, sigma = 0;
    uint32_t S = 0;              // z*m samples per seed
    uint32_t Lpad = 0;           // stride of Rstep rows
    uint32_t nw = 0;             // stride of Rwords rows (u32)
    uint32_t Jmax = 0;           // max over seeds of (last sampled step + 1)
    uint32_t *d_Rwords = nullptr;  // [r][nw]
    uint32_t *d_Rstep = nullptr;   // [r][Lpad] bits of step j (sigma <= 32)
    uint32_t *d_pos = nullptr;     // [r][z][m]
    uint64_t *d_v = nullptr;       // [r][z][m]
    uint32_t *d_spos = nullptr;    // [r][S] sampled steps, ascending
    uint32_t *d_sslot = nullptr;   // [r][S] slot (j*m + k) of each sample
    uint32_t *d_J = nullptr;       // [r] last sampled step + 1
};

// Computes lengths, alphabet, truncation and encodings of a device string set.
// If `fixed_alphabet` is non-null its 256-entry table (code or 0xFF) is used
// and bytes outside it are an error.
void prepare(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
             uint32_t L_req, Prep &pp, const char *tag, const uint8_t *fixed_lut = nullptr,
             uint32_t fixed_sigma = 0, uint32_t fixed_L = 0, bool need_perm = true);
void draw_randomness(ej_ctx *ctx, const ej_params &p, uint32_t L, uint32_t sigma, Rand &rd,
                     const char *tag);
// With d_dk (and d_rank_ids), also the bucketing sort's input: for table t
// and length rank k, d_dk[t*n + k] = key >> dk_shift of the string of rank k
// and d_rank_ids[t*n + k] = that string's index.
void embed_keys(ej_ctx *ctx, const Prep &pp, const Rand &rd, uint64_t *d_keys, uint8_t *d_sig,
                uint32_t *d_dk = nullptr, uint32_t *d_rank_ids = nullptr, uint32_t dk_shift = 0);

// Distortion diagnostic: d_ham[e * r + l] = Hamming distance between the
// first L symbols of the embeddings of pair e's strings under seed l (the
// minimum over the kappa^2 suffix pairs, suffix k starting at k * delta).
void embed_hamming(ej_ctx *ctx, const Prep &pp, const Rand &rd, const uint64_t *d_pairs,
                   uint64_t count, uint32_t kappa, uint32_t delta, uint32_t *d_ham);
// Rejects (EJ_EINVAL) pairs whose positions are not below n_a / n_b.
void check_pairs(ej_ctx *ctx, const uint64_t *d_pairs, uint64_t count, uint32_t n_a,
                 uint32_t n_b);

struct Buckets {
    uint32_t T = 0, n = 0;
    uint32_t *d_ids = nullptr;        // [T*n]
    uint32_t *d_gid = nullptr;        // [T*n] group id of each sorted entry
    uint32_t *d_gstart = nullptr;     // [ngroups + 1]
    uint64_t ngroups = 0;
    // [T*n] sorted top key bits: set instead of d_gid/d_gstart when the
    // groups are not built (the pair walk then ends a group where they change)
    uint32_t *d_dk = nullptr;
};
// Key bits the bucketing sorts (key_bits 0: the context's knob, then
// ceil(log2 n) + 6).
uint32_t bucket_key_bits(ej_ctx *ctx, uint32_t n, uint32_t key_bits);
// The workspace buffers of bucket()'s sort input (top key bits and string
// indexes in length order, per table); inputs_ready = the caller filled them
// (embed_keys with d_dk) and bucket() skips its gather.
void bucket_inputs(ej_ctx *ctx, uint64_t tot, const char *tag, uint32_t **d_dk, uint32_t **d_ids);
// bk.ngroups is read back to the host only when want_ngroups is set.
// want_groups = false skips the group ids and starts and leaves the sorted
// top key bits in bk.d_dk (all that candidates() needs).
void bucket(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_len, const uint32_t *d_perm,
            uint32_t n, uint32_t T, uint32_t key_bits, Buckets &bk, const char *tag,
            bool want_ngroups = false, bool inputs_ready = false, bool want_groups = true);
// The candidate stage sized on the device (for a join captured as one graph):
// raw pairs into raw_cap entries, distinct pairs into cnt_cap; counts left in
// cnt_dev[0] (raw), [1] (distinct), [2] (nonzero: the grouped de-duplication
// overflowed).  The result is valid only when both counts fit and [2] is 0.
void candidates_dev(ej_ctx *ctx, const uint64_t *d_keys, const Buckets &bk,
                    const uint32_t *d_len, uint32_t K, uint64_t raw_cap, uint64_t cnt_cap,
                    bool want_order, bool sort_dedup, uint64_t *cnt_dev, uint64_t **d_pairs_out,
                    uint32_t **d_order_out, const char *tag);
// Exact buckets: every table sorted by (full key, length, position), one group
// per distinct key (d_gid, d_gstart and ngroups set).
void bucket_exact(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_perm, uint32_t n,
                  uint32_t T, Buckets &bk, const char *tag);

// Candidate pairs as packed codes (a << 32 | b), a < b, sorted and unique.
// Returns the count; *n_raw gets the pre-dedup count.
// With d_order_out, also a verification order of the pairs: by decreasing
// number of tables that produced the pair (ties by position), so that pairs
// likely to run their full length start first.
uint64_t candidates(ej_ctx *ctx, const uint64_t *d_keys, const Buckets &bk, const uint32_t *d_len,
                    uint32_t K, uint64_t **d_pairs_out, uint64_t *n_raw, const char *tag,
                    uint32_t **d_order_out = nullptr);

// EmbedJoin+ candidates over bucketed suffix entries (entry e = suffix
// e % kappa of string e / kappa; d_len_entry = the whole string's length):
// pairs of strings with some (suffix, suffix) tuple found by at least T
// tables, codes (a << 32) | b, a < b, sorted and unique.  *n_raw gets the
// number of tuples found (with repetition).
uint64_t candidates_plus(ej_ctx *ctx, const uint64_t *d_keys, const Buckets &bk,
                         const uint32_t *d_len_entry, uint32_t K, uint32_t nstr, uint32_t kappa,
                         uint32_t T, uint64_t **d_pairs_out, uint64_t *n_raw, const char *tag);

// One of each code of a sorted array of pair codes (a << B | b), unpacked to
// (a << 32) | b into a workspace buffer named after `tag`; returns the count.
uint64_t unique_sorted_pairs(ej_ctx *ctx, const uint64_t *d_sorted, uint64_t cnt, uint32_t B,
                             uint64_t **d_out, const char *tag);

// Match masks of a string set, one bit array per (string, symbol): bit b of
// word w of string s and symbol c is set iff x_s[32w + b] == c, for
// W_s = ceil(|x_s| / 32) words; string s's arrays start at word off[s].
struct RowMasks {
    const uint32_t *words = nullptr;
    const uint64_t *off = nullptr;
    uint32_t n = 0;  // strings (0: unknown)
};
// Builds the masks of n strings (codes laid out like the characters, offsets
// relative to `base`) into workspace buffers named after `tag`, or into
// `own_words`/`own_off` when given (capacity mask_words_bound / n).
void build_masks(ej_ctx *ctx, const uint8_t *d_codes, const uint64_t *d_offsets, uint64_t base,
                 uint32_t n, uint64_t total, uint32_t sigma, RowMasks &rm, const char *tag,
                 uint32_t *own_words = nullptr, uint64_t *own_off = nullptr);
inline uint64_t mask_words_bound(uint64_t total, uint32_t n, uint32_t sigma) {
    return (uint64_t)(sigma ? sigma : 1) * (total / 32 + n + 1);
}

// Threshold edit distance of `count` pairs (codes a << 32 | b) over the
// symbol codes of a string set (a) and a second set (b, or a again).
void verify(ej_ctx *ctx, const uint8_t *d_codes, const uint64_t *d_offsets, uint64_t base,
            uint32_t sigma, uint32_t maxlen, const RowMasks &masks, const uint64_t *d_pairs,
            uint64_t count, uint32_t K, const uint32_t *d_Kq, int32_t *d_dist,
            const uint8_t *d_codes_b = nullptr, const uint64_t *d_offsets_b = nullptr,
            uint64_t base_b = 0, uint32_t maxlen_b = 0, const RowMasks *masks_b = nullptr,
            unsigned long long *d_columns = nullptr, const uint32_t *d_order = nullptr,
            const uint64_t *d_count = nullptr, uint32_t minlen = 0);

uint32_t verify_lanes_for(uint32_t K);  // lanes per pair, 0 if unsupported

template <typename F>
ej_status run_guarded(ej_ctx *ctx, F &&fn) {
    if (!ctx) return EJ_EINVAL;
    try {
        EJ_HIP(hipSetDevice(ctx->device));
        fn();
        ctx->err.clear();
        return EJ_OK;
    } catch (const Error &e) {
        ctx->err = e.msg;
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipGetLastError();
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return EJ_ENOMEM;
    }
}

}  // namespace ej
