// End-to-end join (A0-A6) and the stage entry points of the C ABI.
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <vector>

#include "ej_internal.h"

namespace ej {

namespace {

inline uint32_t grid_for(ej_ctx *ctx, uint64_t work, uint32_t block) {
    uint64_t g = (work + block - 1) / block;
    uint64_t cap = (uint64_t)ctx->num_cu * 16;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return (uint32_t)g;
}

__global__ void k_out_flags(const int32_t *__restrict__ dist, uint64_t cnt,
                            const uint64_t *__restrict__ cnt_dev, uint32_t K,
                            uint32_t *__restrict__ flags) {
    // with a count on the device, entries past it hold no distance
    const uint64_t live = cnt_dev ? min(*cnt_dev, cnt) : cnt;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x)
        flags[e] = (e < live && dist[e] >= 0 && (uint32_t)dist[e] <= K) ? 1u : 0u;
}

__global__ void k_out_compact(const uint64_t *__restrict__ pairs, const int32_t *__restrict__ dist,
                              uint64_t cnt, const uint32_t *__restrict__ flags,
                              const uint32_t *__restrict__ pos, uint32_t *__restrict__ out_pairs,
                              int32_t *__restrict__ out_dist) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x) {
        if (flags[e]) {
            uint32_t p = pos[e];
            uint64_t c = pairs[e];
            out_pairs[2 * (uint64_t)p] = (uint32_t)(c >> 32);
            out_pairs[2 * (uint64_t)p + 1] = (uint32_t)c;
            out_dist[p] = dist[e];
        }
    }
}

__global__ void k_gid_from_starts(const uint32_t *__restrict__ gstart, uint64_t ngroups,
                                  uint32_t *__restrict__ gid) {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ngroups;
         g += (uint64_t)gridDim.x * blockDim.x)
        for (uint32_t e = gstart[g]; e < gstart[g + 1]; e++) gid[e] = (uint32_t)g;
}

__global__ void k_max_len_shim(const uint32_t *__restrict__ a, uint32_t n, uint32_t *__restrict__ out) {
    uint32_t mx = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        mx = max(mx, a[i]);
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, mx);
}

__global__ void k_iota_shim(uint32_t *__restrict__ a, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        a[i] = i;
}

// Flags (bit 0) a pair whose positions are not below n_a / n_b.
__global__ void k_check_pairs(const uint64_t *__restrict__ pairs, uint64_t cnt, uint32_t n_a,
                              uint32_t n_b, uint32_t *__restrict__ bad) {
    uint32_t b = 0;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t c = pairs[e];
        if ((uint32_t)(c >> 32) >= n_a || (uint32_t)c >= n_b) b = 1;
    }
    if (b) atomicOr(bad, 1u);
}

// Flags group starts that are not increasing from 0 to tot.
__global__ void k_check_groups(const uint32_t *__restrict__ gs, uint64_t ng, uint64_t tot,
                               uint32_t *__restrict__ bad) {
    uint32_t b = 0;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < ng;
         g += (uint64_t)gridDim.x * blockDim.x) {
        if (gs[g] >= gs[g + 1] || gs[g + 1] > tot) b = 1;
        if (g == 0 && gs[0] != 0) b = 1;
        if (g == ng - 1 && gs[ng] != tot) b = 1;
    }
    if (b) atomicOr(bad, 1u);
}

// EmbedJoin+ suffix entries (Algorithm 4): entry e = i * kappa + k is
// s_i[k * delta ..] (empty once k * delta >= |s_i|): its start offset and
// length for the walk, and the whole string's length for the length window.
__global__ void k_suffix_entries(const uint64_t *__restrict__ offsets,
                                 const uint32_t *__restrict__ len, uint32_t n, uint32_t kappa,
                                 uint32_t delta, uint64_t *__restrict__ sstart,
                                 uint32_t *__restrict__ slen, uint32_t *__restrict__ flen) {
    const uint64_t ne = (uint64_t)n * kappa;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < ne;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(e / kappa), k = (uint32_t)(e - (uint64_t)i * kappa);
        const uint32_t l = len[i];
        const uint64_t want = (uint64_t)k * delta;
        const uint32_t skip = want < l ? (uint32_t)want : l;
        sstart[e] = offsets[i] + skip;
        slen[e] = l - skip;
        flen[e] = l;
    }
}

// Entries in the strings' length order, each string's suffixes together:
// rank r is suffix r % kappa of the string of length rank r / kappa.
__global__ void k_entry_perm(const uint32_t *__restrict__ perm, uint32_t n, uint32_t kappa,
                             uint32_t *__restrict__ eperm) {
    const uint64_t ne = (uint64_t)n * kappa;
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < ne;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(r / kappa), k = (uint32_t)(r - (uint64_t)i * kappa);
        eperm[r] = perm[i] * kappa + k;
    }
}

// Grouping: the strings of one length group copied into a compact set
// (block b copies string ids[b] to dst + soff[b]).
__global__ void k_gather_strings(const uint8_t *__restrict__ chars,
                                 const uint64_t *__restrict__ offsets,
                                 const uint32_t *__restrict__ ids, uint32_t k,
                                 const uint64_t *__restrict__ soff, uint8_t *__restrict__ dst) {
    for (uint32_t b = blockIdx.x; b < k; b += gridDim.x) {
        const uint8_t *src = chars + offsets[ids[b]];
        uint8_t *d = dst + soff[b];
        const uint64_t len = soff[b + 1] - soff[b];
        for (uint64_t i = threadIdx.x; i < len; i += blockDim.x) d[i] = src[i];
    }
}

// A group's candidate codes (local positions) to positions in the whole set.
__global__ void k_map_pairs(const uint64_t *__restrict__ pairs, uint64_t cnt,
                            const uint32_t *__restrict__ ids, uint64_t *__restrict__ out) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t c = pairs[e];
        out[e] = ((uint64_t)ids[c >> 32] << 32) | ids[(uint32_t)c];
    }
}

// ---- exhaustive pass over short strings
//
// The paper notes that LSH filtering suits long strings and that short ones
// may want another filter.  When K is large next to a string's length, random
// strings of such lengths are within K of each other by chance, and no
// embedding brings them into one bucket.  With ej_params.exact_len = S > 0,
// every pair of strings both no longer than S whose lengths differ by at most
// K (the length filter) joins the candidates.  In length order the short
// strings are a prefix of the permutation, and string i pairs with the run of
// following strings whose lengths are within K of its own.

__global__ void k_sorted_lengths(const uint32_t *__restrict__ len, const uint32_t *__restrict__ perm,
                                 uint32_t n, uint32_t *__restrict__ ls) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        ls[i] = len[perm[i]];
}

// first position in ls[lo, hi) (ascending) holding a value above x
__device__ inline uint32_t upper_bound_u32(const uint32_t *ls, uint32_t lo, uint32_t hi,
                                           uint64_t x) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)ls[mid] <= x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// *ns = the number of strings no longer than S (one thread)
__global__ void k_short_count(const uint32_t *__restrict__ ls, uint32_t n, uint32_t S,
                              uint64_t *__restrict__ ns) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *ns = upper_bound_u32(ls, 0, n, S);
}

// row[i] = the number of partners of short string i among the later ones
__global__ void k_short_rows(const uint32_t *__restrict__ ls, uint32_t ns, uint32_t K,
                             uint64_t *__restrict__ row) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x)
        row[i] = upper_bound_u32(ls, i + 1, ns, (uint64_t)ls[i] + K) - (i + 1);
}

// the P pairs, (lo << 32) | hi, row by row: output e belongs to the last row
// starting at or before e (start = exclusive prefix of the row counts)
__global__ void k_short_emit(const uint32_t *__restrict__ perm, const uint64_t *__restrict__ start,
                             uint32_t ns, uint64_t P, uint64_t *__restrict__ out) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < P;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = ns;  // first row starting after e, minus one
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (start[mid] <= e)
                lo = mid + 1;
            else
                hi = mid;
        }
        const uint32_t i = lo - 1;
        const uint32_t j = i + 1 + (uint32_t)(e - start[i]);
        const uint32_t a = perm[i], b = perm[j];
        out[e] = a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a;
    }
}

void check_params(const ej_params &p, uint32_t n) {
    if (p.r == 0 || p.z == 0 || p.m == 0) fail(EJ_EINVAL, "r, z and m must be positive");
    if (p.m > 64) fail(EJ_EINVAL, "m must be at most 64");
    if ((uint64_t)p.r * p.z > 4096) fail(EJ_EINVAL, "r*z must be at most 4096");
    if (n >= 0x80000000u) fail(EJ_EINVAL, "n must be below 2^31");
    if (p.K > 0x7FFFFFFFu) fail(EJ_EINVAL, "K must be below 2^31");
    if (verify_lanes_for(p.K) == 0) fail(EJ_EUNSUPPORTED, "K above 2046 is not supported");
    if (p.reserved != 0) fail(EJ_EINVAL, "ej_params.reserved must be 0");
}

struct StageTimer {
    ej_ctx *ctx;
    bool on;
    int idx = 0;
    explicit StageTimer(ej_ctx *c, bool o) : ctx(c), on(o) {}
    void mark() {
        if (on && idx < 8) EJ_HIP(hipEventRecord(ctx->timers.ev[idx++], ctx->stream));
    }
    float between(int a, int b) {
        if (!on || b >= idx) return 0.f;
        float ms = 0.f;
        EJ_HIP(hipEventElapsedTime(&ms, ctx->timers.ev[a], ctx->timers.ev[b]));
        return ms;
    }
};

}  // namespace

// Verification (A5) and output (A6) of a join whose candidates are known:
// distances, the pairs within K with their distances in host memory, and the
// timing fields.  walk_entries = the number of walks per seed (strings, or
// suffixes in EmbedJoin+).
void finish_join(ej_ctx *ctx, const Prep &pp, const uint64_t *d_offsets, const ej_params &p,
                 const Rand &rd, uint64_t walk_entries, const uint64_t *pairs, uint64_t cnt,
                 uint64_t raw, const uint32_t *order, StageTimer &tm, ej_result *out) {
    const uint32_t n = pp.n;
    out->n_candidates = cnt;
    out->n_raw = raw;
    int32_t *dist = ws<int32_t>(ctx, "j_dist", cnt);
    unsigned long long *d_cols = nullptr;
    if (tm.on) {
        d_cols = ws<unsigned long long>(ctx, "j_vcols", 1);
        EJ_HIP(hipMemsetAsync(d_cols, 0, 8, ctx->stream));
    }
    tm.mark();  // 4: the verification stage follows
    {
        // graph mode and the kernel timers apply to this verification only,
        // also when it fails
        struct Reset {
            ej_ctx *c;
            ~Reset() {
                c->timers.on = false;
                c->graph_on = false;
            }
        } reset{ctx};
        ctx->timers.on = tm.on;
        ctx->timers.nkv = 0;
        ctx->timers.more = 0;
        ctx->graph_on = (p.flags & EJ_FLAG_GRAPH) != 0 && ctx->tune.verify_mode >= 1;
        RowMasks masks;
        if (cnt)
            build_masks(ctx, pp.d_codes, d_offsets, pp.base, n, pp.total, pp.sigma, masks, "j");
        verify(ctx, pp.d_codes, d_offsets, pp.base, pp.sigma, pp.maxlen, masks, pairs, cnt, p.K,
               nullptr, dist, nullptr, nullptr, 0, 0, nullptr, d_cols, order, nullptr, pp.minlen);
    }
    tm.mark();  // 5
    uint64_t nout = 0;
    uint32_t *opairs = nullptr;
    int32_t *odist = nullptr;
    if (cnt) {
        uint32_t *flags = ws<uint32_t>(ctx, "j_oflags", cnt);
        uint32_t *pos = ws<uint32_t>(ctx, "j_opos", cnt);
        uint64_t *d_no = ws<uint64_t>(ctx, "j_nout", 1);
        hipLaunchKernelGGL(k_out_flags, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0, ctx->stream,
                           (const int32_t *)dist, cnt, (const uint64_t *)nullptr, p.K, flags);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u32(ctx, flags, pos, cnt, d_no);
        read_back(ctx, d_no, 8, &nout);
        // pairs then distances in one buffer: one copy to the host
        opairs = ws<uint32_t>(ctx, "j_out", 3 * nout);
        odist = (int32_t *)(opairs + 2 * nout);
        hipLaunchKernelGGL(k_out_compact, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0, ctx->stream,
                           (const uint64_t *)pairs, (const int32_t *)dist, cnt,
                           (const uint32_t *)flags, (const uint32_t *)pos, opairs, odist);
        EJ_CHECK_LAUNCH();
    }
    // host results go through the context's pinned staging buffer (grown when
    // too small): one DMA at full link speed instead of staged copies to
    // pageable memory.  With timing on, the verified columns and the walk
    // lengths J follow the results in the same buffer and share their
    // synchronisation.  EJ_FLAG_DEVICE_OUT leaves the results where the
    // compaction wrote them.
    const bool dev_out = (p.flags & EJ_FLAG_DEVICE_OUT) != 0;
    const size_t obytes = dev_out ? 0 : 12 * nout;
    const size_t xbytes = tm.on ? 8 + 4ull * p.r : 0;
    const size_t need = obytes + xbytes;
    if (need && ctx->pinned_out_bytes < need) {
        if (ctx->pinned_out) EJ_HIP(hipHostFree(ctx->pinned_out));
        ctx->pinned_out = nullptr;
        ctx->pinned_out_bytes = 0;
        const size_t want = std::max<size_t>(need + need / 4, 1 << 20);
        EJ_HIP(hipHostMalloc((void **)&ctx->pinned_out, want, hipHostMallocDefault));
        ctx->pinned_out_bytes = want;
    }
    out->count = nout;
    if (dev_out) {
        if (!opairs) {
            opairs = ws<uint32_t>(ctx, "j_out", 3);
            odist = (int32_t *)(opairs + 2 * nout);
        }
        out->pairs = opairs;
        out->dist = odist;
        out->on_device = 1;
    } else {
        out->pairs = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (nout ? nout : 1));
        out->dist = (int32_t *)malloc(sizeof(int32_t) * (nout ? nout : 1));
        if (!out->pairs || !out->dist) {
            free(out->pairs);
            free(out->dist);
            out->pairs = nullptr;
            out->dist = nullptr;
            fail(EJ_ENOMEM, "host allocation of the result failed");
        }
        if (nout)
            EJ_HIP(hipMemcpyAsync(ctx->pinned_out, opairs, obytes, hipMemcpyDeviceToHost,
                                  ctx->stream));
    }
    tm.mark();  // 6
    uint8_t *xp = ctx->pinned_out + obytes;
    if (xbytes) {
        if (cnt)
            EJ_HIP(hipMemcpyAsync(xp, d_cols, 8, hipMemcpyDeviceToHost, ctx->stream));
        if (rd.d_J)
            EJ_HIP(hipMemcpyAsync(xp + 8, rd.d_J, 4ull * p.r, hipMemcpyDeviceToHost, ctx->stream));
        else
            memset(xp + 8, 0, 4ull * p.r);
    }
    sync(ctx);
    if (nout && !dev_out) {
        memcpy(out->pairs, ctx->pinned_out, 8 * nout);
        memcpy(out->dist, ctx->pinned_out + 8 * nout, 4 * nout);
    }
    out->ms_prep = tm.between(0, 1);
    out->ms_embed = tm.between(1, 2);
    out->ms_bucket = tm.between(2, 3);
    out->ms_candidates = tm.between(3, 4);
    out->ms_verify = tm.between(4, 5);
    out->ms_output = tm.between(5, 6);
    if (tm.on) {
        std::vector<uint32_t> J(p.r);
        memcpy(J.data(), xp + 8, 4ull * p.r);
        uint64_t steps = 0;
        for (uint32_t x : J) steps += x;
        out->walk_steps = steps * walk_entries;
        if (cnt) memcpy(&out->verify_columns, xp, 8);
        float kms = 0.f;
        for (int i = 0; i + 1 < ctx->timers.nkv; i += 2) {
            float ms = 0.f;
            EJ_HIP(hipEventElapsedTime(&ms, ctx->timers.kv[i], ctx->timers.kv[i + 1]));
            kms += ms;
        }
        out->ms_verify_kernel = kms;
        out->verify_launches = (uint32_t)(ctx->timers.nkv / 2) + ctx->timers.more;
        out->verify_form = ctx->last_verify_form;
    }
}


// The candidates united with the short strings' pairs (exact_len = S > 0):
// returns the count of the sorted, distinct union at *out; with no short pair
// the candidates are returned as they are.
uint64_t add_short_pairs(ej_ctx *ctx, const Prep &pp, uint32_t K, uint32_t S,
                         const uint64_t *pairs, uint64_t cnt, const uint64_t **out) {
    *out = pairs;
    const uint32_t n = pp.n;
    if (S == 0 || n < 2) return cnt;
    uint32_t *ls = ws<uint32_t>(ctx, "sh_len", n);
    hipLaunchKernelGGL(k_sorted_lengths, dim3(grid_for(ctx, n, 256)), dim3(256), 0, ctx->stream,
                       (const uint32_t *)pp.d_len, (const uint32_t *)pp.d_perm, n, ls);
    EJ_CHECK_LAUNCH();
    uint64_t *d_tot = ws<uint64_t>(ctx, "sh_total", 2);
    hipLaunchKernelGGL(k_short_count, dim3(1), dim3(64), 0, ctx->stream, (const uint32_t *)ls, n,
                       S, d_tot);
    EJ_CHECK_LAUNCH();
    uint64_t ns = 0;
    read_back(ctx, d_tot, 8, &ns);
    if (ns < 2) return cnt;
    uint64_t *row = ws<uint64_t>(ctx, "sh_rows", ns);
    hipLaunchKernelGGL(k_short_rows, dim3(grid_for(ctx, ns, 256)), dim3(256), 0, ctx->stream,
                       (const uint32_t *)ls, (uint32_t)ns, K, row);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u64(ctx, row, row, ns, d_tot + 1);
    uint64_t P = 0;
    read_back(ctx, d_tot + 1, 8, &P);
    if (P == 0) return cnt;
    const uint64_t tot = cnt + P;
    if (tot >= 0xFFFFFFFFull)
        fail(EJ_EUNSUPPORTED, "more than 2^32 candidates with the short strings' pairs (" +
                                  std::to_string(tot) + ")");
    uint64_t *uni = ws<uint64_t>(ctx, "sh_union", tot);
    if (cnt)
        EJ_HIP(hipMemcpyAsync(uni, pairs, 8 * cnt, hipMemcpyDeviceToDevice, ctx->stream));
    hipLaunchKernelGGL(k_short_emit, dim3(grid_for(ctx, P, 256)), dim3(256), 0, ctx->stream,
                       (const uint32_t *)pp.d_perm, (const uint64_t *)row, (uint32_t)ns, P,
                       uni + cnt);
    EJ_CHECK_LAUNCH();
    uint64_t *sorted = ws<uint64_t>(ctx, "sh_sorted", tot);
    radix_sort_u64(ctx, uni, sorted, tot, 32 + std::max(1u, bits_for(n - 1)),
                   ctx->tune.radix_bits);
    uint64_t *u = nullptr;
    const uint64_t c = unique_sorted_pairs(ctx, sorted, tot, 32, &u, "sh");
    *out = u;
    return c;
}

// ---- the whole join as one graph (EJ_FLAG_GRAPH)
//
// After the preparation (whose read-back of the alphabet and lengths fixes
// the launch shapes) the join A1-A6 runs sized on the device: its candidate
// buffers have capacities taken from an earlier host-sized join of the same
// input shape, every kernel after a count reads the count from device memory,
// and only the counts come back at the end.  The first device-sized run of a
// shape allocates every buffer at its capacity, uncaptured; later runs with
// no buffer moved since are captured once into a graph, cached in the
// context, and replayed.  A count above its capacity (or a de-duplication
// group too large for the grouped form) voids the run: the join is redone
// host-sized and the capacities grow.

__global__ void k_join_counts(const uint64_t *__restrict__ c, uint64_t *__restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x < 4) out[threadIdx.x] = c[threadIdx.x];
}

std::string join_shape(ej_ctx *ctx, const Prep &pp, const uint8_t *d_chars,
                       const uint64_t *d_offsets, const ej_params &p) {
    const Tuning &t = ctx->tune;
    char key[512];
    snprintf(key, sizeof(key),
             "join %p %p %u %llu %llu %u %u %u %u %u %u %u %llu | %u %u %u %u %u %u %u %u %u %u "
             "%u %u %u %u",
             (const void *)d_chars, (const void *)d_offsets, pp.n, (unsigned long long)pp.base,
             (unsigned long long)pp.total, pp.sigma, pp.maxlen, pp.L, p.K, p.r, p.z, p.m,
             (unsigned long long)p.seed, t.verify_mode, t.verify_order, t.verify_split,
             t.verify_pass1_cols, t.verify_blocks_per_cu, t.verify_ring, t.verify_lds_budget,
             t.embed_lds_budget, t.radix_bits, t.bucket_key_bits, t.dedup_sort, t.raw_limit,
             t.verify_wpl, t.verify_len_order);
    return key;
}

// One device-sized join; returns false when its result is void (the caller
// then runs the host-sized join, which also sets the capacities).
bool join_graph(ej_ctx *ctx, const Prep &pp, const Rand &rd, const uint64_t *d_offsets,
                const ej_params &p, const std::string &shape, JoinCaps &caps, ej_result *out) {
    const uint32_t n = pp.n;
    const uint32_t T = p.r * p.z;
    const uint64_t raw_cap = caps.raw_cap, cnt_cap = caps.cnt_cap;
    // the multiplicity order schedules the two-pass, persistent and lane
    // forms (the grouped form orders by pattern itself)
    const bool want_order = ctx->tune.verify_mode <= 2 && ctx->tune.verify_order == 1;
    uint64_t *cnt_dev = ws<uint64_t>(ctx, "jg_counts", 4);
    uint64_t *cnt_out = ws<uint64_t>(ctx, "jg_counts_out", 4);
    // results: pairs [2 * cnt_cap] u32, then distances [cnt_cap] (looked up
    // here: a replay does not run the enqueue below)
    uint32_t *opairs = ws<uint32_t>(ctx, "j_out", 3 * cnt_cap);
    int32_t *odist = (int32_t *)(opairs + 2 * cnt_cap);
    auto enqueue = [&] {
        uint64_t *keys = ws<uint64_t>(ctx, "j_keys", (uint64_t)T * n);
        const uint32_t kb = bucket_key_bits(ctx, n, 0);
        uint32_t *bdk = nullptr, *bids = nullptr;
        bucket_inputs(ctx, (uint64_t)T * n, "j", &bdk, &bids);
        embed_keys(ctx, pp, rd, keys, nullptr, bdk, bids, 61u - kb);
        Buckets bk;
        bucket(ctx, keys, pp.d_len, pp.d_perm, n, T, kb, bk, "j", false, true, false);
        uint64_t *pairs = nullptr;
        uint32_t *order = nullptr;
        candidates_dev(ctx, keys, bk, pp.d_len, p.K, raw_cap, cnt_cap, want_order,
                       caps.sort_dedup || ctx->tune.dedup_sort != 0, cnt_dev, &pairs, &order,
                       "j");
        int32_t *dist = ws<int32_t>(ctx, "j_dist", cnt_cap);
        RowMasks masks;
        build_masks(ctx, pp.d_codes, d_offsets, pp.base, n, pp.total, pp.sigma, masks, "j");
        verify(ctx, pp.d_codes, d_offsets, pp.base, pp.sigma, pp.maxlen, masks, pairs, cnt_cap,
               p.K, nullptr, dist, nullptr, nullptr, 0, 0, nullptr, nullptr, order, cnt_dev + 1,
               pp.minlen);
        uint32_t *flags = ws<uint32_t>(ctx, "j_oflags", cnt_cap);
        uint32_t *pos = ws<uint32_t>(ctx, "j_opos", cnt_cap);
        hipLaunchKernelGGL(k_out_flags, dim3(grid_for(ctx, cnt_cap, 256)), dim3(256), 0,
                           ctx->stream, (const int32_t *)dist, cnt_cap,
                           (const uint64_t *)(cnt_dev + 1), p.K, flags);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u32(ctx, flags, pos, cnt_cap, cnt_dev + 3);
        hipLaunchKernelGGL(k_out_compact, dim3(grid_for(ctx, cnt_cap, 256)), dim3(256), 0,
                           ctx->stream, (const uint64_t *)pairs, (const int32_t *)dist, cnt_cap,
                           (const uint32_t *)flags, (const uint32_t *)pos, opairs, odist);
        EJ_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_join_counts, dim3(1), dim3(64), 0, ctx->stream,
                           (const uint64_t *)cnt_dev, cnt_out);
        EJ_CHECK_LAUNCH();
    };
    {
        // graph mode applies to this join only; the verification inside runs
        // as part of the outer launch sequence
        struct Reset {
            ej_ctx *c;
            ~Reset() { c->graph_on = false; }
        } reset{ctx};
        if (caps.gen == ctx->ws_gen) {
            char g[96];
            snprintf(g, sizeof(g), " | %llu %llu %llu", (unsigned long long)raw_cap,
                     (unsigned long long)cnt_cap, (unsigned long long)caps.gen);
            ctx->graph_on = true;
            out->graph = 2;
            try {
                run_captured(ctx, shape + g, enqueue);
            } catch (const Error &) {
                // the capture failed (an operation that cannot be captured):
                // this shape runs host-sized from now on
                (void)hipGetLastError();
                caps.no_graph = true;
                out->graph = 0;
                return false;
            }
        } else {
            // every buffer at its capacity, uncaptured: a later join of this
            // shape can be captured without allocating
            ctx->graph_on = false;
            enqueue();
            caps.gen = ctx->ws_gen;
            out->graph = 1;
        }
    }
    uint64_t c[4] = {0, 0, 0, 0};  // raw, distinct, overflow, output
    read_back(ctx, cnt_out, sizeof(c), c);
    if (c[2] != 0 || c[0] > raw_cap || c[1] > cnt_cap) out->graph = 0;
    if (c[2] != 0) {
        // a group too large for the grouped de-duplication: sort instead
        caps.sort_dedup = true;
        caps.gen = ~0ull;
        return false;
    }
    if (c[0] > raw_cap || c[1] > cnt_cap) {
        caps.raw_cap = std::max(raw_cap, c[0] + c[0] / 8 + 4096);
        caps.cnt_cap = std::max(cnt_cap, c[1] + c[1] / 8 + 4096);
        caps.gen = ~0ull;
        return false;
    }
    const uint64_t nout = c[3];
    out->n_raw = c[0];
    out->n_candidates = c[1];
    out->count = nout;
    out->sigma = pp.sigma;
    out->L = pp.L;
    if (p.flags & EJ_FLAG_DEVICE_OUT) {
        out->pairs = opairs;
        out->dist = odist;
        out->on_device = 1;
        return true;
    }
    const size_t need = 12 * nout;
    if (need && ctx->pinned_out_bytes < need) {
        if (ctx->pinned_out) EJ_HIP(hipHostFree(ctx->pinned_out));
        ctx->pinned_out = nullptr;
        ctx->pinned_out_bytes = 0;
        const size_t want = std::max<size_t>(need + need / 4, 1 << 20);
        EJ_HIP(hipHostMalloc((void **)&ctx->pinned_out, want, hipHostMallocDefault));
        ctx->pinned_out_bytes = want;
    }
    out->pairs = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (nout ? nout : 1));
    out->dist = (int32_t *)malloc(sizeof(int32_t) * (nout ? nout : 1));
    if (!out->pairs || !out->dist) {
        free(out->pairs);
        free(out->dist);
        out->pairs = nullptr;
        out->dist = nullptr;
        fail(EJ_ENOMEM, "host allocation of the result failed");
    }
    if (nout) {
        EJ_HIP(hipMemcpyAsync(ctx->pinned_out, opairs, 8 * nout, hipMemcpyDeviceToHost,
                              ctx->stream));
        EJ_HIP(hipMemcpyAsync(ctx->pinned_out + 8 * nout, odist, 4 * nout,
                              hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
        memcpy(out->pairs, ctx->pinned_out, 8 * nout);
        memcpy(out->dist, ctx->pinned_out + 8 * nout, 4 * nout);
    }
    return true;
}

// The whole path on device-resident strings.
void join_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                 const ej_params &p, ej_result *out) {
    check_params(p, n);
    memset(out, 0, sizeof(*out));
    StageTimer tm(ctx, (p.flags & EJ_FLAG_TIMING) != 0);
    tm.mark();  // 0
    Prep pp;
    prepare(ctx, d_chars, d_offsets, n, p.L, pp, "j");
    out->sigma = pp.sigma;
    out->L = pp.L;
    Rand rd;
    draw_randomness(ctx, p, pp.L, pp.sigma, rd, "j");
    const uint32_t T = p.r * p.z;
    // the whole join as one graph: not with stage timing (its events go
    // between the stages) nor with the short-string pass
    const bool as_graph = (p.flags & EJ_FLAG_GRAPH) != 0 && (p.flags & EJ_FLAG_TIMING) == 0 &&
                          p.exact_len == 0 && n >= 2;
    std::string shape;
    if (as_graph) {
        shape = join_shape(ctx, pp, d_chars, d_offsets, p);
        auto it = ctx->join_caps.find(shape);
        if (it != ctx->join_caps.end() && !it->second.no_graph &&
            join_graph(ctx, pp, rd, d_offsets, p, shape, it->second, out))
            return;
    }
    uint64_t *keys = ws<uint64_t>(ctx, "j_keys", (uint64_t)T * n);
    tm.mark();  // 1: the walk kernel alone follows
    // the walk also writes the bucketing sort's input (top key bits and
    // string indexes in length order)
    const uint32_t kb = bucket_key_bits(ctx, n, 0);
    uint32_t *bdk = nullptr, *bids = nullptr;
    bucket_inputs(ctx, (uint64_t)T * n, "j", &bdk, &bids);
    embed_keys(ctx, pp, rd, keys, nullptr, bdk, bids, 61u - kb);
    tm.mark();  // 2
    Buckets bk;
    bucket(ctx, keys, pp.d_len, pp.d_perm, n, T, kb, bk, "j", false, true, false);
    tm.mark();  // 3
    uint64_t *pairs = nullptr;
    uint64_t raw = 0;
    uint32_t *order = nullptr;
    // the multiplicity order schedules the two-pass, persistent and lane
    // forms (the grouped form orders by pattern itself)
    const bool want_order = ctx->tune.verify_mode <= 2 && ctx->tune.verify_order == 1;
    uint64_t cnt = candidates(ctx, keys, bk, pp.d_len, p.K, &pairs, &raw, "j",
                              want_order && !p.exact_len ? &order : nullptr);
    const uint64_t *cp = pairs;
    cnt = add_short_pairs(ctx, pp, p.K, p.exact_len, pairs, cnt, &cp);
    finish_join(ctx, pp, d_offsets, p, rd, n, cp, cnt, raw, order, tm, out);
    if (as_graph) {
        // capacities for the next join of this shape, with headroom
        if (ctx->join_caps.size() >= 64) ctx->join_caps.clear();
        JoinCaps &c = ctx->join_caps[shape];
        c.raw_cap = std::max(c.raw_cap, raw + raw / 16 + 4096);
        c.cnt_cap = std::max(c.cnt_cap, cnt + cnt / 16 + 4096);
        c.sort_dedup = c.sort_dedup || ctx->last_dedup_sorted;
        // capacities at 2^32 or more (or raw pairs past the one-sort limit,
        // which the host-sized join takes in passes): this shape stays
        // host-sized
        if (c.raw_cap >= 0xFFFFFFFFull || c.cnt_cap >= 0xFFFFFFFFull ||
            (ctx->tune.raw_limit && raw > ctx->tune.raw_limit))
            c.no_graph = true;
    }
}

// Suffix step and threshold of EmbedJoin+ (Section 5): delta = 0 selects
// floor(sqrt(ceil(average length))), at least 1 (the paper sets delta to about
// the square root of the average length); T = 0 selects 2 when a string has
// more than one suffix (ceil(K / delta) > 1), else 1.
void plus_params(uint64_t total, uint32_t n, uint32_t K, uint32_t &delta, uint32_t &T,
                 uint32_t &kappa) {
    if (delta == 0) {
        const uint64_t avg = n ? (total + n - 1) / n : 0;
        uint64_t d = 0;
        while ((d + 1) * (d + 1) <= avg) d++;
        delta = (uint32_t)std::max<uint64_t>(d, 1);
    }
    kappa = std::max<uint32_t>(1u, (uint32_t)((K + (uint64_t)delta - 1) / delta));
    if (T == 0) T = kappa > 1 ? 2u : 1u;
}

// EmbedJoin+ (Algorithms 4-5) on device-resident strings: every string's
// kappa = ceil(K / delta) suffixes are walked and hashed as entries of their
// own, bucketed by (key bits, whole-string length, entry), and a pair of
// strings is a candidate when one (suffix, suffix) tuple is found by at least
// T tables; verification and output are the join's.
void join_plus_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                      const ej_params &p, uint32_t delta, uint32_t T, ej_result *out) {
    check_params(p, n);
    memset(out, 0, sizeof(*out));
    StageTimer tm(ctx, (p.flags & EJ_FLAG_TIMING) != 0);
    tm.mark();  // 0
    Prep pp;
    prepare(ctx, d_chars, d_offsets, n, p.L, pp, "j");
    out->sigma = pp.sigma;
    out->L = pp.L;
    uint32_t kappa = 1;
    plus_params(pp.total, n, p.K, delta, T, kappa);
    const uint64_t ne64 = (uint64_t)n * kappa;
    const uint32_t NT = p.r * p.z;
    if (ne64 * NT >= 0xFFFFFFFFull)
        fail(EJ_EUNSUPPORTED, "r*z*n*ceil(K/delta) must stay below 2^32");
    const uint32_t ne = (uint32_t)ne64;
    Rand rd;
    draw_randomness(ctx, p, pp.L, pp.sigma, rd, "j");
    // the suffix entries, as a string set of their own over the same codes
    Prep ps = pp;
    ps.n = ne;
    uint64_t *sstart = ws<uint64_t>(ctx, "p_sstart", ne64 + 1);
    uint32_t *slen = ws<uint32_t>(ctx, "p_slen", ne64 + 1);
    uint32_t *flen = ws<uint32_t>(ctx, "p_flen", ne64 + 1);
    uint32_t *eperm = ws<uint32_t>(ctx, "p_eperm", ne64 + 1);
    if (ne) {
        hipLaunchKernelGGL(k_suffix_entries, dim3(grid_for(ctx, ne64, 256)), dim3(256), 0,
                           ctx->stream, d_offsets, (const uint32_t *)pp.d_len, n, kappa, delta,
                           sstart, slen, flen);
        EJ_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_entry_perm, dim3(grid_for(ctx, ne64, 256)), dim3(256), 0,
                           ctx->stream, (const uint32_t *)pp.d_perm, n, kappa, eperm);
        EJ_CHECK_LAUNCH();
    }
    ps.d_offsets = sstart;
    ps.d_len = slen;
    ps.d_perm = eperm;
    uint64_t *keys = ws<uint64_t>(ctx, "p_keys", ne64 * NT);
    tm.mark();  // 1
    embed_keys(ctx, ps, rd, keys, nullptr);
    tm.mark();  // 2
    const uint32_t kb = bucket_key_bits(ctx, ne, 0);
    Buckets bk;
    bucket(ctx, keys, flen, eperm, ne, NT, kb, bk, "p", false, false, false);
    tm.mark();  // 3
    uint64_t *pairs = nullptr;
    uint64_t raw = 0;
    uint64_t cnt = candidates_plus(ctx, keys, bk, flen, p.K, n, kappa, T, &pairs, &raw, "p");
    const uint64_t *cp = pairs;
    cnt = add_short_pairs(ctx, pp, p.K, p.exact_len, pairs, cnt, &cp);
    finish_join(ctx, pp, d_offsets, p, rd, ne64, cp, cnt, raw, nullptr, tm, out);
}

void check_pairs(ej_ctx *ctx, const uint64_t *d_pairs, uint64_t count, uint32_t n_a,
                 uint32_t n_b) {
    if (!count) return;
    uint32_t *d_bad = ws<uint32_t>(ctx, "v_bad", 1);
    EJ_HIP(hipMemsetAsync(d_bad, 0, 4, ctx->stream));
    hipLaunchKernelGGL(k_check_pairs, dim3(grid_for(ctx, count, 256)), dim3(256), 0, ctx->stream,
                       d_pairs, count, n_a, n_b, d_bad);
    EJ_CHECK_LAUNCH();
    uint32_t bad = 0;
    read_back(ctx, d_bad, 4, &bad);
    if (bad) fail(EJ_EINVAL, "a pair refers to a position >= n");
}

// Length groups of the grouping alternative to truncation (Section 4.1):
// group g holds the strings of length in (gK, (g+2)K] (group 0 also the
// empty ones; one group per length when K = 0), g < max(1, ceil(N/K) - 1).
inline bool in_group(uint64_t len, uint64_t g, uint32_t K) {
    if (K == 0) return len == g;
    if (g == 0 && len == 0) return true;
    return len > g * K && len <= (g + 2) * K;
}

// EmbedJoin with grouping instead of truncation: the front end (A0-A4) runs
// on each group's strings as a set of its own (its alphabet; walks of
// L = 3 x its longest string, or the caller's L), the groups' candidates are
// mapped to positions in the whole set and de-duplicated, and the union is
// verified once (a pair found by two groups is verified once, not twice).
void join_grouped_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                         uint32_t n, const ej_params &p, ej_result *out) {
    check_params(p, n);
    memset(out, 0, sizeof(*out));
    StageTimer tm(ctx, (p.flags & EJ_FLAG_TIMING) != 0);
    tm.mark();  // 0
    Prep pp;
    prepare(ctx, d_chars, d_offsets, n, 0, pp, "j");
    out->sigma = pp.sigma;
    std::vector<uint32_t> len(n);
    if (n) {
        EJ_HIP(hipMemcpyAsync(len.data(), pp.d_len, 4ull * n, hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
    }
    const uint64_t N = pp.maxlen;
    const uint64_t G = p.K == 0 ? N + 1 : std::max<uint64_t>(1, (N + p.K - 1) / p.K - 1);
    const uint32_t NT = p.r * p.z;
    tm.mark();  // 1: the groups' front ends follow
    // the grouping's own buffers ("grp_*") must not share a name with the
    // stage buffers of the groups' front ends (tag "g": "g_ids", "g_keys" ...),
    // which grow -- and so free -- their buffers as the groups change size
    uint64_t raw = 0, ucount = 0, ucap = 0;
    uint64_t *uni = nullptr;
    int which = 0;  // the union grows into two alternating buffers
    std::vector<uint32_t> ids;
    std::vector<uint64_t> soff;
    for (uint64_t g = 0; g < G; g++) {
        ids.clear();
        soff.assign(1, 0);
        uint64_t Ng = 0;
        for (uint32_t i = 0; i < n; i++)
            if (in_group(len[i], g, p.K)) {
                ids.push_back(i);
                soff.push_back(soff.back() + len[i]);
                Ng = std::max<uint64_t>(Ng, len[i]);
            }
        const uint32_t k = (uint32_t)ids.size();
        if (k < 2) continue;
        uint32_t *d_ids = ws<uint32_t>(ctx, "grp_ids", k);
        uint64_t *d_soff = ws<uint64_t>(ctx, "grp_soff", (uint64_t)k + 1);
        uint8_t *d_sub = ws<uint8_t>(ctx, "grp_chars", soff.back() + 16);
        EJ_HIP(hipMemcpyAsync(d_ids, ids.data(), 4ull * k, hipMemcpyHostToDevice, ctx->stream));
        EJ_HIP(hipMemcpyAsync(d_soff, soff.data(), 8ull * (k + 1), hipMemcpyHostToDevice,
                              ctx->stream));
        hipLaunchKernelGGL(k_gather_strings, dim3(std::min<uint32_t>(k, 65535)), dim3(256), 0,
                           ctx->stream, d_chars, d_offsets, (const uint32_t *)d_ids, k,
                           (const uint64_t *)d_soff, d_sub);
        EJ_CHECK_LAUNCH();
        const uint64_t Lg = p.L ? p.L : std::max<uint64_t>(1, 3 * Ng);
        if (Lg > 0x7FFFFFFFull) fail(EJ_EUNSUPPORTED, "group walk length too large");
        Prep pg;
        prepare(ctx, d_sub, d_soff, k, (uint32_t)Lg, pg, "g");
        Rand rd;
        draw_randomness(ctx, p, pg.L, pg.sigma, rd, "g");
        uint64_t *keys = ws<uint64_t>(ctx, "g_keys", (uint64_t)NT * k);
        const uint32_t kb = bucket_key_bits(ctx, k, 0);
        uint32_t *bdk = nullptr, *bids = nullptr;
        bucket_inputs(ctx, (uint64_t)NT * k, "g", &bdk, &bids);
        embed_keys(ctx, pg, rd, keys, nullptr, bdk, bids, 61u - kb);
        Buckets bk;
        bucket(ctx, keys, pg.d_len, pg.d_perm, k, NT, kb, bk, "g", false, true, false);
        uint64_t *gp = nullptr;
        uint64_t graw = 0;
        const uint64_t gc = candidates(ctx, keys, bk, pg.d_len, p.K, &gp, &graw, "g");
        raw += graw;
        if (!gc) continue;
        if (ucount + gc > ucap) {
            const uint64_t cap = std::max<uint64_t>(2 * ucap, ucount + gc);
            uint64_t *nb = ws<uint64_t>(ctx, which ? "grp_unionA" : "grp_unionB", cap);
            if (ucount)
                EJ_HIP(hipMemcpyAsync(nb, uni, 8 * ucount, hipMemcpyDeviceToDevice, ctx->stream));
            uni = nb;
            ucap = cap;
            which ^= 1;
        }
        hipLaunchKernelGGL(k_map_pairs, dim3(grid_for(ctx, gc, 256)), dim3(256), 0, ctx->stream,
                           (const uint64_t *)gp, gc, (const uint32_t *)d_ids, uni + ucount);
        EJ_CHECK_LAUNCH();
        ucount += gc;
        sync(ctx);  // the host vectors of this group are reused by the next
    }
    out->L = p.L;  // 0: each group walked 3 x its longest string
    tm.mark();  // 2
    tm.mark();  // 3: the union's de-duplication follows
    uint64_t *pairs = nullptr;
    uint64_t cnt = 0;
    if (ucount) {
        uint64_t *sorted = ws<uint64_t>(ctx, "grp_union_sorted", ucount);
        radix_sort_u64(ctx, uni, sorted, ucount, 32 + std::max(1u, bits_for(n - 1)),
                       ctx->tune.radix_bits);
        cnt = unique_sorted_pairs(ctx, sorted, ucount, 32, &pairs, "grp");
    }
    const uint64_t *cp = pairs;
    cnt = add_short_pairs(ctx, pp, p.K, p.exact_len, pairs, cnt, &cp);
    Rand none;
    finish_join(ctx, pp, d_offsets, p, none, 0, cp, cnt, raw, nullptr, tm, out);
}

// ej_verify's work: preparation of the strings, their match masks and the
// verification kernels, on the context's workspace.
void verify_entry(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                  const uint64_t *d_pairs, uint64_t count, uint32_t K, const uint32_t *d_Kq,
                  int32_t *d_dist) {
    if (!d_Kq && verify_lanes_for(K) == 0) fail(EJ_EUNSUPPORTED, "K above 2046 is not supported");
    Prep pp;
    prepare(ctx, d_chars, d_offsets, n, 0, pp, "v", nullptr, 0, 0, false);
    check_pairs(ctx, d_pairs, count, n, n);
    RowMasks masks;
    if (count)
        build_masks(ctx, pp.d_codes, d_offsets, pp.base, n, pp.total, pp.sigma, masks, "v");
    verify(ctx, pp.d_codes, d_offsets, pp.base, pp.sigma, pp.maxlen, masks, d_pairs, count, K,
           d_Kq, d_dist, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr, pp.minlen);
    sync(ctx);
}

}  // namespace ej

using namespace ej;

namespace {

struct HostInput {
    uint8_t *d_chars = nullptr;
    uint64_t *d_offsets = nullptr;
};

// Copies host strings into the context workspace (offsets rebased to 0).
HostInput upload(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                 const char *tag) {
    if (!offsets) fail(EJ_EINVAL, "null offsets");
    for (uint32_t i = 0; i < n; i++)
        if (offsets[i + 1] < offsets[i]) fail(EJ_EINVAL, "offsets are not non-decreasing");
    uint64_t base = offsets[0], total = offsets[n] - offsets[0];
    if (total && !strings) fail(EJ_EINVAL, "null strings");
    HostInput h;
    std::string t(tag);
    h.d_chars = ws<uint8_t>(ctx, t + "_hchars", total + 16);
    h.d_offsets = ws<uint64_t>(ctx, t + "_hoffsets", (uint64_t)n + 1);
    std::vector<uint64_t> rebased(offsets, offsets + n + 1);
    for (auto &o : rebased) o -= base;
    if (total)
        EJ_HIP(hipMemcpyAsync(h.d_chars, strings + base, total, hipMemcpyHostToDevice, ctx->stream));
    EJ_HIP(hipMemcpyAsync(h.d_offsets, rebased.data(), sizeof(uint64_t) * (n + 1),
                          hipMemcpyHostToDevice, ctx->stream));
    sync(ctx);  // the rebased vector is pageable and local
    return h;
}

}  // namespace

extern "C" {

ej_status ej_join_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                         const ej_params *p, ej_result *out) {
    if (!p || !out || !d_offsets) return EJ_EINVAL;
    return run_guarded(ctx, [&] { join_device(ctx, d_chars, d_offsets, n, *p, out); });
}

ej_status ej_join_plus_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                              uint32_t n, const ej_params *p, uint32_t delta, uint32_t T,
                              ej_result *out) {
    if (!p || !out || !d_offsets) return EJ_EINVAL;
    return run_guarded(ctx, [&] { join_plus_device(ctx, d_chars, d_offsets, n, *p, delta, T, out); });
}

ej_status ej_join_plus(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                       const ej_params *p, uint32_t delta, uint32_t T, ej_result *out) {
    if (!p || !out) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        check_params(*p, n);
        HostInput h = upload(ctx, strings, offsets, n, "in");
        join_plus_device(ctx, h.d_chars, h.d_offsets, n, *p, delta, T, out);
    });
}

ej_status ej_join_grouped_device(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                                 uint32_t n, const ej_params *p, ej_result *out) {
    if (!p || !out || !d_offsets) return EJ_EINVAL;
    return run_guarded(ctx, [&] { join_grouped_device(ctx, d_chars, d_offsets, n, *p, out); });
}

ej_status ej_join_grouped(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets,
                          uint32_t n, const ej_params *p, ej_result *out) {
    if (!p || !out) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        check_params(*p, n);
        HostInput h = upload(ctx, strings, offsets, n, "in");
        join_grouped_device(ctx, h.d_chars, h.d_offsets, n, *p, out);
    });
}

ej_status ej_autotune(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                      const ej_params *p, uint32_t reps, float *best_ms) {
    if (!p || !d_offsets) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        check_params(*p, n);
        if (reps == 0) reps = 1;
        ej_params q = *p;
        q.flags &= ~(uint32_t)EJ_FLAG_TIMING;
        auto trial = [&]() {
            double best = 1e30;
            for (uint32_t i = 0; i < reps; i++) {
                ej_result res;
                memset(&res, 0, sizeof(res));
                auto t0 = std::chrono::steady_clock::now();
                try {
                    join_device(ctx, d_chars, d_offsets, n, q, &res);
                } catch (...) {
                    ej_result_free(&res);
                    throw;
                }
                auto t1 = std::chrono::steady_clock::now();
                ej_result_free(&res);
                best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
            }
            return best;
        };
        // a setting the kernels cannot run (say, the whole-pattern mask layout
        // of strings too long for LDS) scores as infinitely slow; the stream
        // is drained and the error cleared before the next trial
        auto trial_or_inf = [&]() {
            try {
                return trial();
            } catch (const Error &) {
                (void)hipStreamSynchronize(ctx->stream);
                (void)hipGetLastError();
                return 1e300;
            }
        };
        trial();  // warm the workspace (the starting knobs must run)
        double cur = trial();
        // coordinate descent, one knob at a time, in order of expected effect
        // which verification forms a knob affects, as a bit mask of verify_mode
        // values (1: two-pass, 2: persistent tiles, 4: lanes, 8: grouped by
        // pattern)
        struct Knob {
            uint32_t Tuning::*field;
            std::vector<uint32_t> vals;
            uint32_t modes;
        };
        const Knob knobs[] = {
            {&Tuning::verify_mode, {0, 1, 2, 3}, 15},
            {&Tuning::verify_split, {0, 1, 2, 4, 8}, 4},
            {&Tuning::verify_wpl, {1, 2, 4}, 1},
            {&Tuning::verify_len_order, {1, 0}, 1},
            {&Tuning::verify_pass1_cols, {512, 1024, 2048, 0}, 1},
            {&Tuning::verify_blocks_per_cu, {8, 16, 32, 64}, 1},
            {&Tuning::verify_blocks_per_cu, {2, 4, 8, 16, 32}, 12},
            {&Tuning::verify_order, {1, 0}, 7},
            {&Tuning::verify_ring, {1, 0}, 3},
            {&Tuning::radix_bits, {6, 7, 8, 11}, 15},
            {&Tuning::bucket_key_bits, {0, 32}, 15},
            {&Tuning::dedup_sort, {0, 1}, 15},
        };
        for (const Knob &k : knobs) {
            if (!((k.modes >> ctx->tune.verify_mode) & 1u)) continue;
            const uint32_t start = ctx->tune.*(k.field);
            uint32_t best_v = start;
            for (uint32_t v : k.vals) {
                if (v == start) continue;
                ctx->tune.*(k.field) = v;
                const double t = trial_or_inf();
                if (t < cur) {
                    cur = t;
                    best_v = v;
                }
            }
            ctx->tune.*(k.field) = best_v;
        }
        if (best_ms) *best_ms = (float)cur;
    });
}

ej_status ej_join_ex(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                     const ej_params *p, ej_result *out) {
    if (!p || !out) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        check_params(*p, n);
        HostInput h = upload(ctx, strings, offsets, n, "in");
        join_device(ctx, h.d_chars, h.d_offsets, n, *p, out);
    });
}

ej_status ej_join(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                  uint32_t K, uint32_t r, uint32_t z, uint32_t m, uint64_t seed, ej_result *out) {
    ej_params p;
    memset(&p, 0, sizeof(p));
    p.K = K;
    p.r = r;
    p.z = z;
    p.m = m;
    p.seed = seed;
    return ej_join_ex(ctx, strings, offsets, n, &p, out);
}

void ej_result_free(ej_result *res) {
    if (!res) return;
    if (!res->on_device) {
        free(res->pairs);
        free(res->dist);
    }
    res->pairs = nullptr;
    res->dist = nullptr;
    res->count = 0;
}

ej_status ej_embed(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                   const ej_params *p, uint8_t *d_sig, uint64_t *d_keys, uint32_t *L_used,
                   uint32_t *sigma) {
    if (!p || !d_offsets || (n && !d_keys)) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        ej_params q = *p;
        q.K = 0;
        check_params(q, n);
        Prep pp;
        prepare(ctx, d_chars, d_offsets, n, p->L, pp, "e");
        Rand rd;
        draw_randomness(ctx, *p, pp.L, pp.sigma, rd, "e");
        embed_keys(ctx, pp, rd, d_keys, d_sig);
        sync(ctx);
        if (L_used) *L_used = pp.L;
        if (sigma) *sigma = pp.sigma;
    });
}

ej_status ej_lsh_bucket(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_len, uint32_t n,
                        uint32_t ntables, uint32_t key_bits, uint32_t *d_ids_sorted,
                        uint32_t *d_group_start, uint64_t *ngroups) {
    if (!ngroups || (n && (!d_keys || !d_len || !d_ids_sorted || !d_group_start)))
        return EJ_EINVAL;
    if (key_bits > 32) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        // length order of the strings, as Algorithm 2 sorts them
        uint32_t maxlen = 0;
        uint32_t *perm = ws<uint32_t>(ctx, "b_perm", n + 1);
        if (n) {
            uint32_t *d_mx = ws<uint32_t>(ctx, "b_maxlen", 1);
            EJ_HIP(hipMemsetAsync(d_mx, 0, 4, ctx->stream));
            hipLaunchKernelGGL(k_max_len_shim, dim3(grid_for(ctx, n, 256)), dim3(256), 0, ctx->stream,
                               d_len, n, d_mx);
            EJ_CHECK_LAUNCH();
            read_back(ctx, d_mx, 4, &maxlen);
            uint32_t *lk = ws<uint32_t>(ctx, "b_lk", n), *lk2 = ws<uint32_t>(ctx, "b_lk2", n);
            uint32_t *iota = ws<uint32_t>(ctx, "b_iota", n);
            EJ_HIP(hipMemcpyAsync(lk, d_len, 4ull * n, hipMemcpyDeviceToDevice, ctx->stream));
            hipLaunchKernelGGL(k_iota_shim, dim3(grid_for(ctx, n, 256)), dim3(256), 0, ctx->stream,
                               iota, n);
            EJ_CHECK_LAUNCH();
            radix_sort_u32(ctx, lk, iota, lk2, perm, 1, n, bits_for(maxlen), 8);
        }
        Buckets bk;
        if (key_bits == 0)
            bucket_exact(ctx, d_keys, perm, n, ntables, bk, "b");
        else
            bucket(ctx, d_keys, d_len, perm, n, ntables, key_bits, bk, "b", true);
        uint64_t tot = (uint64_t)ntables * n;
        if (tot)
            EJ_HIP(hipMemcpyAsync(d_ids_sorted, bk.d_ids, 4 * tot, hipMemcpyDeviceToDevice,
                                  ctx->stream));
        EJ_HIP(hipMemcpyAsync(d_group_start, bk.d_gstart, 4 * (bk.ngroups + 1),
                              hipMemcpyDeviceToDevice, ctx->stream));
        sync(ctx);
        *ngroups = bk.ngroups;
    });
}

ej_status ej_candidates(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_ids_sorted,
                        const uint32_t *d_group_start, uint64_t ngroups, const uint32_t *d_len,
                        uint32_t n, uint32_t ntables, uint32_t K, uint64_t *d_pairs,
                        uint64_t capacity, uint64_t *count, uint64_t *n_raw) {
    if (!count) return EJ_EINVAL;
    if ((uint64_t)ntables * n && (!d_keys || !d_ids_sorted || !d_group_start || !d_len))
        return EJ_EINVAL;
    ej_status st = run_guarded(ctx, [&] {
        Buckets bk;
        bk.T = ntables;
        bk.n = n;
        bk.ngroups = ngroups;
        bk.d_ids = const_cast<uint32_t *>(d_ids_sorted);
        bk.d_gstart = const_cast<uint32_t *>(d_group_start);
        uint64_t tot = (uint64_t)ntables * n;
        if ((ngroups == 0) != (tot == 0) || ngroups > tot) fail(EJ_EINVAL, "inconsistent group count");
        if (ngroups) {
            uint32_t *d_bad = ws<uint32_t>(ctx, "c_bad", 1);
            EJ_HIP(hipMemsetAsync(d_bad, 0, 4, ctx->stream));
            hipLaunchKernelGGL(k_check_groups, dim3(grid_for(ctx, ngroups, 256)), dim3(256), 0,
                               ctx->stream, d_group_start, ngroups, tot, d_bad);
            EJ_CHECK_LAUNCH();
            uint32_t bad = 0;
            read_back(ctx, d_bad, 4, &bad);
            if (bad) fail(EJ_EINVAL, "group starts are not increasing from 0 to ntables*n");
        }
        bk.d_gid = ws<uint32_t>(ctx, "c_gid", tot + 1);
        if (ngroups)
            hipLaunchKernelGGL(k_gid_from_starts, dim3(grid_for(ctx, ngroups, 256)), dim3(256), 0,
                               ctx->stream, d_group_start, ngroups, bk.d_gid);
        EJ_CHECK_LAUNCH();
        uint64_t *pairs = nullptr;
        uint64_t raw = 0;
        uint64_t cnt = candidates(ctx, d_keys, bk, d_len, K, &pairs, &raw, "c");
        *count = cnt;
        if (n_raw) *n_raw = raw;
        if (cnt > capacity) fail(EJ_ECAPACITY, "candidate buffer too small");
        if (cnt)
            EJ_HIP(hipMemcpyAsync(d_pairs, pairs, 8 * cnt, hipMemcpyDeviceToDevice, ctx->stream));
        sync(ctx);
    });
    return st;
}

ej_status ej_verify(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
                    const uint64_t *d_pairs, uint64_t count, uint32_t K, const uint32_t *d_Kq,
                    int32_t *d_dist) {
    if (!d_offsets || (count && (!d_pairs || !d_dist))) return EJ_EINVAL;
    return run_guarded(ctx, [&] { verify_entry(ctx, d_chars, d_offsets, n, d_pairs, count, K, d_Kq, d_dist); });
}

ej_status ej_verify_static(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets,
                           uint32_t n, const uint64_t *d_pairs, uint64_t count, uint32_t K,
                           const uint32_t *d_Kq, int32_t *d_dist) {
    if (!d_offsets || (count && (!d_pairs || !d_dist))) return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        uint8_t *base = (uint8_t *)static_scratch(ctx);
        // sizes known before anything is enqueued: lengths and mask offsets
        if (24ull * ((uint64_t)n + 1) + 4096 > STATIC_SCRATCH_BYTES)
            fail(EJ_ENOMEM, std::to_string(n) + " strings exceed the " +
                                std::to_string(STATIC_SCRATCH_BYTES >> 20) +
                                " MiB of static scratch");
        // every workspace request of this call is carved from the scratch
        // array; the two-pass form (saved state per pair) becomes the
        // persistent form, which needs only a counter
        struct Scope {
            ej_ctx *c;
            uint32_t mode;
            ~Scope() {
                c->arena = Arena();
                c->tune.verify_mode = mode;
            }
        } scope{ctx, ctx->tune.verify_mode};
        ctx->arena.base = base;
        ctx->arena.cap = STATIC_SCRATCH_BYTES;
        if (ctx->tune.verify_mode == 0) ctx->tune.verify_mode = 1;
        verify_entry(ctx, d_chars, d_offsets, n, d_pairs, count, K, d_Kq, d_dist);
    });
}

}  // extern "C"
