// Stages A3-A4: bucketing and candidate pairs.
//
// Algorithm 3 walks the strings in length order, probes the bucket of each
// table, adds (s, s_i) for every stored s with |s_i| - |s| <= K, evicts the
// others (they can never pair with a later, longer string) and de-duplicates
// pairs found by several tables.  Its result is the set of pairs that share a
// bucket in some table and differ in length by at most K.  The GPU computes
// that set directly:
//   1. every table is sorted by (top key bits, length, position) with a
//      stable segmented LSD radix sort whose input is already in (length,
//      position) order, so each group of equal top bits lists its strings by
//      length;
//   2. for each entry p of a group, the partners are the following entries q
//      of the group with len[q] <= len[p] + K (a contiguous window, the
//      sliding window of the paper) whose full 61-bit key equals p's;
//   3. the pairs are counted, scanned and emitted at deterministic offsets,
//      then sorted and de-duplicated across tables.
#include <algorithm>
#include <type_traits>

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

__global__ void k_bucket_gather(const uint64_t *__restrict__ keys,
                                const uint32_t *__restrict__ perm, uint32_t n, uint64_t tot,
                                uint32_t shift, uint32_t *__restrict__ dk,
                                uint32_t *__restrict__ ids) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t t = e / n;
        uint32_t rk = (uint32_t)(e - t * n);
        uint32_t id = perm[rk];
        dk[e] = (uint32_t)(keys[t * n + id] >> shift);
        ids[e] = id;
    }
}

__global__ void k_group_flags(const uint32_t *__restrict__ dk, uint32_t n, uint64_t tot,
                              uint32_t *__restrict__ flags) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        bool f = (e % n == 0) || dk[e] != dk[e - 1];
        flags[e] = f ? 1u : 0u;
    }
}

// gid[e] = inclusive group index; gstart[g] = first entry of group g.
__global__ void k_group_starts(const uint32_t *__restrict__ dk, uint32_t n, uint64_t tot,
                               const uint32_t *__restrict__ gexcl, uint32_t *__restrict__ gid,
                               uint32_t *__restrict__ gstart, const uint64_t *__restrict__ ngroups) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        bool f = (e % n == 0) || dk[e] != dk[e - 1];
        uint32_t g = gexcl[e] + (f ? 1u : 0u) - 1u;
        gid[e] = g;
        if (f) gstart[g] = (uint32_t)e;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) gstart[*ngroups] = (uint32_t)tot;
}

// Sorted copies of the full key and the length of every bucket entry.
__global__ void k_sorted_attrs(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ ids,
                               const uint32_t *__restrict__ len, uint32_t n, uint64_t tot,
                               uint64_t *__restrict__ key_s, uint32_t *__restrict__ len_s) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t t = e / n;
        uint32_t id = ids[e];
        key_s[e] = keys[t * n + id];
        len_s[e] = len[id];
    }
}

// Pairs of entry e: following entries of its group inside the length window
// with an equal full key.  EMIT = false counts, EMIT = true writes packed
// codes (min << B | max) from out + offs[e]; C is 32 bits when 2B <= 32.
template <bool EMIT, typename C>
__global__ void k_pairs(const uint64_t *__restrict__ key_s, const uint32_t *__restrict__ len_s,
                        const uint32_t *__restrict__ ids, const uint32_t *__restrict__ gid,
                        const uint32_t *__restrict__ gstart, uint64_t tot, uint32_t K,
                        uint32_t B, uint64_t *__restrict__ counts,
                        const uint64_t *__restrict__ offs, C *__restrict__ out) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t ge = gstart[gid[e] + 1];
        const uint64_t ke = key_s[e];
        const uint64_t lim = (uint64_t)len_s[e] + K;
        const uint32_t ide = ids[e];
        uint64_t c = 0;
        uint64_t o = EMIT ? offs[e] : 0;
        for (uint64_t q = e + 1; q < ge; q++) {
            if ((uint64_t)len_s[q] > lim) break;
            if (key_s[q] == ke) {
                if (EMIT) {
                    uint32_t idq = ids[q];
                    uint32_t a = min(ide, idq), b = max(ide, idq);
                    out[o + c] = (C)(((uint64_t)a << B) | b);
                }
                c++;
            }
        }
        if (!EMIT) counts[e] = c;
    }
}

template <typename C>
__global__ void k_unique_flags(const C *__restrict__ codes, uint64_t cnt,
                               uint32_t *__restrict__ flags) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x)
        flags[e] = (e == 0 || codes[e] != codes[e - 1]) ? 1u : 0u;
}

template <typename C>
__global__ void k_unique_compact(const C *__restrict__ codes, uint64_t cnt, uint32_t B,
                                 const uint32_t *__restrict__ flags,
                                 const uint32_t *__restrict__ pos, uint64_t *__restrict__ out,
                                 uint32_t *__restrict__ first) {
    const uint64_t mask = (1ULL << B) - 1ULL;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x) {
        if (flags[e]) {
            const uint64_t c = codes[e];
            out[pos[e]] = ((c >> B) << 32) | (c & mask);
            if (first) first[pos[e]] = (uint32_t)e;
        }
    }
}

// Sort key of unique pair u: 0xFFFF - (number of raw copies, at most 0xFFFF),
// so that an ascending sort puts the most frequent pairs first.
__global__ void k_mult_keys(const uint32_t *__restrict__ first, uint64_t cnt, uint64_t raw,
                            uint32_t *__restrict__ key, uint32_t *__restrict__ idx) {
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < cnt;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t end = u + 1 < cnt ? first[u + 1] : raw;
        const uint64_t m = end - first[u];
        key[u] = 0xFFFFu - (uint32_t)(m < 0xFFFFu ? m : 0xFFFFu);
        idx[u] = (uint32_t)u;
    }
}

}  // namespace

void bucket(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_len, const uint32_t *d_perm,
            uint32_t n, uint32_t T, uint32_t key_bits, Buckets &bk, const char *tag,
            bool want_ngroups) {
    std::string t(tag);
    bk.T = T;
    bk.n = n;
    uint64_t tot = (uint64_t)T * n;
    if (tot >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "r*z*n must stay below 2^32");
    if (key_bits == 0) key_bits = ctx->tune.bucket_key_bits;
    // enough bits that different keys rarely share a group (the pair scan
    // compares full keys, so a shared group costs time, never results)
    if (key_bits == 0) key_bits = std::min(32u, bits_for(n) + 6);
    if (key_bits > 32) key_bits = 32;
    bk.d_ids = ws<uint32_t>(ctx, t + "_ids", tot);
    bk.d_gid = ws<uint32_t>(ctx, t + "_gid", tot);
    bk.d_gstart = ws<uint32_t>(ctx, t + "_gstart", tot + 1);
    bk.ngroups = 0;
    if (tot == 0) {
        uint32_t zero = 0;
        EJ_HIP(hipMemcpyAsync(bk.d_gstart, &zero, 4, hipMemcpyHostToDevice, ctx->stream));
        sync(ctx);
        return;
    }
    uint32_t *dk = ws<uint32_t>(ctx, t + "_dk", tot);
    uint32_t *dk2 = ws<uint32_t>(ctx, t + "_dk2", tot);
    uint32_t *ids0 = ws<uint32_t>(ctx, t + "_ids0", tot);
    hipLaunchKernelGGL(k_bucket_gather, dim3(grid_for(ctx, tot, 256)), dim3(256), 0, ctx->stream,
                       d_keys, d_perm, n, tot, 61u - key_bits, dk, ids0);
    EJ_CHECK_LAUNCH();
    radix_sort_u32(ctx, dk, ids0, dk2, bk.d_ids, T, n, key_bits, ctx->tune.radix_bits);
    uint32_t *flags = ws<uint32_t>(ctx, t + "_flags", tot);
    uint64_t *d_ng = ws<uint64_t>(ctx, t + "_ngroups", 1);
    hipLaunchKernelGGL(k_group_flags, dim3(grid_for(ctx, tot, 256)), dim3(256), 0, ctx->stream,
                       (const uint32_t *)dk2, n, tot, flags);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, flags, flags, tot, d_ng);
    hipLaunchKernelGGL(k_group_starts, dim3(grid_for(ctx, tot, 256)), dim3(256), 0, ctx->stream,
                       (const uint32_t *)dk2, n, tot, (const uint32_t *)flags, bk.d_gid,
                       bk.d_gstart, (const uint64_t *)d_ng);
    EJ_CHECK_LAUNCH();
    if (want_ngroups) read_back(ctx, d_ng, 8, &bk.ngroups);
}

uint64_t candidates(ej_ctx *ctx, const uint64_t *d_keys, const Buckets &bk, const uint32_t *d_len,
                    uint32_t K, uint64_t **d_pairs_out, uint64_t *n_raw, const char *tag,
                    uint32_t **d_order_out) {
    std::string t(tag);
    const uint32_t n = bk.n;
    const uint64_t tot = (uint64_t)bk.T * n;
    *d_pairs_out = ws<uint64_t>(ctx, t + "_pairs", 1);
    if (n_raw) *n_raw = 0;
    if (tot == 0 || n < 2) return 0;
    uint64_t *key_s = ws<uint64_t>(ctx, t + "_key_s", tot);
    uint32_t *len_s = ws<uint32_t>(ctx, t + "_len_s", tot);
    hipLaunchKernelGGL(k_sorted_attrs, dim3(grid_for(ctx, tot, 256)), dim3(256), 0, ctx->stream,
                       d_keys, (const uint32_t *)bk.d_ids, d_len, n, tot, key_s, len_s);
    EJ_CHECK_LAUNCH();
    uint64_t *counts = ws<uint64_t>(ctx, t + "_counts", tot);
    uint64_t *d_raw = ws<uint64_t>(ctx, t + "_nraw", 1);
    const uint32_t B = std::max(1u, bits_for(n - 1));
    hipLaunchKernelGGL((k_pairs<false, uint64_t>), dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                       ctx->stream, (const uint64_t *)key_s, (const uint32_t *)len_s,
                       (const uint32_t *)bk.d_ids, (const uint32_t *)bk.d_gid,
                       (const uint32_t *)bk.d_gstart, tot, K, B, counts, nullptr,
                       (uint64_t *)nullptr);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u64(ctx, counts, counts, tot, d_raw);
    uint64_t raw = 0;
    read_back(ctx, d_raw, 8, &raw);
    if (n_raw) *n_raw = raw;
    if (raw == 0) return 0;
    if (raw >= 0xFFFFFFFFull)
        fail(EJ_EUNSUPPORTED, "more than 2^32 raw candidate pairs (" + std::to_string(raw) + ")");
    uint32_t *flags = ws<uint32_t>(ctx, t + "_uflags", raw);
    uint32_t *pos = ws<uint32_t>(ctx, t + "_upos", raw);
    uint64_t *d_cnt = ws<uint64_t>(ctx, t + "_ucount", 1);
    // the packed codes are sorted, then the first of each run of equal codes
    // kept; 32-bit codes when both indexes fit in 16 bits, which halves the
    // sort's traffic
    auto emit_sort_unique = [&](auto *rawbuf, auto *sorted) -> uint64_t {
        using C = std::remove_pointer_t<decltype(rawbuf)>;
        hipLaunchKernelGGL((k_pairs<true, C>), dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                           ctx->stream, (const uint64_t *)key_s, (const uint32_t *)len_s,
                           (const uint32_t *)bk.d_ids, (const uint32_t *)bk.d_gid,
                           (const uint32_t *)bk.d_gstart, tot, K, B, (uint64_t *)nullptr,
                           (const uint64_t *)counts, rawbuf);
        EJ_CHECK_LAUNCH();
        if constexpr (sizeof(C) == 4)
            radix_sort_u32(ctx, rawbuf, nullptr, sorted, nullptr, 1, (uint32_t)raw, 2 * B,
                           ctx->tune.radix_bits);
        else
            radix_sort_u64(ctx, rawbuf, sorted, raw, 2 * B, ctx->tune.radix_bits);
        hipLaunchKernelGGL(k_unique_flags<C>, dim3(grid_for(ctx, raw, 256)), dim3(256), 0,
                           ctx->stream, (const C *)sorted, raw, flags);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u32(ctx, flags, pos, raw, d_cnt);
        uint64_t cnt = 0;
        read_back(ctx, d_cnt, 8, &cnt);
        uint64_t *pairs = ws<uint64_t>(ctx, t + "_pairs", cnt);
        uint32_t *first = d_order_out ? ws<uint32_t>(ctx, t + "_first", cnt) : nullptr;
        hipLaunchKernelGGL(k_unique_compact<C>, dim3(grid_for(ctx, raw, 256)), dim3(256), 0,
                           ctx->stream, (const C *)sorted, raw, B, (const uint32_t *)flags,
                           (const uint32_t *)pos, pairs, first);
        EJ_CHECK_LAUNCH();
        *d_pairs_out = pairs;
        return cnt;
    };
    uint64_t cnt;
    if (2 * B <= 32)
        cnt = emit_sort_unique(ws<uint32_t>(ctx, t + "_raw32", raw),
                               ws<uint32_t>(ctx, t + "_raw32_sorted", raw));
    else
        cnt = emit_sort_unique(ws<uint64_t>(ctx, t + "_raw", raw),
                               ws<uint64_t>(ctx, t + "_raw_sorted", raw));
    if (d_order_out && cnt) {
        const uint32_t *first = ws<uint32_t>(ctx, t + "_first", cnt);
        uint32_t *k0 = ws<uint32_t>(ctx, t + "_okey", cnt);
        uint32_t *v0 = ws<uint32_t>(ctx, t + "_oidx", cnt);
        uint32_t *k1 = ws<uint32_t>(ctx, t + "_okey2", cnt);
        uint32_t *order = ws<uint32_t>(ctx, t + "_order", cnt);
        hipLaunchKernelGGL(k_mult_keys, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0, ctx->stream,
                           first, cnt, raw, k0, v0);
        EJ_CHECK_LAUNCH();
        radix_sort_u32(ctx, k0, v0, k1, order, 1, (uint32_t)cnt, 16, 8);
        *d_order_out = order;
    }
    return cnt;
}

}  // namespace ej
