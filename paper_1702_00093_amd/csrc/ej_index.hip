// Stage A8: a device-resident LSH index answering batches of similarity
// queries with per-query thresholds.
//
// Build: the index strings go through A0-A3 once (alphabet, truncation,
// randomness, embedding, per-table sort by (top key bits, length,
// position)); the sorted tables, the full keys and the lengths stay in HBM.
// Query batch: the queries are embedded with the same random streams,
// truncation and alphabet (A1-A2); for every (table, query) a binary search
// finds the group of entries with the query key's top bits and, inside it,
// the length window [|q| - K_q, |q| + K_q]; entries with the same full key
// are candidates.  Candidates are de-duplicated per query, verified with the
// banded kernel at the query's own threshold (A5) and returned per query
// sorted by index position.
#include <string.h>

#include <algorithm>

#include "ej_internal.h"

using namespace ej;

struct ej_index {
    ej_ctx *ctx = nullptr;
    ej_params p{};
    uint32_t n = 0, sigma = 0, L = 0, maxlen = 0, T = 0;
    uint64_t total = 0;            // characters of the indexed strings
    uint8_t lut[256];
    uint64_t hbm_limit = 0;
    // owned device memory
    uint8_t *d_codes = nullptr;
    uint64_t *d_offsets = nullptr;
    uint32_t *d_dk = nullptr;      // [T][n] top 32 key bits, sorted per table
    uint64_t *d_key_s = nullptr;   // [T][n] full keys in sorted order
    uint32_t *d_len_s = nullptr;   // [T][n] lengths in sorted order
    uint32_t *d_ids = nullptr;     // [T][n] positions in sorted order
    RowMasks masks;                // match masks of the index strings (verification)
    Rand rd;                       // random streams (owned copies)
    std::vector<void *> owned;
};

namespace {

inline uint32_t grid_for(ej_ctx *ctx, uint64_t work, uint32_t block) {
    uint64_t g = (work + block - 1) / block;
    uint64_t cap = (uint64_t)ctx->num_cu * 16;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return (uint32_t)g;
}

template <typename T>
T *own_copy(ej_index *ix, const T *src, size_t count) {
    T *dst = nullptr;
    size_t bytes = std::max<size_t>(count * sizeof(T), 16);
    hipError_t e = hipMalloc((void **)&dst, bytes);
    if (e != hipSuccess) fail(EJ_ENOMEM, "index allocation failed");
    ix->owned.push_back(dst);
    if (src && count)
        EJ_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToDevice,
                              ix->ctx->stream));
    return dst;
}

__global__ void k_sorted_attrs_full(const uint64_t *__restrict__ keys,
                                    const uint32_t *__restrict__ ids,
                                    const uint32_t *__restrict__ len, uint32_t n, uint64_t tot,
                                    uint32_t *__restrict__ dk, uint64_t *__restrict__ key_s,
                                    uint32_t *__restrict__ len_s) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t t = e / n;
        uint32_t id = ids[e];
        uint64_t k = keys[t * n + id];
        key_s[e] = k;
        dk[e] = (uint32_t)(k >> 29);
        len_s[e] = len[id];
    }
}

// One thread per (table, query): candidates are the entries of the table
// with the query's full key whose length is within K_q of the query's.
template <bool EMIT>
__global__ void k_query_probe(const uint64_t *__restrict__ qkeys, const uint32_t *__restrict__ qlen,
                              const uint32_t *__restrict__ Kq, uint32_t nq,
                              const uint32_t *__restrict__ dk, const uint64_t *__restrict__ key_s,
                              const uint32_t *__restrict__ len_s, const uint32_t *__restrict__ ids,
                              uint32_t n, uint32_t T, uint32_t B, uint64_t *__restrict__ counts,
                              const uint64_t *__restrict__ offs, uint64_t *__restrict__ out) {
    const uint64_t tot = (uint64_t)T * nq;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t t = (uint32_t)(e / nq), q = (uint32_t)(e % nq);
        const uint64_t key = qkeys[(uint64_t)t * nq + q];
        const uint32_t top = (uint32_t)(key >> 29);
        const uint32_t *d = dk + (uint64_t)t * n;
        const uint64_t *ks = key_s + (uint64_t)t * n;
        const uint32_t *ls = len_s + (uint64_t)t * n;
        // [lo, hi): entries whose top bits equal the query's
        uint32_t lo = 0, hi = n;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (d[mid] < top) lo = mid + 1; else hi = mid;
        }
        uint32_t g0 = lo;
        hi = n;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (d[mid] <= top) lo = mid + 1; else hi = mid;
        }
        const uint32_t g1 = lo;
        const uint32_t lq = qlen[q], kq = Kq[q];
        const uint32_t lmin = lq > kq ? lq - kq : 0u;
        const uint64_t lmax = (uint64_t)lq + kq;
        lo = g0;
        hi = g1;
        while (lo < hi) {  // first entry of the group with length >= lmin
            uint32_t mid = (lo + hi) >> 1;
            if (ls[mid] < lmin) lo = mid + 1; else hi = mid;
        }
        uint64_t c = 0, o = EMIT ? offs[e] : 0;
        for (uint32_t x = lo; x < g1 && (uint64_t)ls[x] <= lmax; x++) {
            if (ks[x] == key) {
                if (EMIT) out[o + c] = ((uint64_t)q << B) | ids[(uint64_t)t * n + x];
                c++;
            }
        }
        if (!EMIT) counts[e] = c;
    }
}

// Incremental insert (Algorithm 3 inserts strings one by one in length
// order; here a batch at once).  Per table, the index's entries and the new
// ones are each sorted by (top key bits, length, position), and every new
// position is above every old one, so the merged order puts an old entry
// before a new one with equal (top bits, length).  Each entry's merged
// position is its own rank plus the number of the other list's entries that
// go before it (binary search); old and new entries are scattered there.
__device__ inline bool before_or_tie(uint32_t d0, uint32_t l0, uint32_t d1, uint32_t l1) {
    return d0 < d1 || (d0 == d1 && l0 <= l1);
}

__global__ void k_merge_tables(const uint32_t *__restrict__ dkA, const uint64_t *__restrict__ keyA,
                               const uint32_t *__restrict__ lenA, const uint32_t *__restrict__ idA,
                               uint32_t nA, const uint32_t *__restrict__ dkB,
                               const uint64_t *__restrict__ keyB, const uint32_t *__restrict__ lenB,
                               const uint32_t *__restrict__ idB, uint32_t nB, uint32_t T,
                               uint32_t *__restrict__ dk, uint64_t *__restrict__ key,
                               uint32_t *__restrict__ len, uint32_t *__restrict__ id) {
    const uint64_t nN = (uint64_t)nA + nB;
    const uint64_t tot = (uint64_t)T * nN;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < tot;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t t = (uint32_t)(g / nN);
        const uint32_t x = (uint32_t)(g - (uint64_t)t * nN);
        const uint64_t a0 = (uint64_t)t * nA, b0 = (uint64_t)t * nB;
        uint32_t rank, d, l;
        uint64_t k;
        uint32_t i;
        if (x < nA) {  // old entry: new entries strictly before it
            d = dkA[a0 + x];
            l = lenA[a0 + x];
            uint32_t lo = 0, hi = nB;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                const uint32_t dm = dkB[b0 + mid], lm = lenB[b0 + mid];
                if (dm < d || (dm == d && lm < l)) lo = mid + 1; else hi = mid;
            }
            rank = x + lo;
            k = keyA[a0 + x];
            i = idA[a0 + x];
        } else {  // new entry: old entries before it or tied with it
            const uint32_t y = x - nA;
            d = dkB[b0 + y];
            l = lenB[b0 + y];
            uint32_t lo = 0, hi = nA;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (before_or_tie(dkA[a0 + mid], lenA[a0 + mid], d, l)) lo = mid + 1; else hi = mid;
            }
            rank = y + lo;
            k = keyB[b0 + y];
            i = idB[b0 + y];
        }
        const uint64_t o = (uint64_t)t * nN + rank;
        dk[o] = d;
        key[o] = k;
        len[o] = l;
        id[o] = i;
    }
}

// New entries' positions after the index's n0 strings.
__global__ void k_add_u32(uint32_t *__restrict__ a, uint64_t cnt, uint32_t add) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x)
        a[e] += add;
}

// Offsets of the inserted strings, relative to the new strings' first
// character, placed after the index's characters.
__global__ void k_append_offsets(const uint64_t *__restrict__ off, uint32_t n, uint64_t base,
                                 uint64_t shift, uint64_t *__restrict__ out) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e <= n;
         e += (uint64_t)gridDim.x * blockDim.x)
        out[e] = off[e] - base + shift;
}

__global__ void k_uniq_flags(const uint64_t *__restrict__ codes, uint64_t cnt,
                             uint32_t *__restrict__ flags) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x)
        flags[e] = (e == 0 || codes[e] != codes[e - 1]) ? 1u : 0u;
}

// Unique (q << B | id) codes -> verification pairs (id << 32 | q) and the
// threshold of each pair.
__global__ void k_to_pairs(const uint64_t *__restrict__ codes, uint64_t cnt, uint32_t B,
                           const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos,
                           const uint32_t *__restrict__ Kq, uint64_t *__restrict__ pairs,
                           uint32_t *__restrict__ pk) {
    const uint64_t mask = (1ULL << B) - 1ULL;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x) {
        if (flags[e]) {
            uint64_t c = codes[e];
            uint32_t q = (uint32_t)(c >> B), id = (uint32_t)(c & mask);
            pairs[pos[e]] = ((uint64_t)id << 32) | q;
            pk[pos[e]] = Kq[q];
        }
    }
}

__global__ void k_q_out_flags(const int32_t *__restrict__ dist, const uint32_t *__restrict__ pk,
                              uint64_t cnt, uint32_t *__restrict__ flags) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x)
        flags[e] = (dist[e] >= 0 && (uint32_t)dist[e] <= pk[e]) ? 1u : 0u;
}

__global__ void k_q_out_compact(const uint64_t *__restrict__ pairs, const int32_t *__restrict__ dist,
                                uint64_t cnt, const uint32_t *__restrict__ flags,
                                const uint32_t *__restrict__ pos, uint32_t *__restrict__ ids,
                                int32_t *__restrict__ od, uint32_t *__restrict__ per_q) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x) {
        if (flags[e]) {
            uint64_t c = pairs[e];
            ids[pos[e]] = (uint32_t)(c >> 32);
            od[pos[e]] = dist[e];
            atomicAdd(&per_q[(uint32_t)c], 1u);
        }
    }
}

// Device bytes of a batch before its candidates are known (the admission
// estimate of ej_query_workspace_estimate).
uint64_t estimate(const ej_index *ix, uint64_t qbytes, uint32_t nq) {
    const uint64_t T = ix->T;
    uint64_t b = 0;
    b += 2 * qbytes + 64 * 1024;                 // chars, codes, packed
    b += (uint64_t)nq * (8 + 4 * 6);             // offsets, lengths, order, thresholds
    b += T * nq * (8 + 8 + 8);                   // keys, counts, scan
    b += T * nq * 4 * 8;                         // expected candidates (a few per table)
    return b;
}

// Bytes of the candidate stage once the raw (pre-de-duplication) count is
// known: raw codes, their sorted copy and the radix sort's scratch, unique
// flags and positions, then the pairs and thresholds.
uint64_t probe_bytes(uint64_t raw) { return raw * (8 + 8 + 8 + 4 + 4 + 8 + 4); }

// Bytes of verification and output once the de-duplicated count is known:
// distances, the queries' match masks, the two-pass form's saved state (Pv
// and Mv of NL band words per pair, rounded up to whole lanes of up to 4
// words) and its ordering buffers, output flags and positions, result ids
// and distances.
uint64_t verify_bytes(const ej_ctx *ctx, uint64_t cnt, uint64_t qbytes, uint32_t nq,
                      uint32_t sigma, uint32_t Kmax) {
    const uint64_t NL = verify_lanes_for(Kmax);
    uint64_t b = cnt * 4;                                           // distances
    b += mask_words_bound(qbytes, nq, sigma) * 4 + 24ull * (nq + 1);  // query masks
    if (ctx->tune.verify_mode == 0) b += cnt * (8 * (NL + 3) + 4 * 8 + 8);  // two-pass state
    b += cnt * (4 + 4 + 4 + 4);                                     // output
    return b;
}

}  // namespace

extern "C" {

ej_status ej_index_build(ej_ctx *ctx, const uint8_t *strings, const uint64_t *offsets, uint32_t n,
                         const ej_params *p, int on_device, ej_index **out) {
    if (!ctx || !p || !out || !offsets) return EJ_EINVAL;
    *out = nullptr;
    ej_index *ix = new (std::nothrow) ej_index();
    if (!ix) return EJ_ENOMEM;
    ix->ctx = ctx;
    ej_status st = run_guarded(ctx, [&] {
        if (p->r == 0 || p->z == 0 || p->m == 0 || p->m > 64 || (uint64_t)p->r * p->z > 4096)
            fail(EJ_EINVAL, "invalid r, z, m");
        if (n >= 0x80000000u) fail(EJ_EINVAL, "n must be below 2^31");
        ix->p = *p;
        ix->n = n;
        ix->T = p->r * p->z;
        const uint8_t *d_chars = strings;
        const uint64_t *d_off = offsets;
        if (!on_device) {
            std::vector<uint64_t> reb(offsets, offsets + n + 1);
            for (uint32_t i = 0; i < n; i++)
                if (offsets[i + 1] < offsets[i]) fail(EJ_EINVAL, "offsets are not non-decreasing");
            uint64_t base = offsets[0], total = offsets[n] - base;
            for (auto &o : reb) o -= base;
            uint8_t *dc = ws<uint8_t>(ctx, "ix_hchars", total + 16);
            uint64_t *dofs = ws<uint64_t>(ctx, "ix_hoff", (uint64_t)n + 1);
            if (total) EJ_HIP(hipMemcpyAsync(dc, strings + base, total, hipMemcpyHostToDevice, ctx->stream));
            EJ_HIP(hipMemcpyAsync(dofs, reb.data(), 8ull * (n + 1), hipMemcpyHostToDevice, ctx->stream));
            sync(ctx);
            d_chars = dc;
            d_off = dofs;
        }
        Prep pp;
        prepare(ctx, d_chars, d_off, n, p->L, pp, "ix");
        ix->sigma = pp.sigma;
        ix->L = pp.L;
        ix->maxlen = pp.maxlen;
        ix->total = pp.total;
        memcpy(ix->lut, pp.lut, 256);
        Rand rd;
        draw_randomness(ctx, *p, pp.L, pp.sigma, rd, "ix");
        const uint64_t tot = (uint64_t)ix->T * n;
        uint64_t *keys = ws<uint64_t>(ctx, "ix_keys", tot);
        embed_keys(ctx, pp, rd, keys, nullptr);
        Buckets bk;
        bucket(ctx, keys, pp.d_len, pp.d_perm, n, ix->T, 32, bk, "ix");
        // owned copies
        ix->d_codes = own_copy(ix, pp.d_codes, pp.total + 64);
        // offsets rebased onto the owned code array
        ix->d_offsets = own_copy(ix, d_off, (uint64_t)n + 1);
        ix->rd = rd;
        ix->rd.d_Rwords = own_copy(ix, rd.d_Rwords, (size_t)rd.r * rd.nw);
        ix->rd.d_Rstep = own_copy(ix, rd.d_Rstep, (size_t)rd.r * rd.Lpad);
        ix->rd.d_pos = own_copy(ix, rd.d_pos, (size_t)ix->T * rd.m);
        ix->rd.d_v = own_copy(ix, rd.d_v, (size_t)ix->T * rd.m);
        ix->rd.d_spos = own_copy(ix, rd.d_spos, (size_t)ix->T * rd.m);
        ix->rd.d_sslot = own_copy(ix, rd.d_sslot, (size_t)ix->T * rd.m);
        ix->rd.d_J = own_copy(ix, rd.d_J, (size_t)rd.r);
        ix->d_ids = own_copy(ix, bk.d_ids, tot);
        ix->d_dk = own_copy<uint32_t>(ix, nullptr, tot);
        ix->d_key_s = own_copy<uint64_t>(ix, nullptr, tot);
        ix->d_len_s = own_copy<uint32_t>(ix, nullptr, tot);
        if (tot)
            hipLaunchKernelGGL(k_sorted_attrs_full, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                               ctx->stream, (const uint64_t *)keys, (const uint32_t *)ix->d_ids,
                               (const uint32_t *)pp.d_len, n, tot, ix->d_dk, ix->d_key_s,
                               ix->d_len_s);
        EJ_CHECK_LAUNCH();
        // match masks of the index strings, kept for every query batch
        {
            uint32_t *mw = own_copy<uint32_t>(ix, nullptr, mask_words_bound(pp.total, n, pp.sigma));
            uint64_t *mo = own_copy<uint64_t>(ix, nullptr, (uint64_t)n + 1);
            build_masks(ctx, pp.d_codes, d_off, pp.base, n, pp.total, pp.sigma, ix->masks, "ixm",
                        mw, mo);
        }
        // the owned offsets must be relative to the owned codes: base 0
        if (pp.base) {
            std::vector<uint64_t> h(n + 1);
            EJ_HIP(hipMemcpyAsync(h.data(), ix->d_offsets, 8ull * (n + 1), hipMemcpyDeviceToHost,
                                  ctx->stream));
            sync(ctx);
            for (auto &o : h) o -= pp.base;
            EJ_HIP(hipMemcpyAsync(ix->d_offsets, h.data(), 8ull * (n + 1), hipMemcpyHostToDevice,
                                  ctx->stream));
        }
        sync(ctx);
    });
    if (st != EJ_OK) {
        ej_index_free(ix);
        return st;
    }
    *out = ix;
    return EJ_OK;
}

ej_status ej_index_insert(ej_index *ix, const uint8_t *strings, const uint64_t *offsets,
                          uint32_t n_new, int on_device) {
    if (!ix || !offsets) return EJ_EINVAL;
    ej_ctx *ctx = ix->ctx;
    std::vector<void *> fresh;  // allocations of this call, released on failure
    ej_status st = run_guarded(ctx, [&] {
        if (n_new == 0) return;
        if ((uint64_t)ix->n + n_new >= 0x80000000ull) fail(EJ_EINVAL, "n must stay below 2^31");
        const uint64_t nN = (uint64_t)ix->n + n_new;
        if (nN * ix->T >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "r*z*n must stay below 2^32");
        const uint8_t *d_chars = strings;
        const uint64_t *d_off = offsets;
        if (!on_device) {
            std::vector<uint64_t> reb(offsets, offsets + n_new + 1);
            for (uint32_t i = 0; i < n_new; i++)
                if (offsets[i + 1] < offsets[i]) fail(EJ_EINVAL, "offsets are not non-decreasing");
            const uint64_t base = offsets[0], total = offsets[n_new] - base;
            if (total && !strings) fail(EJ_EINVAL, "null strings");
            for (auto &o : reb) o -= base;
            uint8_t *dc = ws<uint8_t>(ctx, "ii_hchars", total + 16);
            uint64_t *dofs = ws<uint64_t>(ctx, "ii_hoff", (uint64_t)n_new + 1);
            if (total)
                EJ_HIP(hipMemcpyAsync(dc, strings + base, total, hipMemcpyHostToDevice,
                                      ctx->stream));
            EJ_HIP(hipMemcpyAsync(dofs, reb.data(), 8ull * (n_new + 1), hipMemcpyHostToDevice,
                                  ctx->stream));
            sync(ctx);
            d_chars = dc;
            d_off = dofs;
        }
        // the new strings under the index's alphabet, truncation and streams
        Prep pq;
        prepare(ctx, d_chars, d_off, n_new, 0, pq, "ii", ix->lut, ix->sigma, ix->L);
        const uint32_t T = ix->T;
        const uint64_t totB = (uint64_t)T * n_new;
        uint64_t *keys = ws<uint64_t>(ctx, "ii_keys", totB);
        embed_keys(ctx, pq, ix->rd, keys, nullptr);
        Buckets bk;
        bucket(ctx, keys, pq.d_len, pq.d_perm, n_new, T, 32, bk, "ii");
        uint32_t *dkB = ws<uint32_t>(ctx, "ii_dkB", totB);
        uint64_t *keyB = ws<uint64_t>(ctx, "ii_keyB", totB);
        uint32_t *lenB = ws<uint32_t>(ctx, "ii_lenB", totB);
        hipLaunchKernelGGL(k_sorted_attrs_full, dim3(grid_for(ctx, totB, 256)), dim3(256), 0,
                           ctx->stream, (const uint64_t *)keys, (const uint32_t *)bk.d_ids,
                           (const uint32_t *)pq.d_len, n_new, totB, dkB, keyB, lenB);
        EJ_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_add_u32, dim3(grid_for(ctx, totB, 256)), dim3(256), 0, ctx->stream,
                           bk.d_ids, totB, ix->n);
        EJ_CHECK_LAUNCH();
        // the grown index, built beside the current one (which stays whole
        // until every allocation has succeeded)
        auto alloc = [&](size_t bytes) -> void * {
            void *p = nullptr;
            if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
                (void)hipGetLastError();
                fail(EJ_ENOMEM, "index insert: device allocation failed");
            }
            fresh.push_back(p);
            return p;
        };
        const uint64_t totN = (uint64_t)T * nN;
        const uint64_t charsN = ix->total + pq.total;
        uint32_t *dk = (uint32_t *)alloc(4 * totN);
        uint64_t *key = (uint64_t *)alloc(8 * totN);
        uint32_t *len = (uint32_t *)alloc(4 * totN);
        uint32_t *id = (uint32_t *)alloc(4 * totN);
        uint8_t *codes = (uint8_t *)alloc(charsN + 64);
        uint64_t *offs = (uint64_t *)alloc(8 * (nN + 1));
        uint32_t *mw = (uint32_t *)alloc(4 * mask_words_bound(charsN, (uint32_t)nN, ix->sigma));
        uint64_t *mo = (uint64_t *)alloc(8 * (nN + 1));
        hipLaunchKernelGGL(k_merge_tables, dim3(grid_for(ctx, totN, 256)), dim3(256), 0,
                           ctx->stream, (const uint32_t *)ix->d_dk, (const uint64_t *)ix->d_key_s,
                           (const uint32_t *)ix->d_len_s, (const uint32_t *)ix->d_ids, ix->n,
                           (const uint32_t *)dkB, (const uint64_t *)keyB, (const uint32_t *)lenB,
                           (const uint32_t *)bk.d_ids, n_new, T, dk, key, len, id);
        EJ_CHECK_LAUNCH();
        // codes and offsets: the new strings after the indexed ones (the new
        // codes carry their zero padding along)
        if (ix->total)
            EJ_HIP(hipMemcpyAsync(codes, ix->d_codes, ix->total, hipMemcpyDeviceToDevice,
                                  ctx->stream));
        EJ_HIP(hipMemcpyAsync(codes + ix->total, pq.d_codes, pq.total + 64,
                              hipMemcpyDeviceToDevice, ctx->stream));
        EJ_HIP(hipMemcpyAsync(offs, ix->d_offsets, 8ull * ix->n, hipMemcpyDeviceToDevice,
                              ctx->stream));
        hipLaunchKernelGGL(k_append_offsets, dim3(grid_for(ctx, (uint64_t)n_new + 1, 256)),
                           dim3(256), 0, ctx->stream, d_off, n_new, pq.base, ix->total,
                           offs + ix->n);
        EJ_CHECK_LAUNCH();
        RowMasks masks;
        build_masks(ctx, codes, offs, 0, (uint32_t)nN, charsN, ix->sigma, masks, "ixm", mw, mo);
        sync(ctx);
        // swap in the grown arrays; release the replaced ones
        void *old[] = {ix->d_dk, ix->d_key_s, ix->d_len_s, ix->d_ids, ix->d_codes, ix->d_offsets,
                       (void *)ix->masks.words, (void *)ix->masks.off};
        for (void *p : old) {
            auto it = std::find(ix->owned.begin(), ix->owned.end(), p);
            if (it != ix->owned.end()) ix->owned.erase(it);
            (void)hipFree(p);
        }
        ix->owned.insert(ix->owned.end(), fresh.begin(), fresh.end());
        fresh.clear();
        ix->d_dk = dk;
        ix->d_key_s = key;
        ix->d_len_s = len;
        ix->d_ids = id;
        ix->d_codes = codes;
        ix->d_offsets = offs;
        ix->masks = masks;
        ix->n = (uint32_t)nN;
        ix->total = charsN;
        ix->maxlen = std::max(ix->maxlen, pq.maxlen);
    });
    for (void *p : fresh) (void)hipFree(p);
    return st;
}

uint64_t ej_query_workspace_estimate(const ej_index *ix, const uint64_t *q_offsets, uint32_t nq,
                                     const uint32_t *Kq) {
    (void)Kq;
    if (!ix || !q_offsets) return 0;
    return estimate(ix, q_offsets[nq] - q_offsets[0], nq);
}

void ej_index_set_hbm_limit(ej_index *ix, uint64_t bytes) {
    if (ix) ix->hbm_limit = bytes;
}

uint32_t ej_index_size(const ej_index *ix) { return ix ? ix->n : 0; }

ej_status ej_query_batch(ej_index *ix, const uint8_t *q, const uint64_t *q_offsets, uint32_t nq,
                         const uint32_t *Kq, ej_qresult *out) {
    if (!ix || !q_offsets || !out || (nq && !Kq)) return EJ_EINVAL;
    ej_ctx *ctx = ix->ctx;
    memset(out, 0, sizeof(*out));
    ej_status st = run_guarded(ctx, [&] {
        for (uint32_t i = 0; i < nq; i++) {
            if (q_offsets[i + 1] < q_offsets[i]) fail(EJ_EINVAL, "query offsets decrease");
            if (verify_lanes_for(Kq[i]) == 0) fail(EJ_EUNSUPPORTED, "query threshold above 2046");
        }
        const uint64_t qbase = q_offsets[0], qtotal = q_offsets[nq] - qbase;
        if (qtotal && !q) fail(EJ_EINVAL, "null query strings");
        // admission by free HBM (or the configured limit)
        size_t freeb = 0, totalb = 0;
        EJ_HIP(hipMemGetInfo(&freeb, &totalb));
        const uint64_t avail = ix->hbm_limit ? ix->hbm_limit : (uint64_t)freeb;
        uint32_t Kmax = 0;
        for (uint32_t i = 0; i < nq; i++) Kmax = std::max(Kmax, Kq[i]);
        // admission, checked again as each data-dependent size becomes known
        // and before any of that stage's memory is requested
        uint64_t need = estimate(ix, qtotal, nq);
        auto admit = [&](const char *what) {
            if (need > avail)
                fail(EJ_ENOMEM, std::string("batch needs ~") + std::to_string(need) +
                                    " bytes (" + what + "), " + std::to_string(avail) +
                                    " admitted");
        };
        admit("before embedding");
        EJ_HIP(hipEventRecord(ctx->timers.ev[0], ctx->stream));
        out->nq = nq;
        out->offsets = (uint64_t *)calloc((size_t)nq + 1, sizeof(uint64_t));
        if (!out->offsets) fail(EJ_ENOMEM, "host allocation failed");
        if (nq == 0) return;
        // upload
        std::vector<uint64_t> reb(q_offsets, q_offsets + nq + 1);
        for (auto &o : reb) o -= qbase;
        uint8_t *dq = ws<uint8_t>(ctx, "q_chars", qtotal + 16);
        uint64_t *dqo = ws<uint64_t>(ctx, "q_off", (uint64_t)nq + 1);
        uint32_t *dK = ws<uint32_t>(ctx, "q_K", nq);
        if (qtotal) EJ_HIP(hipMemcpyAsync(dq, q + qbase, qtotal, hipMemcpyHostToDevice, ctx->stream));
        EJ_HIP(hipMemcpyAsync(dqo, reb.data(), 8ull * (nq + 1), hipMemcpyHostToDevice, ctx->stream));
        EJ_HIP(hipMemcpyAsync(dK, Kq, 4ull * nq, hipMemcpyHostToDevice, ctx->stream));
        // A0-A2 on the queries with the index's alphabet, truncation and randomness
        Prep pq;
        prepare(ctx, dq, dqo, nq, 0, pq, "q", ix->lut, ix->sigma, ix->L);
        const uint32_t T = ix->T;
        uint64_t *qkeys = ws<uint64_t>(ctx, "q_keys", (uint64_t)T * nq);
        embed_keys(ctx, pq, ix->rd, qkeys, nullptr);
        // probe
        const uint64_t tot = (uint64_t)T * nq;
        uint64_t *counts = ws<uint64_t>(ctx, "q_counts", tot);
        uint64_t *d_raw = ws<uint64_t>(ctx, "q_raw", 1);
        const uint32_t B = std::max(1u, std::max(bits_for(ix->n ? ix->n - 1 : 0), bits_for(nq - 1)));
        hipLaunchKernelGGL(k_query_probe<false>, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                           ctx->stream, (const uint64_t *)qkeys, (const uint32_t *)pq.d_len,
                           (const uint32_t *)dK, nq, (const uint32_t *)ix->d_dk,
                           (const uint64_t *)ix->d_key_s, (const uint32_t *)ix->d_len_s,
                           (const uint32_t *)ix->d_ids, ix->n, T, B, counts, nullptr, nullptr);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u64(ctx, counts, counts, tot, d_raw);
        uint64_t raw = 0;
        read_back(ctx, d_raw, 8, &raw);
        need += probe_bytes(raw);
        admit("with the candidate stage");
        uint64_t cnt = 0;
        uint64_t *pairs = nullptr;
        uint32_t *pk = nullptr;
        if (raw) {
            if (raw >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "more than 2^32 raw query candidates");
            uint64_t *rb = ws<uint64_t>(ctx, "q_rawbuf", raw);
            uint64_t *sorted = ws<uint64_t>(ctx, "q_sorted", raw);
            hipLaunchKernelGGL(k_query_probe<true>, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                               ctx->stream, (const uint64_t *)qkeys, (const uint32_t *)pq.d_len,
                               (const uint32_t *)dK, nq, (const uint32_t *)ix->d_dk,
                               (const uint64_t *)ix->d_key_s, (const uint32_t *)ix->d_len_s,
                               (const uint32_t *)ix->d_ids, ix->n, T, B, nullptr,
                               (const uint64_t *)counts, rb);
            EJ_CHECK_LAUNCH();
            radix_sort_u64(ctx, rb, sorted, raw, 2 * B, ctx->tune.radix_bits);
            uint32_t *flags = ws<uint32_t>(ctx, "q_uflags", raw);
            uint32_t *pos = ws<uint32_t>(ctx, "q_upos", raw);
            uint64_t *d_cnt = ws<uint64_t>(ctx, "q_ucnt", 1);
            hipLaunchKernelGGL(k_uniq_flags, dim3(grid_for(ctx, raw, 256)), dim3(256), 0,
                               ctx->stream, (const uint64_t *)sorted, raw, flags);
            EJ_CHECK_LAUNCH();
            scan_exclusive_u32(ctx, flags, pos, raw, d_cnt);
            read_back(ctx, d_cnt, 8, &cnt);
            pairs = ws<uint64_t>(ctx, "q_pairs", cnt);
            pk = ws<uint32_t>(ctx, "q_pk", cnt);
            hipLaunchKernelGGL(k_to_pairs, dim3(grid_for(ctx, raw, 256)), dim3(256), 0,
                               ctx->stream, (const uint64_t *)sorted, raw, B,
                               (const uint32_t *)flags, (const uint32_t *)pos,
                               (const uint32_t *)dK, pairs, pk);
            EJ_CHECK_LAUNCH();
        }
        out->n_candidates = cnt;
        need += verify_bytes(ctx, cnt, qtotal, nq, ix->sigma, Kmax);
        admit("with verification");
        out->workspace_bytes = need;
        uint64_t nout = 0;
        uint32_t *per_q = ws<uint32_t>(ctx, "q_perq", nq);
        EJ_HIP(hipMemsetAsync(per_q, 0, 4ull * nq, ctx->stream));
        uint32_t *oids = nullptr;
        int32_t *odist = nullptr;
        if (cnt) {
            int32_t *dist = ws<int32_t>(ctx, "q_dist", cnt);
            RowMasks qmasks;
            build_masks(ctx, pq.d_codes, dqo, 0, nq, pq.total, ix->sigma, qmasks, "qm");
            verify(ctx, ix->d_codes, ix->d_offsets, 0, ix->sigma, ix->maxlen, ix->masks, pairs,
                   cnt, 0, pk, dist, pq.d_codes, dqo, 0, pq.maxlen, &qmasks);
            uint32_t *flags = ws<uint32_t>(ctx, "q_oflags", cnt);
            uint32_t *pos = ws<uint32_t>(ctx, "q_opos", cnt);
            uint64_t *d_no = ws<uint64_t>(ctx, "q_nout", 1);
            hipLaunchKernelGGL(k_q_out_flags, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0,
                               ctx->stream, (const int32_t *)dist, (const uint32_t *)pk, cnt, flags);
            EJ_CHECK_LAUNCH();
            scan_exclusive_u32(ctx, flags, pos, cnt, d_no);
            read_back(ctx, d_no, 8, &nout);
            oids = ws<uint32_t>(ctx, "q_oids", nout);
            odist = ws<int32_t>(ctx, "q_odist", nout);
            hipLaunchKernelGGL(k_q_out_compact, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0,
                               ctx->stream, (const uint64_t *)pairs, (const int32_t *)dist, cnt,
                               (const uint32_t *)flags, (const uint32_t *)pos, oids, odist, per_q);
            EJ_CHECK_LAUNCH();
        }
        out->ids = (uint32_t *)malloc(4 * (nout ? nout : 1));
        out->dist = (int32_t *)malloc(4 * (nout ? nout : 1));
        std::vector<uint32_t> hq(nq);
        if (!out->ids || !out->dist) fail(EJ_ENOMEM, "host allocation failed");
        if (nout) {
            EJ_HIP(hipMemcpyAsync(out->ids, oids, 4 * nout, hipMemcpyDeviceToHost, ctx->stream));
            EJ_HIP(hipMemcpyAsync(out->dist, odist, 4 * nout, hipMemcpyDeviceToHost, ctx->stream));
        }
        EJ_HIP(hipMemcpyAsync(hq.data(), per_q, 4ull * nq, hipMemcpyDeviceToHost, ctx->stream));
        EJ_HIP(hipEventRecord(ctx->timers.ev[1], ctx->stream));
        sync(ctx);
        for (uint32_t i = 0; i < nq; i++) out->offsets[i + 1] = out->offsets[i] + hq[i];
        float ms = 0.f;
        EJ_HIP(hipEventElapsedTime(&ms, ctx->timers.ev[0], ctx->timers.ev[1]));
        out->ms_total = ms;
    });
    if (st != EJ_OK) ej_qresult_free(out);
    return st;
}

void ej_qresult_free(ej_qresult *res) {
    if (!res) return;
    free(res->offsets);
    free(res->ids);
    free(res->dist);
    memset(res, 0, sizeof(*res));
}

void ej_index_free(ej_index *ix) {
    if (!ix) return;
    if (ix->ctx) {
        (void)hipSetDevice(ix->ctx->device);
        (void)hipStreamSynchronize(ix->ctx->stream);
    }
    for (void *p : ix->owned) (void)hipFree(p);
    delete ix;
}

}  // extern "C"
