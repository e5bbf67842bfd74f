// Device-wide primitives used by the stages: exclusive prefix sums and a
// stable, segmented LSD radix sort.  Both are written for 64-lane waves:
// wave-level steps use ballots and DPP-backed shuffles, block-level steps
// combine the waves of a 256-thread workgroup through LDS.
#include "ej_internal.h"

namespace ej {

namespace {

constexpr int BLK = 256;            // threads per workgroup (4 waves)
constexpr int NWAVE = BLK / 64;
constexpr int IPT = 8;              // items per thread
constexpr int TILE = BLK * IPT;     // items per workgroup tile

template <typename T>
__device__ inline T wave_inclusive_scan(T x, uint32_t lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread across the workgroup.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T *lds, T &total) {
    uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T x = wave_inclusive_scan(v, lane);
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NWAVE; w++) {
        T s = lds[w];
        if (w < (int)wave) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + x - v;
}

template <typename T>
__global__ void __launch_bounds__(BLK) k_scan_reduce(const T *__restrict__ in, uint64_t n,
                                                     T *__restrict__ partials) {
    __shared__ T lds[NWAVE];
    uint64_t base = (uint64_t)blockIdx.x * TILE;
    T s = 0;
#pragma unroll
    for (int i = 0; i < IPT; i++) {
        uint64_t e = base + (uint64_t)i * BLK + threadIdx.x;
        if (e < n) s += in[e];
    }
    T total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the per-tile partial sums.
template <typename T>
__global__ void __launch_bounds__(BLK) k_scan_partials(T *__restrict__ partials, uint64_t nb,
                                                       uint64_t *__restrict__ total_out) {
    __shared__ T lds[NWAVE];
    T carry = 0;
    for (uint64_t base = 0; base < nb; base += TILE) {
        T v[IPT];
        T s = 0;
#pragma unroll
        for (int i = 0; i < IPT; i++) {
            uint64_t e = base + (uint64_t)threadIdx.x * IPT + i;
            v[i] = e < nb ? partials[e] : 0;
            s += v[i];
        }
        T total;
        T ex = block_exclusive_scan(s, lds, total) + carry;
#pragma unroll
        for (int i = 0; i < IPT; i++) {
            uint64_t e = base + (uint64_t)threadIdx.x * IPT + i;
            if (e < nb) partials[e] = ex;
            ex += v[i];
        }
        carry += total;
    }
    if (threadIdx.x == 0 && total_out) *total_out = (uint64_t)carry;
}

template <typename T>
__global__ void __launch_bounds__(BLK) k_scan_down(const T *in, T *out, uint64_t n,
                                                   const T *__restrict__ partials) {
    __shared__ T lds[NWAVE];
    uint64_t base = (uint64_t)blockIdx.x * TILE + (uint64_t)threadIdx.x * IPT;
    T v[IPT];
    T s = 0;
#pragma unroll
    for (int i = 0; i < IPT; i++) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    T total;
    T ex = block_exclusive_scan(s, lds, total) + partials[blockIdx.x];
#pragma unroll
    for (int i = 0; i < IPT; i++) {
        if (base + i < n) out[base + i] = ex;
        ex += v[i];
    }
}

// Small inputs: one workgroup of 1024 threads walks the array in tiles of
// 1024 * IPT with a running carry (one launch instead of three).  In place
// is fine: each element is read and written by the same thread.  Used up to
// one tile: each further tile costs about as much as the three-kernel scan.
constexpr int SBLK = 1024, SNWAVE = SBLK / 64;
constexpr uint64_t SCAN_SINGLE_MAX = (uint64_t)SBLK * IPT;

template <typename T>
__global__ void __launch_bounds__(SBLK) k_scan_single(const T *in, T *out, uint64_t n,
                                                      uint64_t *__restrict__ total_out) {
    __shared__ T wsum[SNWAVE];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T carry = 0;
    for (uint64_t base = 0; base < n; base += (uint64_t)SBLK * IPT) {
        const uint64_t e0 = base + (uint64_t)threadIdx.x * IPT;
        T v[IPT];
        T s = 0;
#pragma unroll
        for (int i = 0; i < IPT; i++) {
            v[i] = e0 + i < n ? in[e0 + i] : 0;
            s += v[i];
        }
        const T x = wave_inclusive_scan(s, lane);
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        T before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < SNWAVE; w++) {
            const T sw = wsum[w];
            if (w < (int)wave) before += sw;
            tot += sw;
        }
        __syncthreads();
        T ex = carry + before + x - s;
#pragma unroll
        for (int i = 0; i < IPT; i++) {
            if (e0 + i < n) out[e0 + i] = ex;
            ex += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = (uint64_t)carry;
}

template <typename T>
void scan_exclusive(ej_ctx *ctx, const T *d_in, T *d_out, uint64_t n, uint64_t *d_total,
                    const char *name) {
    if (n == 0) {
        if (d_total) EJ_HIP(hipMemsetAsync(d_total, 0, sizeof(uint64_t), ctx->stream));
        return;
    }
    if (n <= SCAN_SINGLE_MAX) {
        hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(SBLK), 0, ctx->stream, d_in, d_out, n,
                           d_total);
        EJ_CHECK_LAUNCH();
        return;
    }
    uint64_t nb = (n + TILE - 1) / TILE;
    T *partials = ws<T>(ctx, std::string("scan_partials_") + name, nb);
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((uint32_t)nb), dim3(BLK), 0, ctx->stream, d_in, n,
                       partials);
    EJ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(BLK), 0, ctx->stream, partials, nb,
                       d_total);
    EJ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_down<T>, dim3((uint32_t)nb), dim3(BLK), 0, ctx->stream, d_in, d_out,
                       n, (const T *)partials);
    EJ_CHECK_LAUNCH();
}

// ---------------------------------------------------------- radix sort --

template <typename K>
__global__ void __launch_bounds__(BLK) k_rs_hist(const K *__restrict__ keys, uint32_t seglen,
                                                 uint32_t tps, uint32_t shift, uint32_t dbits,
                                                 uint32_t *__restrict__ hist) {
    extern __shared__ uint32_t cnt[];
    const uint32_t NB = 1u << dbits, mask = NB - 1;
    uint32_t seg = blockIdx.x / tps, tile = blockIdx.x % tps;
    for (uint32_t d = threadIdx.x; d < NB; d += BLK) cnt[d] = 0;
    __syncthreads();
    uint64_t segbase = (uint64_t)seg * seglen;
    uint32_t t0 = tile * TILE;
#pragma unroll
    for (int i = 0; i < IPT; i++) {
        uint32_t e = t0 + i * BLK + threadIdx.x;
        if (e < seglen) {
            uint32_t d = (uint32_t)(keys[segbase + e] >> shift) & mask;
            atomicAdd(&cnt[d], 1u);
        }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < NB; d += BLK)
        hist[((uint64_t)seg * NB + d) * tps + tile] = cnt[d];
}

// Stable scatter of one tile.  Wave w takes the tile's elements
// [512 w, 512 w + 512) in 8 rounds of 64 consecutive ones and ranks them
// among equal digits on its own: a ballot match gives the rank inside a
// round, a wave-private LDS counter per digit the elements of earlier
// rounds (no workgroup barrier while ranking).  One pass over the digits
// then turns the per-wave counts into each wave's first position of each
// digit inside the tile (digits in order, waves in order within a digit:
// the tile's order, so the sort is stable).  The tile is placed in LDS in
// digit order and written out in that order, so that consecutive threads
// write consecutive addresses of a digit's run.
template <typename K, bool HAS_VAL>
__global__ void __launch_bounds__(BLK) k_rs_scatter(const K *__restrict__ kin,
                                                    const uint32_t *__restrict__ vin,
                                                    K *__restrict__ kout,
                                                    uint32_t *__restrict__ vout, uint32_t seglen,
                                                    uint32_t tps, uint32_t shift, uint32_t dbits,
                                                    const uint32_t *__restrict__ hist) {
    extern __shared__ uint32_t sm[];
    __shared__ uint32_t scan_tmp[NWAVE];
    const uint32_t NB = 1u << dbits, mask = NB - 1;
    uint32_t *base_off = sm;           // [NB] output position of the tile's digit-d run
    uint32_t *lstart = sm + NB;        // [NB] start of digit d inside the tile
    uint32_t *wcnt = sm + 2 * NB;      // [NWAVE][NB] counts, then first positions
    K *lkey = (K *)(sm + (3 + NWAVE) * NB);     // [TILE]
    uint32_t *lval = (uint32_t *)(lkey + TILE);  // [TILE]
    const uint32_t seg = blockIdx.x / tps, tile = blockIdx.x % tps;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *mycnt = wcnt + wave * NB;
    for (uint32_t d = threadIdx.x; d < NB; d += BLK)
        base_off[d] = hist[((uint64_t)seg * NB + d) * tps + tile];
    for (uint32_t d = lane; d < NB; d += 64) mycnt[d] = 0;
    const uint64_t segbase = (uint64_t)seg * seglen;
    const uint32_t t0 = tile * TILE;
    const uint32_t nvalid = seglen - t0 < (uint32_t)TILE ? seglen - t0 : (uint32_t)TILE;
    // ---- load and rank the wave's elements (LDS reads and writes of one
    // wave happen in program order: a round's counter reads precede the
    // leaders' updates, which precede the next round's reads)
    K key[IPT];
    uint32_t val[IPT], dg[IPT], lr[IPT];
    const uint64_t lt_mask = (1ULL << lane) - 1ULL;
#pragma unroll
    for (int rd = 0; rd < IPT; rd++) {
        const uint32_t e = wave * (64 * IPT) + rd * 64 + lane;
        const bool valid = e < nvalid;
        key[rd] = 0;
        val[rd] = 0;
        if (valid) {
            key[rd] = kin[segbase + t0 + e];
            if (HAS_VAL) val[rd] = vin[segbase + t0 + e];
        }
        const uint32_t d = valid ? (uint32_t)(key[rd] >> shift) & mask : 0u;
        dg[rd] = d;
        uint64_t peers = __builtin_amdgcn_ballot_w64(valid);
        for (uint32_t b = 0; b < dbits; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __builtin_amdgcn_ballot_w64(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint64_t lower = peers & lt_mask;
        const uint32_t before = valid ? mycnt[d] : 0u;
        lr[rd] = before + (uint32_t)__popcll(lower);
        if (valid && lower == 0) mycnt[d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // ---- digit starts inside the tile, and each wave's first position of
    // each digit (NB / BLK consecutive digits per thread)
    {
        const uint32_t per = (NB + BLK - 1) / BLK;
        const uint32_t d0 = threadIdx.x * per;
        uint32_t sum = 0;
        for (uint32_t q = 0; q < per; q++)
            if (d0 + q < NB)
#pragma unroll
                for (int w = 0; w < NWAVE; w++) sum += wcnt[w * NB + d0 + q];
        uint32_t total;
        uint32_t ex = block_exclusive_scan(sum, scan_tmp, total);
        for (uint32_t q = 0; q < per; q++)
            if (d0 + q < NB) {
                lstart[d0 + q] = ex;
#pragma unroll
                for (int w = 0; w < NWAVE; w++) {
                    const uint32_t c = wcnt[w * NB + d0 + q];
                    wcnt[w * NB + d0 + q] = ex;
                    ex += c;
                }
            }
    }
    __syncthreads();
    // ---- digit-ordered tile in LDS
#pragma unroll
    for (int rd = 0; rd < IPT; rd++) {
        const uint32_t e = wave * (64 * IPT) + rd * 64 + lane;
        if (e < nvalid) {
            const uint32_t lpos = mycnt[dg[rd]] + lr[rd];
            lkey[lpos] = key[rd];
            if (HAS_VAL) lval[lpos] = val[rd];
        }
    }
    __syncthreads();
    // ---- write out in digit order
#pragma unroll
    for (int rd = 0; rd < IPT; rd++) {
        const uint32_t i = rd * BLK + threadIdx.x;
        if (i < nvalid) {
            const K k = lkey[i];
            const uint32_t d = (uint32_t)(k >> shift) & mask;
            const uint32_t pos = base_off[d] + (i - lstart[d]);
            kout[pos] = k;
            if (HAS_VAL) vout[pos] = lval[i];
        }
    }
}

template <typename K, bool HAS_VAL>
void radix_sort_impl(ej_ctx *ctx, K *kin, uint32_t *vin, K *kout, uint32_t *vout, uint32_t nseg,
                     uint32_t seglen, uint32_t key_bits, uint32_t dbits) {
    uint64_t n = (uint64_t)nseg * seglen;
    if (n == 0) return;
    // widest digit whose staged scatter fits the LDS of one workgroup
    uint32_t dmax = 11;
    while (dmax > 4 && (3 + NWAVE) * 4 * ((size_t)1 << dmax) + (size_t)TILE * (sizeof(K) + 4) >
                           (size_t)ctx->lds_max)
        dmax--;
    if (dbits < 4) dbits = 4;
    if (dbits > dmax) dbits = dmax;
    uint32_t passes = (key_bits + dbits - 1) / dbits;
    // an odd number of passes ends in kout: take one pass fewer with wider
    // digits when they stay within dmax bits; otherwise the first pass writes
    // a scratch buffer, so that an even count ends in kout too
    bool via_tmp = false;
    if (passes > 0 && passes % 2 == 0) {
        if ((key_bits + passes - 2) / (passes - 1) <= dmax)
            passes -= 1;
        else
            via_tmp = true;
    }
    // bits split as evenly as possible: the first key_bits % passes passes
    // take one bit more
    if (passes > 0) dbits = (key_bits + passes - 1) / passes;
    if (passes == 0) {
        EJ_HIP(hipMemcpyAsync(kout, kin, n * sizeof(K), hipMemcpyDeviceToDevice, ctx->stream));
        if (HAS_VAL)
            EJ_HIP(hipMemcpyAsync(vout, vin, n * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                  ctx->stream));
        return;
    }
    // passes alternate kin -> kout -> kin ... (odd count), or kin -> tmp ->
    // kout -> tmp ... (even count): the last one writes kout
    uint32_t tps = ceil_div(seglen, TILE);
    uint32_t NB = 1u << dbits;
    uint64_t hn = (uint64_t)nseg * NB * tps;
    uint32_t *hist = ws<uint32_t>(ctx, "rs_hist", hn);
    K *a = kin, *b = kout;
    uint32_t *va = vin, *vb = vout;
    if (via_tmp) {
        b = ws<K>(ctx, "rs_tmp_keys", n);
        if (HAS_VAL) vb = ws<uint32_t>(ctx, "rs_tmp_vals", n);
    }
    size_t hist_lds = NB * sizeof(uint32_t);
    size_t scat_lds = (3 + NWAVE) * NB * sizeof(uint32_t) + (size_t)TILE * (sizeof(K) + 4);
    if (scat_lds > (size_t)ctx->lds_max) fail(EJ_EUNSUPPORTED, "radix sort: digit too wide for LDS");
    if (scat_lds > 65536)
        EJ_HIP(hipFuncSetAttribute((const void *)k_rs_scatter<K, HAS_VAL>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)scat_lds));
    const uint32_t base_bits = key_bits / passes, extra = key_bits % passes;
    uint32_t shift = 0;
    for (uint32_t p = 0; p < passes; p++) {
        const uint32_t db = base_bits + (p < extra ? 1u : 0u);
        hipLaunchKernelGGL(k_rs_hist<K>, dim3(nseg * tps), dim3(BLK), hist_lds, ctx->stream,
                           (const K *)a, seglen, tps, shift, db, hist);
        EJ_CHECK_LAUNCH();
        scan_exclusive<uint32_t>(ctx, hist, hist, (uint64_t)nseg * (1u << db) * tps, nullptr,
                                 "rs");
        hipLaunchKernelGGL((k_rs_scatter<K, HAS_VAL>), dim3(nseg * tps), dim3(BLK), scat_lds,
                           ctx->stream, (const K *)a, (const uint32_t *)va, b, vb, seglen, tps,
                           shift, db, (const uint32_t *)hist);
        EJ_CHECK_LAUNCH();
        shift += db;
        K *t = a;
        a = b;
        b = (via_tmp && p == 0) ? kout : t;
        uint32_t *tv = va;
        va = vb;
        vb = (via_tmp && p == 0) ? vout : tv;
    }
}

}  // namespace

void scan_exclusive_u32(ej_ctx *ctx, const uint32_t *d_in, uint32_t *d_out, uint64_t n,
                        uint64_t *d_total) {
    scan_exclusive<uint32_t>(ctx, d_in, d_out, n, d_total, "u32");
}

void scan_exclusive_u64(ej_ctx *ctx, const uint64_t *d_in, uint64_t *d_out, uint64_t n,
                        uint64_t *d_total) {
    scan_exclusive<uint64_t>(ctx, d_in, d_out, n, d_total, "u64");
}

void radix_sort_u32(ej_ctx *ctx, uint32_t *keys_in, uint32_t *vals_in, uint32_t *keys_out,
                    uint32_t *vals_out, uint32_t nseg, uint32_t seglen, uint32_t key_bits,
                    uint32_t digit_bits) {
    if (vals_in)
        radix_sort_impl<uint32_t, true>(ctx, keys_in, vals_in, keys_out, vals_out, nseg, seglen,
                                        key_bits, digit_bits);
    else
        radix_sort_impl<uint32_t, false>(ctx, keys_in, nullptr, keys_out, nullptr, nseg, seglen,
                                         key_bits, digit_bits);
}

void radix_sort_u64_kv(ej_ctx *ctx, uint64_t *keys_in, uint32_t *vals_in, uint64_t *keys_out,
                       uint32_t *vals_out, uint32_t nseg, uint32_t seglen, uint32_t key_bits,
                       uint32_t digit_bits) {
    radix_sort_impl<uint64_t, true>(ctx, keys_in, vals_in, keys_out, vals_out, nseg, seglen,
                                    key_bits, digit_bits);
}

void radix_sort_u64(ej_ctx *ctx, uint64_t *keys_in, uint64_t *keys_out, uint64_t n,
                    uint32_t key_bits, uint32_t digit_bits) {
    if (n > 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "radix_sort_u64: more than 2^32 keys");
    radix_sort_impl<uint64_t, false>(ctx, keys_in, nullptr, keys_out, nullptr, 1, (uint32_t)n,
                                     key_bits, digit_bits);
}

}  // namespace ej
