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

// Full keys of every table in length order, for exact buckets.
__global__ void k_bucket_gather_full(const uint64_t *__restrict__ keys,
                                     const uint32_t *__restrict__ perm, uint32_t n, uint64_t tot,
                                     uint64_t *__restrict__ fk, uint32_t *__restrict__ ids) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t t = e / n;
        const uint32_t id = perm[(uint32_t)(e - t * n)];
        fk[e] = keys[t * n + id];
        ids[e] = id;
    }
}

template <typename D>
__global__ void k_group_flags(const D *__restrict__ dk, uint32_t n, uint64_t tot,
                              uint32_t *__restrict__ flags) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        bool f = (e % n == 0) || dk[e] != dk[e - 1];
        flags[e] = f ? 1u : 0u;
    }
}

// gid[e] = inclusive group index; gstart[g] = first entry of group g.
template <typename D>
__global__ void k_group_starts(const D *__restrict__ dk, uint32_t n, uint64_t tot,
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

// ---- pair walk over groups told apart by the sorted top key bits dk
//
// The same pairs as k_pairs over gid/gstart, in another deterministic order
// (the de-duplication that follows does not depend on it).  An entry whose
// successor in its table has other top bits is alone in its group and reads
// nothing else.  Entry indexes are 32-bit (the bucketing keeps T*n below
// 2^32).

// Full key and length of the entries that share their top bits with a
// neighbour in their table; the others are never read by the walk.
__global__ void k_sorted_attrs_dk(const uint64_t *__restrict__ keys,
                                  const uint32_t *__restrict__ ids,
                                  const uint32_t *__restrict__ len,
                                  const uint32_t *__restrict__ dk, uint32_t n, uint32_t tot,
                                  uint64_t *__restrict__ key_s, uint32_t *__restrict__ len_s) {
    for (uint64_t e64 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e64 < tot;
         e64 += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t e = (uint32_t)e64;
        const uint32_t t = e / n, s0 = t * n, s1 = s0 + n;
        const uint32_t d = dk[e];
        const bool grouped = (e > s0 && dk[e - 1] == d) || (e + 1 < s1 && dk[e + 1] == d);
        if (!grouped) continue;
        const uint32_t id = ids[e];
        key_s[e] = keys[(uint64_t)t * n + id];
        len_s[e] = len[id];
    }
}

// How the pair walk codes what it finds.  The join: entries are strings and
// a pair is (min << B | max).  EmbedJoin+ (Algorithm 5): entry e is suffix
// e % kappa of string e / kappa; two suffixes of one string never pair, and a
// pair is the tuple (string a, string b, suffix of a, suffix of b), a < b,
// coded as a << (B + 2 KB) | b << 2 KB | ka << KB | kb.
struct PairCoder {
    uint32_t B;
    __device__ bool pairs(uint32_t, uint32_t) const { return true; }
    __device__ uint64_t code(uint32_t x, uint32_t y) const {
        const uint32_t a = min(x, y), b = max(x, y);
        return ((uint64_t)a << B) | b;
    }
};
// The join's pairs whose smaller index lies in [lo, hi): the candidate stage
// in passes over ranges of the first index when the raw pairs of the whole
// join would not fit one sort (their codes are PairCoder's).
struct RangeCoder {
    uint32_t B, lo, hi;
    __device__ bool pairs(uint32_t x, uint32_t y) const {
        const uint32_t a = min(x, y);
        return a >= lo && a < hi;
    }
    __device__ uint64_t code(uint32_t x, uint32_t y) const {
        const uint32_t a = min(x, y), b = max(x, y);
        return ((uint64_t)a << B) | b;
    }
};
struct TupleCoder {
    uint32_t B, kappa, KB;
    __device__ bool pairs(uint32_t x, uint32_t y) const { return x / kappa != y / kappa; }
    __device__ uint64_t code(uint32_t x, uint32_t y) const {
        const uint32_t sx = x / kappa, sy = y / kappa;
        const uint32_t kx = x - sx * kappa, ky = y - sy * kappa;
        const bool swap = sy < sx;
        const uint64_t a = swap ? sy : sx, b = swap ? sx : sy;
        const uint64_t ka = swap ? ky : kx, kb = swap ? kx : ky;
        return (a << (B + 2 * KB)) | (b << (2 * KB)) | (ka << KB) | kb;
    }
};

// The window of entry e (its table ends at send, its top bits are d): the
// following entries with top bits d and length at most lim.  A table's
// entries are sorted by (top bits, length), so the window is the run
// [e + 1, e + 1 + W) and membership is monotone along the table: doubling
// steps, then bisection, find W in O(log W) reads.
__device__ inline uint32_t pw_window(uint32_t e, uint32_t d, uint32_t send, uint64_t lim,
                                     const uint32_t *__restrict__ dk,
                                     const uint32_t *__restrict__ len_s) {
    auto in = [&](uint64_t q) {
        return q < send && dk[q] == d && (uint64_t)len_s[q] <= lim;
    };
    uint64_t lo = e, step = 1;  // every q in (e, lo] is in the window
    while (in(lo + step)) {
        lo += step;
        step *= 2;
    }
    uint64_t hi = lo + step;  // not in the window
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (in(mid))
            lo = mid;
        else
            hi = mid;
    }
    return (uint32_t)(lo - e);
}

constexpr uint32_t PW_WAVES = 4;        // waves per workgroup of the light walk
constexpr uint32_t PW_LIGHT = 64;       // windows up to this size: the light walk
constexpr uint32_t PW_SEG = 64 * 64;    // positions per heavy task (64 sweeps of a wave)

// Light walk: one wave per 64 consecutive entries, one per lane.  The lanes
// find their windows (pw_window); windows of at most PW_LIGHT positions are
// then run by the whole wave, laid end to end, 64 positions at a time:
// position f belongs to the lane whose window covers it (bisection over the
// wave's inclusive scan of window sizes, read across lanes) and is a pair
// when the entry there has the owner's full key (and, for tuples, is a
// suffix of another string).  Loads of consecutive positions are
// consecutive entries, and the pairs are written contiguously (ballot and
// popcount give the slots).  Longer windows are cut into tasks of PW_SEG
// positions for k_pairs_heavy, so no wave runs more than 64 sweeps.
// EMIT = false: wlen[e] = the window size, cnt[w] = the wave's light pairs,
// ntask[w] = the wave's heavy tasks.
// EMIT = true: writes the light pairs from cur[w] (the exclusive scan of the
// wave totals, light and heavy) and leaves cur[w] just past them, where
// k_pairs_heavy continues.  Nothing at or past cap is written (a buffer
// sized before the count may be too small: the caller sees the count and
// redoes the join).
template <bool EMIT, typename C, typename Coder>
__global__ void __launch_bounds__(256)
    k_pairs_dk(const uint32_t *__restrict__ dk, const uint64_t *__restrict__ key_s,
               const uint32_t *__restrict__ len_s, const uint32_t *__restrict__ ids, uint32_t n,
               uint32_t tot, uint32_t K, Coder coder, uint32_t *__restrict__ wlen,
               uint64_t *__restrict__ cnt, uint32_t *__restrict__ ntask,
               uint64_t *__restrict__ cur, C *__restrict__ out, uint64_t cap) {
    constexpr bool ALWAYS = std::is_same<Coder, PairCoder>::value;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wv = blockIdx.x * PW_WAVES + (threadIdx.x >> 6);
    const uint64_t rbase = (uint64_t)wv * 64;
    const uint64_t e64 = rbase + lane;
    const uint32_t e = (uint32_t)e64;
    uint32_t W = 0;
    if (e64 < tot) {
        if (EMIT) {
            W = wlen[e];
        } else {
            const uint32_t send = (e / n + 1) * n;
            const uint32_t d = dk[e];
            if (e + 1 < send && dk[e + 1] == d)
                W = pw_window(e, d, send, (uint64_t)len_s[e] + K, dk, len_s);
            wlen[e] = W;
        }
    }
    const uint32_t Wl = W <= PW_LIGHT ? W : 0u;
    if (!EMIT) {
        uint32_t tasks = W > PW_LIGHT ? (W + PW_SEG - 1) / PW_SEG : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tasks += __shfl_xor(tasks, o, 64);
        if (lane == 0 && rbase < tot) ntask[wv] = tasks;
    }
    uint32_t incl = Wl;  // at most 64 * PW_LIGHT
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const uint32_t y = __shfl_up(incl, (unsigned)s, 64);
        if (lane >= (uint32_t)s) incl += y;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    uint64_t o = 0, c = 0;
    if (EMIT && rbase < tot) o = cur[wv];
    if (total) {
        const uint64_t ke = Wl ? key_s[e] : 0;
        const uint32_t ide = (Wl && (EMIT || !ALWAYS)) ? ids[e] : 0u;
        for (uint32_t b = 0; b < total; b += 64) {
            const uint32_t f = b + lane;
            // owner: the number of lanes whose windows end at or before f
            uint32_t j = 0;
#pragma unroll
            for (uint32_t s = 32; s > 0; s >>= 1)
                if ((uint32_t)__shfl(incl, (int)(j + s - 1), 64) <= f) j += s;
            j = min(j, 63u);
            const uint32_t jend = __shfl(incl, (int)j, 64);
            const uint32_t jw = __shfl(Wl, (int)j, 64);
            const uint64_t kj = __shfl(ke, (int)j, 64);
            const uint32_t idj = (EMIT || !ALWAYS) ? __shfl(ide, (int)j, 64) : 0u;
            bool hit = false;
            uint32_t idq = 0;
            if (f < total) {
                const uint64_t q = rbase + j + 1 + (f - (jend - jw));
                if (key_s[q] == kj) {
                    if (EMIT || !ALWAYS) {
                        idq = ids[q];
                        hit = coder.pairs(idj, idq);
                    } else {
                        hit = true;
                    }
                }
            }
            const uint64_t m = __ballot(hit);
            if (EMIT) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const uint64_t slot = o + below;
                if (hit && slot < cap) out[slot] = (C)coder.code(idj, idq);
                o += (uint64_t)__popcll(m);
            } else {
                c += (uint64_t)__popcll(m);
            }
        }
    }
    if (lane == 0 && rbase < tot) {
        if (EMIT)
            cur[wv] = o;
        else
            cnt[wv] = c;
    }
}

// Heavy tasks: task t of the tasks numbered wave by wave (tbase = exclusive
// scan of the per-wave task counts, ntot = their total) is segment s of the
// window of one entry: positions [s * PW_SEG, min(W, (s + 1) * PW_SEG)).
// Each wave of a persistent grid takes tasks t = its index, + the number of
// waves: the task's wave by bisection over tbase, its lane and segment by
// bisection over that wave's inclusive scan of task counts (read across
// lanes).  All positions of a task share one owner.
// EMIT = false: each task adds its pairs to cnt[w].
// EMIT = true: a first sweep marks the pairs (one bit per sweep per lane),
// one atomic on cur[w] reserves their slots, a second sweep writes them; the
// slots of a wave's tasks follow its light pairs, in the order the tasks
// reserve them.  A task total of 2^32 or more (impossible below 2^32 window
// positions) poisons cnt[0] so that the caller's count is out of range.
template <bool EMIT, typename C, typename Coder>
__global__ void __launch_bounds__(256)
    k_pairs_heavy(const uint64_t *__restrict__ key_s, const uint32_t *__restrict__ ids,
                  uint32_t tot, Coder coder, const uint32_t *__restrict__ wlen,
                  const uint32_t *__restrict__ tbase, uint32_t nw,
                  const uint64_t *__restrict__ ntot, uint64_t *__restrict__ cnt,
                  uint64_t *__restrict__ cur, C *__restrict__ out, uint64_t cap) {
    constexpr bool ALWAYS = std::is_same<Coder, PairCoder>::value;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nt = *ntot;
    const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t ngw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    if (nt >> 32) {
        if (!EMIT && gw == 0 && lane == 0) atomicAdd(cnt, 1ull << 40);
        return;
    }
    for (uint64_t t = gw; t < nt; t += ngw) {
        // the wave: the last w with tbase[w] <= t
        uint32_t lo = 0, hi = nw - 1;
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo + 1) / 2;
            if ((uint64_t)tbase[mid] <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint32_t w = lo;
        const uint64_t e64 = (uint64_t)w * 64 + lane;
        const uint32_t W = e64 < tot ? wlen[e64] : 0u;
        const uint32_t segs = W > PW_LIGHT ? (W + PW_SEG - 1) / PW_SEG : 0u;
        uint32_t incl = segs;
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const uint32_t y = __shfl_up(incl, (unsigned)s, 64);
            if (lane >= (uint32_t)s) incl += y;
        }
        const uint32_t local = (uint32_t)(t - tbase[w]);
        uint32_t j = 0;
#pragma unroll
        for (uint32_t s = 32; s > 0; s >>= 1)
            if ((uint32_t)__shfl(incl, (int)(j + s - 1), 64) <= local) j += s;
        j = min(j, 63u);
        const uint32_t seg = local - ((uint32_t)__shfl(incl, (int)j, 64) -
                                      (uint32_t)__shfl(segs, (int)j, 64));
        const uint32_t Wj = (uint32_t)__shfl(W, (int)j, 64);
        const uint64_t ej = (uint64_t)w * 64 + j;
        const uint64_t kj = key_s[ej];
        const uint32_t idj = (EMIT || !ALWAYS) ? ids[ej] : 0u;
        const uint32_t p0 = seg * PW_SEG;
        const uint32_t p1 = min(Wj, p0 + PW_SEG);
        uint64_t bits = 0, c = 0;
        for (uint32_t it = 0; p0 + it * 64 < p1; it++) {
            const uint32_t p = p0 + it * 64 + lane;
            bool hit = false;
            if (p < p1) {
                const uint64_t q = ej + 1 + p;
                if (key_s[q] == kj) hit = ALWAYS ? true : coder.pairs(idj, ids[q]);
            }
            bits |= (uint64_t)hit << it;
            c += (uint64_t)__popcll(__ballot(hit));
        }
        if (!EMIT) {
            if (lane == 0 && c) atomicAdd(&cnt[w], c);
            continue;
        }
        if (c == 0) continue;
        uint64_t o = 0;
        if (lane == 0) o = atomicAdd(&cur[w], c);
        o = __shfl(o, 0, 64);
        for (uint32_t it = 0; p0 + it * 64 < p1; it++) {
            const bool hit = (bits >> it) & 1ull;
            const uint64_t m = __ballot(hit);
            if (hit) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const uint64_t slot = o + below;
                if (slot < cap) out[slot] = (C)coder.code(idj, ids[ej + 1 + p0 + it * 64 + lane]);
            }
            o += (uint64_t)__popcll(m);
        }
    }
}

// Buffers of the pair walk over nw = ceil(tot / 64) waves.
struct PairWalk {
    uint32_t *wlen, *ntask, *tbase;
    uint64_t *cnt, *ntot;
    uint32_t nw, nwg;
};

PairWalk pw_buffers(ej_ctx *ctx, const std::string &t, uint64_t tot) {
    PairWalk pw;
    pw.nw = (uint32_t)((tot + 63) / 64);
    pw.nwg = (pw.nw + PW_WAVES - 1) / PW_WAVES;
    pw.wlen = ws<uint32_t>(ctx, t + "_wlen", tot);
    pw.ntask = ws<uint32_t>(ctx, t + "_ntask", pw.nw);
    pw.tbase = ws<uint32_t>(ctx, t + "_tbase", pw.nw);
    pw.cnt = ws<uint64_t>(ctx, t + "_counts", pw.nw);
    pw.ntot = ws<uint64_t>(ctx, t + "_ntasks", 1);
    return pw;
}

uint32_t pw_heavy_grid(ej_ctx *ctx) { return (uint32_t)ctx->num_cu * 8; }

// Counting pass: window sizes, per-wave pair counts, and their exclusive
// scan in place (cnt becomes the waves' first slots); the total pairs go to
// d_total.
template <typename Coder>
void pw_count(ej_ctx *ctx, const PairWalk &pw, const uint32_t *dk, const uint64_t *key_s,
              const uint32_t *len_s, const uint32_t *ids, uint32_t n, uint32_t tot, uint32_t K,
              const Coder &coder, uint64_t *d_total) {
    hipLaunchKernelGGL((k_pairs_dk<false, uint64_t, Coder>), dim3(pw.nwg), dim3(256), 0,
                       ctx->stream, dk, key_s, len_s, ids, n, tot, K, coder, pw.wlen, pw.cnt,
                       pw.ntask, (uint64_t *)nullptr, (uint64_t *)nullptr, (uint64_t)0);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, pw.ntask, pw.tbase, pw.nw, pw.ntot);
    hipLaunchKernelGGL((k_pairs_heavy<false, uint64_t, Coder>), dim3(pw_heavy_grid(ctx)),
                       dim3(256), 0, ctx->stream, key_s, ids, tot, coder,
                       (const uint32_t *)pw.wlen, (const uint32_t *)pw.tbase, pw.nw,
                       (const uint64_t *)pw.ntot, pw.cnt, (uint64_t *)nullptr,
                       (uint64_t *)nullptr, (uint64_t)0);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u64(ctx, pw.cnt, pw.cnt, pw.nw, d_total);
}

// Emitting pass (after pw_count on the same buffers): the pairs into out,
// nothing at or past cap.
template <typename C, typename Coder>
void pw_emit(ej_ctx *ctx, const PairWalk &pw, const uint32_t *dk, const uint64_t *key_s,
             const uint32_t *len_s, const uint32_t *ids, uint32_t n, uint32_t tot, uint32_t K,
             const Coder &coder, C *out, uint64_t cap) {
    hipLaunchKernelGGL((k_pairs_dk<true, C, Coder>), dim3(pw.nwg), dim3(256), 0, ctx->stream, dk,
                       key_s, len_s, ids, n, tot, K, coder, pw.wlen, (uint64_t *)nullptr,
                       (uint32_t *)nullptr, pw.cnt, out, cap);
    EJ_CHECK_LAUNCH();
    hipLaunchKernelGGL((k_pairs_heavy<true, C, Coder>), dim3(pw_heavy_grid(ctx)), dim3(256), 0,
                       ctx->stream, key_s, ids, tot, coder, (const uint32_t *)pw.wlen,
                       (const uint32_t *)pw.tbase, pw.nw, (const uint64_t *)pw.ntot,
                       (uint64_t *)nullptr, pw.cnt, out, cap);
    EJ_CHECK_LAUNCH();
}

// EmbedJoin+ tuple counts: in the sorted tuple codes, a run of equal codes
// is one tuple and its length is the number of tables that found it.  Flags
// the first entry of each run of at least T entries (the run is sorted, so
// its T-th entry decides).
__global__ void k_tuple_qualify(const uint64_t *__restrict__ t, uint64_t cnt, uint32_t T,
                                uint32_t *__restrict__ flags) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t c = t[e];
        const bool start = e == 0 || t[e - 1] != c;
        flags[e] = (start && e + T - 1 < cnt && t[e + T - 1] == c) ? 1u : 0u;
    }
}

// The pair code (a << B | b) of every flagged tuple, at its scanned position;
// the result is sorted (the tuples were) and may repeat a pair.
__global__ void k_tuple_pairs(const uint64_t *__restrict__ t, uint64_t cnt, uint32_t shift,
                              const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos,
                              uint64_t *__restrict__ out) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x)
        if (flags[e]) out[pos[e]] = t[e] >> shift;
}

// cnt_dev: a count on the device; past cnt the entries were never written,
// so then nothing is flagged (the host sees the count and redoes the join)
template <typename C>
__global__ void k_unique_flags(const C *__restrict__ codes, uint64_t cnt,
                               const uint64_t *__restrict__ cnt_dev,
                               uint32_t *__restrict__ flags) {
    const uint64_t live = cnt_dev ? (*cnt_dev > cnt ? 0 : *cnt_dev) : cnt;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x)
        flags[e] = (e < live && (e == 0 || codes[e] != codes[e - 1])) ? 1u : 0u;
}

// Entries past the count on the device get the largest code, which no pair
// has (a < b), so that a sort of the whole buffer leaves them at the end.
template <typename C>
__global__ void k_pad_codes(C *__restrict__ codes, uint64_t cap,
                            const uint64_t *__restrict__ cnt_dev, C pad) {
    const uint64_t from = min(*cnt_dev, cap);
    for (uint64_t e = from + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cap;
         e += (uint64_t)gridDim.x * blockDim.x)
        codes[e] = pad;
}

template <typename C>
__global__ void k_unique_compact(const C *__restrict__ codes, uint64_t cnt, uint32_t B,
                                 const uint32_t *__restrict__ flags,
                                 const uint32_t *__restrict__ pos, uint64_t *__restrict__ out,
                                 uint32_t *__restrict__ first, uint64_t cap) {
    const uint64_t mask = (1ULL << B) - 1ULL;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < cnt;
         e += (uint64_t)gridDim.x * blockDim.x) {
        if (flags[e] && pos[e] < cap) {
            const uint64_t c = codes[e];
            out[pos[e]] = ((c >> B) << 32) | (c & mask);
            if (first) first[pos[e]] = (uint32_t)e;
        }
    }
}

// Partitioned de-duplication.  The raw codes (2B bits) are grouped by their
// top GB bits (k_group_count / k_group_place), which leaves each code's low
// 2B - GB <= 31 bits as a 32-bit local code; one workgroup per group then
// collects the group's distinct local codes and their multiplicities in an
// LDS hash table and ranks them, so that the groups in order and each group's
// codes in rank order are the distinct codes sorted.  A group with more than
// DD_UCAP distinct codes sets *overflow and the caller sorts the raw codes
// instead.
constexpr uint32_t DD_HCAP = 4096;  // hash slots per group (a power of two)
constexpr uint32_t DD_UCAP = 1024;  // distinct codes per group handled here
constexpr uint32_t DD_EMPTY = 0xFFFFFFFFu;  // never a local code (< 2^31)

__global__ void __launch_bounds__(256)
    k_dedup_groups(const uint32_t *__restrict__ codes, const uint32_t *__restrict__ gstart,
                   uint32_t *__restrict__ ucode, uint32_t *__restrict__ umult,
                   uint32_t *__restrict__ ucount, uint32_t *__restrict__ overflow) {
    __shared__ uint32_t hk[DD_HCAP], hc[DD_HCAP], lk[DD_UCAP], lc[DD_UCAP];
    __shared__ uint32_t nuniq, npos, bad;
    const uint32_t g = blockIdx.x, tid = threadIdx.x;
    for (uint32_t i = tid; i < DD_HCAP; i += 256) {
        hk[i] = DD_EMPTY;
        hc[i] = 0;
    }
    if (tid == 0) {
        nuniq = 0;
        npos = 0;
        bad = 0;
    }
    __syncthreads();
    const uint32_t b = gstart[g], e = gstart[g + 1];
    for (uint32_t i = b + tid; i < e; i += 256) {
        if (nuniq > DD_UCAP) break;  // this group goes to the fallback anyway
        const uint32_t c = codes[i];
        uint32_t h = (c * 0x9E3779B1u) >> 20;  // 12 bits
        uint32_t probe = 0;
        for (;;) {
            const uint32_t old = atomicCAS(&hk[h], DD_EMPTY, c);
            if (old == DD_EMPTY) atomicAdd(&nuniq, 1u);
            if (old == DD_EMPTY || old == c) {
                atomicAdd(&hc[h], 1u);
                break;
            }
            if (++probe >= DD_HCAP) {
                bad = 1u;
                break;
            }
            h = (h + 1) & (DD_HCAP - 1);
        }
    }
    __syncthreads();
    const uint32_t u = nuniq;
    if (u > DD_UCAP || bad) {
        if (tid == 0) {
            atomicOr(overflow, 1u);
            ucount[g] = 0;
        }
        return;
    }
    for (uint32_t i = tid; i < DD_HCAP; i += 256)
        if (hk[i] != DD_EMPTY) {
            const uint32_t j = atomicAdd(&npos, 1u);
            lk[j] = hk[i];
            lc[j] = hc[i];
        }
    __syncthreads();
    for (uint32_t i = tid; i < u; i += 256) {
        const uint32_t c = lk[i];
        uint32_t r = 0;
        for (uint32_t j = 0; j < u; j++) r += lk[j] < c ? 1u : 0u;
        ucode[(uint64_t)g * DD_UCAP + r] = c;
        umult[(uint64_t)g * DD_UCAP + r] = lc[i];
    }
    if (tid == 0) ucount[g] = u;
}

// Grouping of the raw codes by their top GB bits (GB <= DD_GBITS), not
// stable: each workgroup counts the groups of its chunk of DD_CHUNK codes in
// LDS (k_group_count, hist[g * nwg + wg]); after an exclusive scan of the
// counts it places the low `shift` bits of its codes from LDS cursors
// (k_group_place).
constexpr uint32_t DD_GBITS = 11;
constexpr uint32_t DD_CHUNK = 16384;

template <typename C>
__global__ void __launch_bounds__(256)
    k_group_count(const C *__restrict__ codes, uint32_t n, const uint64_t *__restrict__ n_dev,
                  uint32_t shift, uint32_t NG, uint32_t *__restrict__ hist) {
    __shared__ uint32_t cnt[1u << DD_GBITS];
    const uint32_t wg = blockIdx.x, nwg = gridDim.x;
    // a count on the device: past n the buffer holds unwritten entries, so
    // then nothing is grouped (the host sees the count and redoes the join)
    if (n_dev) n = *n_dev > n ? 0u : (uint32_t)*n_dev;
    for (uint32_t g = threadIdx.x; g < NG; g += 256) cnt[g] = 0;
    __syncthreads();
    const uint32_t b = wg * DD_CHUNK, e = min(n, b + DD_CHUNK);
    for (uint32_t i = b + threadIdx.x; i < e; i += 256)
        atomicAdd(&cnt[(uint32_t)(codes[i] >> shift)], 1u);
    __syncthreads();
    for (uint32_t g = threadIdx.x; g < NG; g += 256) hist[(uint64_t)g * nwg + wg] = cnt[g];
}

template <typename C>
__global__ void __launch_bounds__(256)
    k_group_place(const C *__restrict__ codes, uint32_t n, const uint64_t *__restrict__ n_dev,
                  uint32_t shift, uint32_t NG, const uint32_t *__restrict__ offs,
                  uint32_t *__restrict__ out) {
    __shared__ uint32_t cur[1u << DD_GBITS];
    const uint32_t wg = blockIdx.x, nwg = gridDim.x;
    if (n_dev) n = *n_dev > n ? 0u : (uint32_t)*n_dev;  // as in k_group_count
    for (uint32_t g = threadIdx.x; g < NG; g += 256) cur[g] = offs[(uint64_t)g * nwg + wg];
    __syncthreads();
    const uint32_t b = wg * DD_CHUNK, e = min(n, b + DD_CHUNK);
    const C low = ((C)1 << shift) - 1;
    for (uint32_t i = b + threadIdx.x; i < e; i += 256) {
        const C c = codes[i];
        out[atomicAdd(&cur[(uint32_t)(c >> shift)], 1u)] = (uint32_t)(c & low);
    }
}

// First position of group g: the scanned count of its first chunk.
__global__ void k_group_first(const uint32_t *__restrict__ offs, uint32_t nwg, uint32_t NG,
                              uint32_t n, const uint64_t *__restrict__ n_dev,
                              uint32_t *__restrict__ gstart) {
    if (n_dev) n = *n_dev > n ? 0u : (uint32_t)*n_dev;  // as in k_group_count
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g <= NG; g += gridDim.x * blockDim.x)
        gstart[g] = g < NG ? offs[(uint64_t)g * nwg] : n;
}

// The groups' distinct codes at their scanned offsets, rebuilt from the group
// and the local code and unpacked to (a << 32 | b); the multiplicities
// alongside when `mult` is given.
__global__ void k_dedup_out(const uint32_t *__restrict__ ucode, const uint32_t *__restrict__ umult,
                            const uint32_t *__restrict__ ucount, const uint32_t *__restrict__ uoff,
                            uint32_t B, uint32_t shift, uint64_t *__restrict__ out,
                            uint32_t *__restrict__ mult, uint64_t cap) {
    const uint32_t g = blockIdx.x;
    const uint32_t o = uoff[g];
    // nothing past `cap` (a buffer sized before the count; the host redoes
    // the join when the count exceeds it)
    const uint32_t m = o >= cap ? 0u : (uint32_t)min<uint64_t>(ucount[g], cap - o);
    const uint64_t mask = (1ull << B) - 1ull;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
        const uint64_t c = ((uint64_t)g << shift) | ucode[(uint64_t)g * DD_UCAP + i];
        out[o + i] = ((c >> B) << 32) | (c & mask);
        if (mult) mult[o + i] = umult[(uint64_t)g * DD_UCAP + i];
    }
}

// Order key of unique pair u from its multiplicity (see k_mult_keys).
__global__ void k_mult_keys_direct(const uint32_t *__restrict__ mult, uint64_t cnt,
                                   const uint64_t *__restrict__ cnt_dev, uint32_t cap,
                                   uint32_t *__restrict__ key, uint32_t *__restrict__ idx) {
    // with a count on the device, the entries past it get the key cap, which
    // no real pair has (m >= 1): a stable sort leaves them behind all real ones
    const uint64_t live = cnt_dev ? min(*cnt_dev, cnt) : cnt;
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < cnt;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t m = u < live ? mult[u] : 0u;
        key[u] = cap - (m < cap ? m : cap);
        idx[u] = (uint32_t)u;
    }
}

// Sort key of unique pair u: cap - (number of raw copies), so that an
// ascending sort puts the most frequent pairs first.  A pair has at most one
// raw copy per table, so cap = 2^bits_for(tables) - 1 keeps every count
// apart in bits_for(tables) key bits.
__global__ void k_mult_keys(const uint32_t *__restrict__ first, uint64_t cnt, uint64_t raw,
                            const uint64_t *__restrict__ cnt_dev,
                            const uint64_t *__restrict__ raw_dev, uint32_t cap,
                            uint32_t *__restrict__ key, uint32_t *__restrict__ idx,
                            uint64_t ibase = 0) {
    // counts on the device: entries past the distinct count get the key cap,
    // which no real pair has (m >= 1), and sort behind all real ones
    const uint64_t live = cnt_dev ? min(*cnt_dev, cnt) : cnt;
    if (raw_dev) raw = *raw_dev;
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < cnt;
         u += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t m = 0;
        if (u < live) m = (u + 1 < live ? first[u + 1] : raw) - first[u];
        key[u] = cap - (uint32_t)(m < cap ? m : cap);
        idx[u] = (uint32_t)(ibase + u);
    }
}

}  // namespace

uint32_t bucket_key_bits(ej_ctx *ctx, uint32_t n, uint32_t key_bits) {
    if (key_bits == 0) key_bits = ctx->tune.bucket_key_bits;
    // enough bits that different keys rarely share a group (the pair scan
    // compares full keys, so a shared group costs time, never results)
    if (key_bits == 0) key_bits = std::min(32u, bits_for(n) + 6);
    return std::min(key_bits, 32u);
}

void bucket_inputs(ej_ctx *ctx, uint64_t tot, const char *tag, uint32_t **d_dk, uint32_t **d_ids) {
    if (tot >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "r*z*n must stay below 2^32");
    std::string t(tag);
    *d_dk = ws<uint32_t>(ctx, t + "_dk", tot);
    *d_ids = ws<uint32_t>(ctx, t + "_ids0", tot);
}

void bucket(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_len, const uint32_t *d_perm,
            uint32_t n, uint32_t T, uint32_t key_bits, Buckets &bk, const char *tag,
            bool want_ngroups, bool inputs_ready, bool want_groups) {
    std::string t(tag);
    bk.T = T;
    bk.n = n;
    uint64_t tot = (uint64_t)T * n;
    if (tot >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "r*z*n must stay below 2^32");
    key_bits = bucket_key_bits(ctx, n, key_bits);
    bk.d_ids = ws<uint32_t>(ctx, t + "_ids", tot);
    bk.d_gid = nullptr;
    bk.d_gstart = nullptr;
    bk.d_dk = nullptr;
    bk.ngroups = 0;
    if (want_groups) {
        bk.d_gid = ws<uint32_t>(ctx, t + "_gid", tot);
        bk.d_gstart = ws<uint32_t>(ctx, t + "_gstart", tot + 1);
    }
    if (tot == 0) {
        if (!want_groups) return;
        uint32_t zero = 0;
        EJ_HIP(hipMemcpyAsync(bk.d_gstart, &zero, 4, hipMemcpyHostToDevice, ctx->stream));
        sync(ctx);
        return;
    }
    uint32_t *dk = nullptr, *ids0 = nullptr;
    bucket_inputs(ctx, tot, tag, &dk, &ids0);
    uint32_t *dk2 = ws<uint32_t>(ctx, t + "_dk2", tot);
    if (!inputs_ready) {
        hipLaunchKernelGGL(k_bucket_gather, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                           ctx->stream, d_keys, d_perm, n, tot, 61u - key_bits, dk, ids0);
        EJ_CHECK_LAUNCH();
    }
    radix_sort_u32(ctx, dk, ids0, dk2, bk.d_ids, T, n, key_bits, ctx->tune.radix_bits);
    if (!want_groups) {
        bk.d_dk = dk2;
        return;
    }
    uint32_t *flags = ws<uint32_t>(ctx, t + "_flags", tot);
    uint64_t *d_ng = ws<uint64_t>(ctx, t + "_ngroups", 1);
    hipLaunchKernelGGL(k_group_flags<uint32_t>, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                       ctx->stream, (const uint32_t *)dk2, n, tot, flags);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, flags, flags, tot, d_ng);
    hipLaunchKernelGGL(k_group_starts<uint32_t>, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                       ctx->stream, (const uint32_t *)dk2, n, tot, (const uint32_t *)flags,
                       bk.d_gid, bk.d_gstart, (const uint64_t *)d_ng);
    EJ_CHECK_LAUNCH();
    if (want_ngroups) read_back(ctx, d_ng, 8, &bk.ngroups);
}

void bucket_exact(ej_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_perm, uint32_t n,
                  uint32_t T, Buckets &bk, const char *tag) {
    std::string t(tag);
    bk.T = T;
    bk.n = n;
    bk.d_dk = nullptr;
    bk.ngroups = 0;
    const uint64_t tot = (uint64_t)T * n;
    if (tot >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "r*z*n must stay below 2^32");
    bk.d_ids = ws<uint32_t>(ctx, t + "_ids", tot);
    bk.d_gid = ws<uint32_t>(ctx, t + "_gid", tot);
    bk.d_gstart = ws<uint32_t>(ctx, t + "_gstart", tot + 1);
    if (tot == 0) {
        uint32_t zero = 0;
        EJ_HIP(hipMemcpyAsync(bk.d_gstart, &zero, 4, hipMemcpyHostToDevice, ctx->stream));
        sync(ctx);
        return;
    }
    uint64_t *fk = ws<uint64_t>(ctx, t + "_fk", tot);
    uint64_t *fk2 = ws<uint64_t>(ctx, t + "_fk2", tot);
    uint32_t *ids0 = ws<uint32_t>(ctx, t + "_ids0", tot);
    hipLaunchKernelGGL(k_bucket_gather_full, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                       ctx->stream, d_keys, d_perm, n, tot, fk, ids0);
    EJ_CHECK_LAUNCH();
    // keys are below 2^61; the stable sort keeps the length order within a key
    radix_sort_u64_kv(ctx, fk, ids0, fk2, bk.d_ids, T, n, 61, ctx->tune.radix_bits);
    uint32_t *flags = ws<uint32_t>(ctx, t + "_flags", tot);
    uint64_t *d_ng = ws<uint64_t>(ctx, t + "_ngroups", 1);
    hipLaunchKernelGGL(k_group_flags<uint64_t>, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                       ctx->stream, (const uint64_t *)fk2, n, tot, flags);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, flags, flags, tot, d_ng);
    hipLaunchKernelGGL(k_group_starts<uint64_t>, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                       ctx->stream, (const uint64_t *)fk2, n, tot, (const uint32_t *)flags,
                       bk.d_gid, bk.d_gstart, (const uint64_t *)d_ng);
    EJ_CHECK_LAUNCH();
    read_back(ctx, d_ng, 8, &bk.ngroups);
}

// The candidate stage in passes over ranges [lo, hi) of the pairs' smaller
// index: a range's raw pairs are counted (a pass of the pair walk that keeps
// only its pairs), halved while they exceed `lim`, then emitted, sorted and
// made unique into the output from the running offset.  The ranges ascend,
// so the concatenation is sorted like the one-pass result, and equal to it.
// A single index has fewer than n partners, which one sort always takes.
static uint64_t candidates_ranged(ej_ctx *ctx, const PairWalk &pw, const Buckets &bk,
                                  const uint64_t *key_s, const uint32_t *len_s, uint32_t K,
                                  uint32_t B, uint64_t lim, uint32_t mult_bits, uint64_t raw_all,
                                  uint64_t **d_pairs_out, const std::string &t,
                                  uint32_t **d_order_out) {
    const uint32_t n = bk.n;
    const uint64_t tot = (uint64_t)bk.T * n;
    const uint32_t mult_cap = mult_bits >= 32 ? 0xFFFFFFFFu : (1u << mult_bits) - 1u;
    ctx->last_dedup_sorted = true;
    // distinct pairs: at most the raw pairs, and fewer than 2^32 (the
    // verification's pair indexes)
    const uint64_t cap = std::min<uint64_t>(raw_all, 0xFFFFFFFEull);
    uint64_t *pairs = ws<uint64_t>(ctx, t + "_pairs", cap);
    uint32_t *k0 = d_order_out ? ws<uint32_t>(ctx, t + "_okey", cap) : nullptr;
    uint32_t *v0 = d_order_out ? ws<uint32_t>(ctx, t + "_oidx", cap) : nullptr;
    uint64_t *d_r = ws<uint64_t>(ctx, t + "_rraw", 1);
    uint64_t *d_c = ws<uint64_t>(ctx, t + "_rcount", 1);
    const uint32_t *dk = (const uint32_t *)bk.d_dk, *ids = (const uint32_t *)bk.d_ids;
    uint64_t base = 0;
    std::vector<std::pair<uint32_t, uint32_t>> todo{{0u, n}};  // a stack, lowest range on top
    while (!todo.empty()) {
        const auto [lo, hi] = todo.back();
        todo.pop_back();
        const RangeCoder coder{B, lo, hi};
        pw_count(ctx, pw, dk, key_s, len_s, ids, n, (uint32_t)tot, K, coder, d_r);
        uint64_t r = 0;
        read_back(ctx, d_r, 8, &r);
        if (r == 0) continue;
        if (r > lim && hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            todo.push_back({mid, hi});
            todo.push_back({lo, mid});
            continue;
        }
        uint64_t *raw64 = ws<uint64_t>(ctx, t + "_raw", r);
        uint64_t *sorted = ws<uint64_t>(ctx, t + "_raw_sorted", r);
        uint32_t *flags = ws<uint32_t>(ctx, t + "_uflags", r);
        uint32_t *pos = ws<uint32_t>(ctx, t + "_upos", r);
        uint32_t *first = d_order_out ? ws<uint32_t>(ctx, t + "_first", r) : nullptr;
        pw_emit(ctx, pw, dk, key_s, len_s, ids, n, (uint32_t)tot, K, coder, raw64, r);
        radix_sort_u64(ctx, raw64, sorted, r, 2 * B, ctx->tune.radix_bits);
        hipLaunchKernelGGL(k_unique_flags<uint64_t>, dim3(grid_for(ctx, r, 256)), dim3(256), 0,
                           ctx->stream, (const uint64_t *)sorted, r, (const uint64_t *)nullptr,
                           flags);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u32(ctx, flags, pos, r, d_c);
        uint64_t c = 0;
        read_back(ctx, d_c, 8, &c);
        if (base + c > cap)
            fail(EJ_EUNSUPPORTED, "2^32 or more distinct candidate pairs");
        hipLaunchKernelGGL(k_unique_compact<uint64_t>, dim3(grid_for(ctx, r, 256)), dim3(256), 0,
                           ctx->stream, (const uint64_t *)sorted, r, B, (const uint32_t *)flags,
                           (const uint32_t *)pos, pairs + base, first, c);
        EJ_CHECK_LAUNCH();
        if (d_order_out) {
            hipLaunchKernelGGL(k_mult_keys, dim3(grid_for(ctx, c, 256)), dim3(256), 0,
                               ctx->stream, (const uint32_t *)first, c, r,
                               (const uint64_t *)nullptr, (const uint64_t *)nullptr, mult_cap,
                               k0 + base, v0 + base, base);
            EJ_CHECK_LAUNCH();
        }
        base += c;
    }
    *d_pairs_out = pairs;
    if (d_order_out && base) {
        uint32_t *k1 = ws<uint32_t>(ctx, t + "_okey2", base);
        uint32_t *order = ws<uint32_t>(ctx, t + "_order", base);
        radix_sort_u32(ctx, k0, v0, k1, order, 1, (uint32_t)base, mult_bits, 11);
        *d_order_out = order;
    }
    return base;
}

uint64_t candidates(ej_ctx *ctx, const uint64_t *d_keys, const Buckets &bk, const uint32_t *d_len,
                    uint32_t K, uint64_t **d_pairs_out, uint64_t *n_raw, const char *tag,
                    uint32_t **d_order_out) {
    std::string t(tag);
    const uint32_t n = bk.n;
    const uint64_t tot = (uint64_t)bk.T * n;
    ctx->last_dedup_sorted = false;
    *d_pairs_out = ws<uint64_t>(ctx, t + "_pairs", 1);
    if (n_raw) *n_raw = 0;
    if (tot == 0 || n < 2) return 0;
    uint64_t *key_s = ws<uint64_t>(ctx, t + "_key_s", tot);
    uint32_t *len_s = ws<uint32_t>(ctx, t + "_len_s", tot);
    uint64_t *d_raw = ws<uint64_t>(ctx, t + "_nraw", 1);
    const uint32_t B = std::max(1u, bits_for(n - 1));
    // key width of the verification order (multiplicities are at most T)
    const uint32_t mult_bits = std::max(1u, bits_for(bk.T));
    const uint32_t mult_cap = mult_bits >= 32 ? 0xFFFFFFFFu : (1u << mult_bits) - 1u;
    // groups from the sorted top key bits (the join) or from group starts
    const bool by_dk = bk.d_dk != nullptr;
    if (by_dk && tot >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "r*z*n must stay below 2^32");
    uint64_t *counts = nullptr;
    PairWalk pw{};
    if (by_dk) {
        hipLaunchKernelGGL(k_sorted_attrs_dk, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                           ctx->stream, d_keys, (const uint32_t *)bk.d_ids, d_len,
                           (const uint32_t *)bk.d_dk, n, (uint32_t)tot, key_s, len_s);
        EJ_CHECK_LAUNCH();
        pw = pw_buffers(ctx, t, tot);
        pw_count(ctx, pw, (const uint32_t *)bk.d_dk, (const uint64_t *)key_s,
                 (const uint32_t *)len_s, (const uint32_t *)bk.d_ids, n, (uint32_t)tot, K,
                 PairCoder{B}, d_raw);
    } else {
        hipLaunchKernelGGL(k_sorted_attrs, dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                           ctx->stream, d_keys, (const uint32_t *)bk.d_ids, d_len, n, tot, key_s,
                           len_s);
        EJ_CHECK_LAUNCH();
        counts = ws<uint64_t>(ctx, t + "_counts", tot);
        hipLaunchKernelGGL((k_pairs<false, uint64_t>), dim3(grid_for(ctx, tot, 256)), dim3(256),
                           0, ctx->stream, (const uint64_t *)key_s, (const uint32_t *)len_s,
                           (const uint32_t *)bk.d_ids, (const uint32_t *)bk.d_gid,
                           (const uint32_t *)bk.d_gstart, tot, K, B, counts, nullptr,
                           (uint64_t *)nullptr);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u64(ctx, counts, counts, tot, d_raw);
    }
    uint64_t raw = 0;
    read_back(ctx, d_raw, 8, &raw);
    if (n_raw) *n_raw = raw;
    if (raw == 0) return 0;
    // one sort takes fewer than 2^32 raw pairs (32-bit ranks); beyond that
    // (or beyond the raw_limit knob) the join's pairs go in passes
    const uint64_t lim = ctx->tune.raw_limit ? ctx->tune.raw_limit : 0xFFFFFFFEull;
    if (raw > lim && by_dk)
        return candidates_ranged(ctx, pw, bk, key_s, len_s, K, B, lim, mult_bits, raw,
                                 d_pairs_out, t, d_order_out);
    if (raw >= 0xFFFFFFFFull)
        fail(EJ_EUNSUPPORTED, "more than 2^32 raw candidate pairs (" + std::to_string(raw) + ")");
    uint32_t *flags = ws<uint32_t>(ctx, t + "_uflags", raw);
    uint32_t *pos = ws<uint32_t>(ctx, t + "_upos", raw);
    uint64_t *d_cnt = ws<uint64_t>(ctx, t + "_ucount", 1);
    auto emit = [&](auto *rawbuf) {
        using C = std::remove_pointer_t<decltype(rawbuf)>;
        if (by_dk) {
            pw_emit(ctx, pw, (const uint32_t *)bk.d_dk, (const uint64_t *)key_s,
                    (const uint32_t *)len_s, (const uint32_t *)bk.d_ids, n, (uint32_t)tot, K,
                    PairCoder{B}, rawbuf, raw);
            return;
        }
        hipLaunchKernelGGL((k_pairs<true, C>), dim3(grid_for(ctx, tot, 256)), dim3(256), 0,
                           ctx->stream, (const uint64_t *)key_s, (const uint32_t *)len_s,
                           (const uint32_t *)bk.d_ids, (const uint32_t *)bk.d_gid,
                           (const uint32_t *)bk.d_gstart, tot, K, B, (uint64_t *)nullptr,
                           (const uint64_t *)counts, rawbuf);
        EJ_CHECK_LAUNCH();
    };
    // sort the packed codes, keep the first of each run of equal codes; the
    // multiplicity order comes from the runs' first positions
    auto sort_unique = [&](auto *rawbuf, auto *sorted) -> uint64_t {
        using C = std::remove_pointer_t<decltype(rawbuf)>;
        if constexpr (sizeof(C) == 4)
            radix_sort_u32(ctx, rawbuf, nullptr, sorted, nullptr, 1, (uint32_t)raw, 2 * B,
                           ctx->tune.radix_bits);
        else
            radix_sort_u64(ctx, rawbuf, sorted, raw, 2 * B, ctx->tune.radix_bits);
        hipLaunchKernelGGL(k_unique_flags<C>, dim3(grid_for(ctx, raw, 256)), dim3(256), 0,
                           ctx->stream, (const C *)sorted, raw, (const uint64_t *)nullptr, flags);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u32(ctx, flags, pos, raw, d_cnt);
        uint64_t cnt = 0;
        read_back(ctx, d_cnt, 8, &cnt);
        uint64_t *pairs = ws<uint64_t>(ctx, t + "_pairs", cnt);
        uint32_t *first = d_order_out ? ws<uint32_t>(ctx, t + "_first", cnt) : nullptr;
        hipLaunchKernelGGL(k_unique_compact<C>, dim3(grid_for(ctx, raw, 256)), dim3(256), 0,
                           ctx->stream, (const C *)sorted, raw, B, (const uint32_t *)flags,
                           (const uint32_t *)pos, pairs, first, cnt);
        EJ_CHECK_LAUNCH();
        *d_pairs_out = pairs;
        if (d_order_out && cnt) {
            uint32_t *k0 = ws<uint32_t>(ctx, t + "_okey", cnt);
            uint32_t *v0 = ws<uint32_t>(ctx, t + "_oidx", cnt);
            hipLaunchKernelGGL(k_mult_keys, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0,
                               ctx->stream, (const uint32_t *)first, cnt, raw,
                               (const uint64_t *)nullptr, (const uint64_t *)nullptr, mult_cap,
                               k0, v0);
            EJ_CHECK_LAUNCH();
        }
        return cnt;
    };
    uint64_t cnt = 0;
    // grouped de-duplication while the low 2B - GB bits fit 31 bits
    auto grouped = [&](auto *rawbuf, uint32_t *part) -> bool {
        using C = std::remove_pointer_t<decltype(rawbuf)>;
        const uint32_t GB = std::min(DD_GBITS, 2 * B);
        const uint32_t NG = 1u << GB, shift = 2 * B - GB;
        const uint32_t nwg = (uint32_t)((raw + DD_CHUNK - 1) / DD_CHUNK);
        uint32_t *ghist = ws<uint32_t>(ctx, t + "_dd_hist", (uint64_t)NG * nwg);
        uint32_t *gst = ws<uint32_t>(ctx, t + "_dd_gstart", NG + 1);
        hipLaunchKernelGGL(k_group_count<C>, dim3(nwg), dim3(256), 0, ctx->stream,
                           (const C *)rawbuf, (uint32_t)raw, (const uint64_t *)nullptr, shift, NG,
                           ghist);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u32(ctx, ghist, ghist, (uint64_t)NG * nwg, nullptr);
        hipLaunchKernelGGL(k_group_place<C>, dim3(nwg), dim3(256), 0, ctx->stream,
                           (const C *)rawbuf, (uint32_t)raw, (const uint64_t *)nullptr, shift, NG,
                           (const uint32_t *)ghist, part);
        EJ_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_group_first, dim3((NG + 256) / 256), dim3(256), 0, ctx->stream,
                           (const uint32_t *)ghist, nwg, NG, (uint32_t)raw,
                           (const uint64_t *)nullptr, gst);
        EJ_CHECK_LAUNCH();
        uint32_t *ucode = ws<uint32_t>(ctx, t + "_dd_code", (uint64_t)NG * DD_UCAP);
        uint32_t *umult = ws<uint32_t>(ctx, t + "_dd_mult", (uint64_t)NG * DD_UCAP);
        uint32_t *ucnt = ws<uint32_t>(ctx, t + "_dd_count", NG);
        uint32_t *uoff = ws<uint32_t>(ctx, t + "_dd_off", NG);
        uint64_t *info = ws<uint64_t>(ctx, t + "_dd_info", 2);  // distinct codes, overflow
        EJ_HIP(hipMemsetAsync(info, 0, 16, ctx->stream));
        hipLaunchKernelGGL(k_dedup_groups, dim3(NG), dim3(256), 0, ctx->stream,
                           (const uint32_t *)part, (const uint32_t *)gst, ucode, umult, ucnt,
                           (uint32_t *)(info + 1));
        EJ_CHECK_LAUNCH();
        scan_exclusive_u32(ctx, ucnt, uoff, NG, info);
        uint64_t hinfo[2] = {0, 0};
        read_back(ctx, info, 16, hinfo);
        if (hinfo[1] != 0) return false;
        cnt = hinfo[0];
        uint64_t *pairs = ws<uint64_t>(ctx, t + "_pairs", cnt);
        uint32_t *mult = d_order_out ? ws<uint32_t>(ctx, t + "_mult", cnt) : nullptr;
        hipLaunchKernelGGL(k_dedup_out, dim3(NG), dim3(256), 0, ctx->stream,
                           (const uint32_t *)ucode, (const uint32_t *)umult, (const uint32_t *)ucnt,
                           (const uint32_t *)uoff, B, shift, pairs, mult, cnt);
        EJ_CHECK_LAUNCH();
        *d_pairs_out = pairs;
        if (d_order_out && cnt) {
            hipLaunchKernelGGL(k_mult_keys_direct, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0,
                               ctx->stream, (const uint32_t *)mult, cnt,
                               (const uint64_t *)nullptr, mult_cap,
                               ws<uint32_t>(ctx, t + "_okey", cnt),
                               ws<uint32_t>(ctx, t + "_oidx", cnt));
            EJ_CHECK_LAUNCH();
        }
        return true;
    };
    const bool fits_grouped = 2 * B <= DD_GBITS + 31 && ctx->tune.dedup_sort == 0;
    if (2 * B <= 32) {
        // 32-bit codes (both indexes below 2^16)
        uint32_t *raw32 = ws<uint32_t>(ctx, t + "_raw32", raw);
        emit(raw32);
        uint32_t *part = ws<uint32_t>(ctx, t + "_raw32_sorted", raw);
        // on overflow: sort them all (raw32 is intact, the grouping wrote `part`)
        if (!fits_grouped || !grouped(raw32, part)) {
            cnt = sort_unique(raw32, part);
            ctx->last_dedup_sorted = true;
        }
    } else {
        uint64_t *raw64 = ws<uint64_t>(ctx, t + "_raw", raw);
        uint64_t *sorted = ws<uint64_t>(ctx, t + "_raw_sorted", raw);
        emit(raw64);
        // the 32-bit local codes go to the first half of `sorted`, which
        // the fallback sort overwrites only after the grouping has failed
        if (!fits_grouped || !grouped(raw64, (uint32_t *)sorted)) {
            cnt = sort_unique(raw64, sorted);
            ctx->last_dedup_sorted = true;
        }
    }
    if (d_order_out && cnt) {
        uint32_t *k0 = ws<uint32_t>(ctx, t + "_okey", cnt);
        uint32_t *v0 = ws<uint32_t>(ctx, t + "_oidx", cnt);
        uint32_t *k1 = ws<uint32_t>(ctx, t + "_okey2", cnt);
        uint32_t *order = ws<uint32_t>(ctx, t + "_order", cnt);
        radix_sort_u32(ctx, k0, v0, k1, order, 1, (uint32_t)cnt, mult_bits, 11);
        *d_order_out = order;
    }
    return cnt;
}

__global__ void k_zero_u64(uint64_t *__restrict__ p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

// The candidate stage of a join sized on the device (the whole join captured
// as one graph, so nothing may be read back between its kernels): the kernels
// of candidates() with the raw pairs written into a buffer of raw_cap entries
// and the distinct pairs into one of cnt_cap, and the counts left in device
// memory: cnt_dev[0] = raw pairs, cnt_dev[1] = distinct pairs, cnt_dev[2] =
// nonzero when a group of the de-duplication held more distinct codes than it
// takes.  A count above its capacity, or that flag, makes the result invalid:
// the caller reads the counts after the join and redoes it.  The
// de-duplication is the grouped one (2B <= DD_GBITS + 31), or with sort_dedup
// a sort of the whole raw buffer (its entries past the count padded to the
// end), as candidates() falls back to when a group is too large.
void candidates_dev(ej_ctx *ctx, const uint64_t *d_keys, const Buckets &bk,
                    const uint32_t *d_len, uint32_t K, uint64_t raw_cap, uint64_t cnt_cap,
                    bool want_order, bool sort_dedup, uint64_t *cnt_dev, uint64_t **d_pairs_out,
                    uint32_t **d_order_out, const char *tag) {
    std::string t(tag);
    const uint32_t n = bk.n;
    const uint64_t tot = (uint64_t)bk.T * n;
    if (tot == 0 || n < 2 || !bk.d_dk) fail(EJ_EINVAL, "candidates_dev: no tables");
    if (raw_cap >= 0xFFFFFFFFull || cnt_cap >= 0xFFFFFFFFull || tot >= 0xFFFFFFFFull)
        fail(EJ_EUNSUPPORTED, "candidates_dev: capacities must stay below 2^32");
    const uint32_t B = std::max(1u, bits_for(n - 1));
    const uint32_t mult_bits = std::max(1u, bits_for(bk.T));
    const uint32_t mult_cap = mult_bits >= 32 ? 0xFFFFFFFFu : (1u << mult_bits) - 1u;
    uint64_t *key_s = ws<uint64_t>(ctx, t + "_key_s", tot);
    uint32_t *len_s = ws<uint32_t>(ctx, t + "_len_s", tot);
    const PairWalk pw = pw_buffers(ctx, t, tot);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, ctx->stream, cnt_dev + 2, 1u);
    EJ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sorted_attrs_dk, dim3(grid_for(ctx, tot, 256)), dim3(256), 0, ctx->stream,
                       d_keys, (const uint32_t *)bk.d_ids, d_len, (const uint32_t *)bk.d_dk, n,
                       (uint32_t)tot, key_s, len_s);
    EJ_CHECK_LAUNCH();
    pw_count(ctx, pw, (const uint32_t *)bk.d_dk, (const uint64_t *)key_s, (const uint32_t *)len_s,
             (const uint32_t *)bk.d_ids, n, (uint32_t)tot, K, PairCoder{B}, cnt_dev);
    if (sort_dedup) {
        // the whole raw buffer sorted (padding at the end), one of each run
        uint32_t *flags = ws<uint32_t>(ctx, t + "_uflags", raw_cap);
        uint32_t *pos = ws<uint32_t>(ctx, t + "_upos", raw_cap);
        uint64_t *pairs = ws<uint64_t>(ctx, t + "_pairs", cnt_cap);
        uint32_t *first = want_order ? ws<uint32_t>(ctx, t + "_first", cnt_cap) : nullptr;
        auto sorted_unique = [&](auto *rawbuf, auto *sorted) {
            using C = std::remove_pointer_t<decltype(rawbuf)>;
            pw_emit(ctx, pw, (const uint32_t *)bk.d_dk, (const uint64_t *)key_s,
                    (const uint32_t *)len_s, (const uint32_t *)bk.d_ids, n, (uint32_t)tot, K,
                    PairCoder{B}, rawbuf, raw_cap);
            const C pad = (C)((2 * B >= 64 ? ~0ull : (1ull << (2 * B)) - 1ull));
            hipLaunchKernelGGL(k_pad_codes<C>, dim3(grid_for(ctx, raw_cap, 256)), dim3(256), 0,
                               ctx->stream, rawbuf, raw_cap, (const uint64_t *)cnt_dev, pad);
            EJ_CHECK_LAUNCH();
            if constexpr (sizeof(C) == 4)
                radix_sort_u32(ctx, rawbuf, nullptr, sorted, nullptr, 1, (uint32_t)raw_cap, 2 * B,
                               ctx->tune.radix_bits);
            else
                radix_sort_u64(ctx, rawbuf, sorted, raw_cap, 2 * B, ctx->tune.radix_bits);
            hipLaunchKernelGGL(k_unique_flags<C>, dim3(grid_for(ctx, raw_cap, 256)), dim3(256), 0,
                               ctx->stream, (const C *)sorted, raw_cap, (const uint64_t *)cnt_dev,
                               flags);
            EJ_CHECK_LAUNCH();
            scan_exclusive_u32(ctx, flags, pos, raw_cap, cnt_dev + 1);
            hipLaunchKernelGGL(k_unique_compact<C>, dim3(grid_for(ctx, raw_cap, 256)), dim3(256),
                               0, ctx->stream, (const C *)sorted, raw_cap, B,
                               (const uint32_t *)flags, (const uint32_t *)pos, pairs, first,
                               cnt_cap);
            EJ_CHECK_LAUNCH();
        };
        if (2 * B <= 32)
            sorted_unique(ws<uint32_t>(ctx, t + "_raw32", raw_cap),
                          ws<uint32_t>(ctx, t + "_raw32_sorted", raw_cap));
        else
            sorted_unique(ws<uint64_t>(ctx, t + "_raw", raw_cap),
                          ws<uint64_t>(ctx, t + "_raw_sorted", raw_cap));
        *d_pairs_out = pairs;
        *d_order_out = nullptr;
        if (want_order) {
            uint32_t *k0 = ws<uint32_t>(ctx, t + "_okey", cnt_cap);
            uint32_t *v0 = ws<uint32_t>(ctx, t + "_oidx", cnt_cap);
            uint32_t *k1 = ws<uint32_t>(ctx, t + "_okey2", cnt_cap);
            uint32_t *order = ws<uint32_t>(ctx, t + "_order", cnt_cap);
            hipLaunchKernelGGL(k_mult_keys, dim3(grid_for(ctx, cnt_cap, 256)), dim3(256), 0,
                               ctx->stream, (const uint32_t *)first, cnt_cap, raw_cap,
                               (const uint64_t *)(cnt_dev + 1), (const uint64_t *)cnt_dev,
                               mult_cap, k0, v0);
            EJ_CHECK_LAUNCH();
            radix_sort_u32(ctx, k0, v0, k1, order, 1, (uint32_t)cnt_cap, mult_bits, 11);
            *d_order_out = order;
        }
        return;
    }
    if (2 * B > DD_GBITS + 31) fail(EJ_EUNSUPPORTED, "candidates_dev: codes too wide to group");
    const uint32_t GB = std::min(DD_GBITS, 2 * B);
    const uint32_t NG = 1u << GB, shift = 2 * B - GB;
    const uint32_t nwd = (uint32_t)((raw_cap + DD_CHUNK - 1) / DD_CHUNK);
    uint32_t *ghist = ws<uint32_t>(ctx, t + "_dd_hist", (uint64_t)NG * nwd);
    uint32_t *gst = ws<uint32_t>(ctx, t + "_dd_gstart", NG + 1);
    auto group = [&](auto *rawbuf, uint32_t *part) {
        using C = std::remove_pointer_t<decltype(rawbuf)>;
        pw_emit(ctx, pw, (const uint32_t *)bk.d_dk, (const uint64_t *)key_s,
                (const uint32_t *)len_s, (const uint32_t *)bk.d_ids, n, (uint32_t)tot, K,
                PairCoder{B}, rawbuf, raw_cap);
        hipLaunchKernelGGL(k_group_count<C>, dim3(nwd), dim3(256), 0, ctx->stream,
                           (const C *)rawbuf, (uint32_t)raw_cap, (const uint64_t *)cnt_dev, shift,
                           NG, ghist);
        EJ_CHECK_LAUNCH();
        scan_exclusive_u32(ctx, ghist, ghist, (uint64_t)NG * nwd, nullptr);
        hipLaunchKernelGGL(k_group_place<C>, dim3(nwd), dim3(256), 0, ctx->stream,
                           (const C *)rawbuf, (uint32_t)raw_cap, (const uint64_t *)cnt_dev, shift,
                           NG, (const uint32_t *)ghist, part);
        EJ_CHECK_LAUNCH();
    };
    uint32_t *part = nullptr;
    if (2 * B <= 32) {
        uint32_t *raw32 = ws<uint32_t>(ctx, t + "_raw32", raw_cap);
        part = ws<uint32_t>(ctx, t + "_raw32_sorted", raw_cap);
        group(raw32, part);
    } else {
        uint64_t *raw64 = ws<uint64_t>(ctx, t + "_raw", raw_cap);
        part = (uint32_t *)ws<uint64_t>(ctx, t + "_raw_sorted", raw_cap);
        group(raw64, part);
    }
    hipLaunchKernelGGL(k_group_first, dim3((NG + 256) / 256), dim3(256), 0, ctx->stream,
                       (const uint32_t *)ghist, nwd, NG, (uint32_t)raw_cap,
                       (const uint64_t *)cnt_dev, gst);
    EJ_CHECK_LAUNCH();
    uint32_t *ucode = ws<uint32_t>(ctx, t + "_dd_code", (uint64_t)NG * DD_UCAP);
    uint32_t *umult = ws<uint32_t>(ctx, t + "_dd_mult", (uint64_t)NG * DD_UCAP);
    uint32_t *ucnt = ws<uint32_t>(ctx, t + "_dd_count", NG);
    uint32_t *uoff = ws<uint32_t>(ctx, t + "_dd_off", NG);
    hipLaunchKernelGGL(k_dedup_groups, dim3(NG), dim3(256), 0, ctx->stream, (const uint32_t *)part,
                       (const uint32_t *)gst, ucode, umult, ucnt, (uint32_t *)(cnt_dev + 2));
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, ucnt, uoff, NG, cnt_dev + 1);
    uint64_t *pairs = ws<uint64_t>(ctx, t + "_pairs", cnt_cap);
    uint32_t *mult = want_order ? ws<uint32_t>(ctx, t + "_mult", cnt_cap) : nullptr;
    hipLaunchKernelGGL(k_dedup_out, dim3(NG), dim3(256), 0, ctx->stream, (const uint32_t *)ucode,
                       (const uint32_t *)umult, (const uint32_t *)ucnt, (const uint32_t *)uoff, B,
                       shift, pairs, mult, cnt_cap);
    EJ_CHECK_LAUNCH();
    *d_pairs_out = pairs;
    *d_order_out = nullptr;
    if (want_order) {
        uint32_t *k0 = ws<uint32_t>(ctx, t + "_okey", cnt_cap);
        uint32_t *v0 = ws<uint32_t>(ctx, t + "_oidx", cnt_cap);
        uint32_t *k1 = ws<uint32_t>(ctx, t + "_okey2", cnt_cap);
        uint32_t *order = ws<uint32_t>(ctx, t + "_order", cnt_cap);
        hipLaunchKernelGGL(k_mult_keys_direct, dim3(grid_for(ctx, cnt_cap, 256)), dim3(256), 0,
                           ctx->stream, (const uint32_t *)mult, cnt_cap,
                           (const uint64_t *)(cnt_dev + 1), mult_cap, k0, v0);
        EJ_CHECK_LAUNCH();
        radix_sort_u32(ctx, k0, v0, k1, order, 1, (uint32_t)cnt_cap, mult_bits, 11);
        *d_order_out = order;
    }
}

// EmbedJoin+ candidates (Algorithm 5): the bucketed entries are suffixes
// (entry e = suffix e % kappa of string e / kappa, lengths those of the whole
// strings).  Every pair of entries of different strings in one bucket of a
// table within K in length is a tuple (a, b, ka, kb); the tuples are counted
// over all tables by sorting their codes, and a pair whose some tuple occurs
// at least T times is a candidate.
uint64_t candidates_plus(ej_ctx *ctx, const uint64_t *d_keys, const Buckets &bk,
                         const uint32_t *d_len_entry, uint32_t K, uint32_t nstr, uint32_t kappa,
                         uint32_t T, uint64_t **d_pairs_out, uint64_t *n_raw, const char *tag) {
    std::string t(tag);
    const uint32_t ne = bk.n;
    const uint64_t tot = (uint64_t)bk.T * ne;
    *d_pairs_out = ws<uint64_t>(ctx, t + "_pairs", 1);
    if (n_raw) *n_raw = 0;
    if (tot == 0 || nstr < 2 || !bk.d_dk) return 0;
    if (tot >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "r*z*n*kappa must stay below 2^32");
    const uint32_t B = std::max(1u, bits_for(nstr - 1));
    const uint32_t KB = std::max(1u, bits_for(kappa - 1));
    if (2 * B + 2 * KB > 64) fail(EJ_EUNSUPPORTED, "tuple codes wider than 64 bits");
    const TupleCoder coder{B, kappa, KB};
    uint64_t *key_s = ws<uint64_t>(ctx, t + "_key_s", tot);
    uint32_t *len_s = ws<uint32_t>(ctx, t + "_len_s", tot);
    uint64_t *d_raw = ws<uint64_t>(ctx, t + "_nraw", 1);
    hipLaunchKernelGGL(k_sorted_attrs_dk, dim3(grid_for(ctx, tot, 256)), dim3(256), 0, ctx->stream,
                       d_keys, (const uint32_t *)bk.d_ids, d_len_entry, (const uint32_t *)bk.d_dk,
                       ne, (uint32_t)tot, key_s, len_s);
    EJ_CHECK_LAUNCH();
    const PairWalk pw = pw_buffers(ctx, t, tot);
    pw_count(ctx, pw, (const uint32_t *)bk.d_dk, (const uint64_t *)key_s, (const uint32_t *)len_s,
             (const uint32_t *)bk.d_ids, ne, (uint32_t)tot, K, coder, d_raw);
    uint64_t raw = 0;
    read_back(ctx, d_raw, 8, &raw);
    if (n_raw) *n_raw = raw;
    if (raw == 0) return 0;
    if (raw >= 0xFFFFFFFFull)
        fail(EJ_EUNSUPPORTED, "more than 2^32 candidate tuples (" + std::to_string(raw) + ")");
    uint64_t *tup = ws<uint64_t>(ctx, t + "_tuples", raw);
    uint64_t *sorted = ws<uint64_t>(ctx, t + "_tuples_sorted", raw);
    pw_emit(ctx, pw, (const uint32_t *)bk.d_dk, (const uint64_t *)key_s, (const uint32_t *)len_s,
            (const uint32_t *)bk.d_ids, ne, (uint32_t)tot, K, coder, tup, raw);
    radix_sort_u64(ctx, tup, sorted, raw, 2 * B + 2 * KB, ctx->tune.radix_bits);
    uint32_t *flags = ws<uint32_t>(ctx, t + "_tflags", raw);
    uint32_t *pos = ws<uint32_t>(ctx, t + "_tpos", raw);
    uint64_t *d_n = ws<uint64_t>(ctx, t + "_tcount_q", 1);
    hipLaunchKernelGGL(k_tuple_qualify, dim3(grid_for(ctx, raw, 256)), dim3(256), 0, ctx->stream,
                       (const uint64_t *)sorted, raw, T, flags);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, flags, pos, raw, d_n);
    uint64_t nq = 0;
    read_back(ctx, d_n, 8, &nq);
    if (nq == 0) return 0;
    // the qualifying tuples' pair codes, sorted, then one of each pair
    uint64_t *q = tup;  // the unsorted tuples are no longer needed
    hipLaunchKernelGGL(k_tuple_pairs, dim3(grid_for(ctx, raw, 256)), dim3(256), 0, ctx->stream,
                       (const uint64_t *)sorted, raw, 2 * KB, (const uint32_t *)flags,
                       (const uint32_t *)pos, q);
    EJ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_unique_flags<uint64_t>, dim3(grid_for(ctx, nq, 256)), dim3(256), 0,
                       ctx->stream, (const uint64_t *)q, nq, (const uint64_t *)nullptr, flags);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, flags, pos, nq, d_n);
    uint64_t cnt = 0;
    read_back(ctx, d_n, 8, &cnt);
    uint64_t *pairs = ws<uint64_t>(ctx, t + "_pairs", cnt);
    hipLaunchKernelGGL(k_unique_compact<uint64_t>, dim3(grid_for(ctx, nq, 256)), dim3(256), 0,
                       ctx->stream, (const uint64_t *)q, nq, B, (const uint32_t *)flags,
                       (const uint32_t *)pos, pairs, (uint32_t *)nullptr, cnt);
    EJ_CHECK_LAUNCH();
    *d_pairs_out = pairs;
    return cnt;
}

uint64_t unique_sorted_pairs(ej_ctx *ctx, const uint64_t *d_sorted, uint64_t cnt, uint32_t B,
                             uint64_t **d_out, const char *tag) {
    std::string t(tag);
    *d_out = ws<uint64_t>(ctx, t + "_upairs", 1);
    if (cnt == 0) return 0;
    if (cnt >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "more than 2^32 pairs to de-duplicate");
    uint32_t *flags = ws<uint32_t>(ctx, t + "_uflags", cnt);
    uint32_t *pos = ws<uint32_t>(ctx, t + "_upos", cnt);
    uint64_t *d_n = ws<uint64_t>(ctx, t + "_ucnt", 1);
    hipLaunchKernelGGL(k_unique_flags<uint64_t>, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0,
                       ctx->stream, d_sorted, cnt, (const uint64_t *)nullptr, flags);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, flags, pos, cnt, d_n);
    uint64_t u = 0;
    read_back(ctx, d_n, 8, &u);
    uint64_t *out = ws<uint64_t>(ctx, t + "_upairs", u);
    hipLaunchKernelGGL(k_unique_compact<uint64_t>, dim3(grid_for(ctx, cnt, 256)), dim3(256), 0,
                       ctx->stream, d_sorted, cnt, B, (const uint32_t *)flags,
                       (const uint32_t *)pos, out, (uint32_t *)nullptr, u);
    EJ_CHECK_LAUNCH();
    *d_out = out;
    return u;
}

}  // namespace ej
