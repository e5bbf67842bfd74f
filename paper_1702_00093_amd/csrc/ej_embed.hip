// Stages A0-A2: preparation of a string set (alphabet, lengths, encodings,
// length order), the counter-based random streams, and the CGK walk with
// sparse sampling and two-level hashing.
//
// CGK embedding (Algorithm 1) truncated to L symbols (Section 4.1): a pointer
// i starts on the first character; step j emits x[i] (or the padding symbol
// once i is past the end) and advances i iff pi_j(x[i]) = 1.  Only the
// symbols at the z*m LSH coordinates of the seed are needed (Section 4,
// sparse embedding), so a walk stops after its last sampled step.
//
// GPU mapping: one lane per (string, seed); a workgroup is one wave of 64
// strings that share a seed, taken in length order so that the walks of a
// wave have similar lengths.  Because the seed is shared, the sampled steps
// and the pi bits of every step are wave-uniform: the pi bits are read with
// scalar loads and the "is this step sampled" test is a scalar branch that
// is taken for whole groups of steps at once.  The strings of the wave are
// staged in LDS as packed symbol codes (2, 4 or 8 bits), each lane reading a
// 32-bit window of codes per group of steps.
#include <string.h>

#include <algorithm>

#include "ej_internal.h"

namespace ej {

namespace {

struct PrepInfo {
    uint32_t mask[8];   // presence bitmap of bytes
    uint32_t maxlen;
    uint32_t minlen;
    uint32_t err;       // 1: offsets decrease, 2: string longer than 2^31-1
    uint64_t off0, offn;
};

__global__ void k_prep_info(const uint64_t *__restrict__ offsets, uint32_t n,
                            PrepInfo *__restrict__ info) {
    if (threadIdx.x == 0) {
        info->off0 = offsets[0];
        info->offn = offsets[n];
    }
    if (threadIdx.x < 8) info->mask[threadIdx.x] = 0;
    if (threadIdx.x == 8) info->maxlen = 0;
    if (threadIdx.x == 9) info->err = 0;
    if (threadIdx.x == 10) info->minlen = 0xFFFFFFFFu;
}

__global__ void k_lengths(const uint64_t *__restrict__ offsets, uint32_t n,
                          uint32_t *__restrict__ len, PrepInfo *__restrict__ info) {
    uint32_t mx = 0, mn = 0xFFFFFFFFu, err = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint64_t a = offsets[i], b = offsets[i + 1];
        uint64_t l = 0;
        if (b < a)
            err |= 1u;
        else
            l = b - a;
        if (l > 0x7FFFFFFFull) {
            err |= 2u;
            l = 0;
        }
        len[i] = (uint32_t)l;
        mx = l > mx ? (uint32_t)l : mx;
        mn = l < mn ? (uint32_t)l : mn;
    }
    // wave reduction then one atomic per wave
    for (int d = 32; d >= 1; d >>= 1) {
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
        mn = min(mn, (uint32_t)__shfl_xor((int)mn, d, 64));
        err |= (uint32_t)__shfl_xor((int)err, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (mx) atomicMax(&info->maxlen, mx);
        if (mn != 0xFFFFFFFFu) atomicMin(&info->minlen, mn);
        if (err) atomicOr(&info->err, err);
    }
}

// Presence bitmap of the bytes in [base, base+total): 16-byte loads over the
// aligned body, single bytes for the unaligned head and tail.
__global__ void k_presence(const uint8_t *__restrict__ chars, PrepInfo *__restrict__ info) {
    // [base, base+total) from the offsets (k_prep_info ran first on the stream);
    // decreasing offsets are reported through info->err and scan nothing here
    const uint64_t base = info->off0;
    const uint64_t total = info->offn >= info->off0 ? info->offn - info->off0 : 0;
    __shared__ uint32_t m[8];
    if (threadIdx.x < 8) m[threadIdx.x] = 0;
    __syncthreads();
    const uint8_t *p = chars + base;
    const uint64_t start = (uint64_t)(uintptr_t)p;
    uint64_t head = ((start + 15) & ~15ull) - start;
    if (head > total) head = total;
    const uint64_t nbody = (total - head) / 16;
    const uint64_t tail0 = head + nbody * 16;
    uint32_t loc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = tid; k < head; k += nth) {
        uint32_t byte = p[k];
        loc[byte >> 5] |= 1u << (byte & 31);
    }
    for (uint64_t k = tail0 + tid; k < total; k += nth) {
        uint32_t byte = p[k];
        loc[byte >> 5] |= 1u << (byte & 31);
    }
    // the body: bytes 64..127 (letters) go to a 64-bit register mask without
    // branches; any other byte to the block's LDS mask, one atomic each
    const uint4 *body = (const uint4 *)(p + head);
    uint64_t letters = 0;
    for (uint64_t c = tid; c < nbody; c += nth) {
        uint4 v = body[c];
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const uint32_t byte = (w[q >> 2] >> ((q & 3) * 8)) & 0xFFu;
            const bool letter = (byte >> 6) == 1u;
            letters |= letter ? (1ull << (byte & 63)) : 0ull;
            if (!letter) atomicOr(&m[byte >> 5], 1u << (byte & 31));
        }
    }
    loc[2] |= (uint32_t)letters;
    loc[3] |= (uint32_t)(letters >> 32);
#pragma unroll
    for (int q = 0; q < 8; q++)
        if (loc[q]) atomicOr(&m[q], loc[q]);
    __syncthreads();
    // most blocks find nothing new: read first, so that the device-wide
    // word sees one atomic per new bit pattern instead of one per block
    if (threadIdx.x < 8 && (m[threadIdx.x] & ~__atomic_load_n(&info->mask[threadIdx.x], __ATOMIC_RELAXED)))
        atomicOr(&info->mask[threadIdx.x], m[threadIdx.x]);
}

// One pass over the characters: thread w maps characters w*CPD ..
// w*CPD+CPD-1 through the alphabet table, stores their codes (as whole
// dwords: CPD is a multiple of 4; the last dword's bytes past the end are 0)
// and their packed word; threads nwords .. nwords+7 write the zero padding:
// 8 packed words, which the walk may read past the end, and 64 code bytes.
template <int BW>
__global__ void k_encode_pack(const uint8_t *__restrict__ chars, uint64_t base, uint64_t total,
                              const uint8_t *__restrict__ lut_g, uint8_t *__restrict__ codes,
                              uint64_t nwords, uint32_t *__restrict__ packed) {
    constexpr int CPD = 32 / BW;
    __shared__ uint8_t lut[256];
    lut[threadIdx.x & 255] = lut_g[threadIdx.x & 255];
    __syncthreads();
    const uint8_t *p = chars + base;
    for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < nwords + 8;
         w += (uint64_t)gridDim.x * blockDim.x) {
        if (w >= nwords) {
            // zero padding: 8 packed words, and the 64 code bytes after the
            // text that the verification's text window may read
            packed[w] = 0;
            const uint64_t pad0 = ((total + 3) & ~3ull) + 8 * (w - nwords);
            uint32_t *cp = (uint32_t *)(codes + pad0);
            cp[0] = 0;
            cp[1] = 0;
            continue;
        }
        const uint64_t k0 = w * CPD;
        uint32_t x = 0;
        uint32_t cw[CPD / 4];
#pragma unroll
        for (int q = 0; q < CPD / 4; q++) cw[q] = 0;
        if (k0 + CPD + 4 <= total) {
            // a whole word with 4 more characters after it: its characters in
            // aligned dwords, funnel-shifted, every read inside the text
            const uint32_t mis = (uint32_t)((uintptr_t)(p + k0) & 3);
            const uint32_t *b4 = (const uint32_t *)(p + k0 - mis);
            const uint32_t sh = mis * 8;
            uint32_t d[CPD / 4 + 1];
#pragma unroll
            for (int q = 0; q < CPD / 4; q++) d[q] = b4[q];
            d[CPD / 4] = sh ? b4[CPD / 4] : 0u;
#pragma unroll
            for (int q = 0; q < CPD / 4; q++) {
                const uint32_t ch = __builtin_amdgcn_alignbit(d[q + 1], d[q], sh);
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const uint32_t c = lut[(ch >> (8 * j)) & 0xFFu];
                    x |= c << ((4 * q + j) * BW);
                    cw[q] |= c << (8 * j);
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < CPD; t++) {
                if (k0 + t < total) {
                    const uint32_t c = lut[p[k0 + t]];
                    x |= c << (t * BW);
                    cw[t >> 2] |= c << (8 * (t & 3));
                }
            }
        }
        packed[w] = x;
        uint32_t *cd = (uint32_t *)(codes + k0);
#pragma unroll
        for (int q = 0; q < CPD / 4; q++)
            if (k0 + 4 * q < total) cd[q] = cw[q];
    }
}

__global__ void k_iota(uint32_t *__restrict__ a, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        a[i] = i;
}

// ------------------------------------------------------------ randomness --

// Rwords[l][w]: 32-bit word w of the random string R^l (bit b of R^l is
// bit b%32 of word b/32, i.e. bit b%64 of the 64-bit word b/64).
__global__ void k_draw_R(uint64_t seed, uint32_t r, uint32_t nw, uint32_t *__restrict__ Rwords) {
    uint64_t tot = (uint64_t)r * nw;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t l = (uint32_t)(e / nw), w = (uint32_t)(e % nw);
        uint64_t key = stream_key(seed, TAG_R, l);
        uint64_t word = rng_word(key, w >> 1);
        Rwords[e] = (uint32_t)(word >> (32 * (w & 1)));
    }
}

// Rstep[l][j]: the sigma bits pi_j(.) of step j, code c at bit c.
__global__ void k_rstep(const uint32_t *__restrict__ Rwords, uint32_t nw, uint32_t r,
                        uint32_t Lpad, uint32_t L, uint32_t sigma, uint32_t *__restrict__ Rstep) {
    uint64_t tot = (uint64_t)r * Lpad;
    uint32_t mask = sigma >= 32 ? 0xFFFFFFFFu : ((1u << sigma) - 1u);
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < tot;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t l = (uint32_t)(e / Lpad), j = (uint32_t)(e % Lpad);
        uint32_t val = 0;
        if (j < L) {
            uint64_t b0 = (uint64_t)j * sigma;
            uint32_t w = (uint32_t)(b0 >> 5), sh = (uint32_t)(b0 & 31);
            const uint32_t *R = Rwords + (size_t)l * nw;
            uint32_t lo = R[w], hi = R[w + 1];
            val = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & mask;
        }
        Rstep[e] = val;
    }
}

// Coordinates and second-level vectors of every table (l, j).
__global__ void k_draw_lsh(uint64_t seed, uint32_t r, uint32_t z, uint32_t m, uint32_t L,
                           uint32_t *__restrict__ pos, uint64_t *__restrict__ v, int draw_pos,
                           int draw_v) {
    uint32_t tot = r * z * m;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
        uint32_t tbl = e / m, k = e % m;
        if (draw_pos) {
            uint64_t kp = stream_key(seed, TAG_POS, tbl);
            pos[e] = (uint32_t)__umul64hi(rng_word(kp, k), (uint64_t)L);
        }
        if (draw_v) {
            uint64_t kv = stream_key(seed, TAG_V, tbl);
            v[e] = (rng_word(kv, k) >> 3) % P61;
        }
    }
}

// Per seed: the z*m samples (step, slot j*m+k) in ascending (step, slot)
// order, and J = last sampled step + 1.  Rank by counting (S is small).
__global__ void k_sample_sort(const uint32_t *__restrict__ pos, uint32_t S,
                              uint32_t *__restrict__ spos, uint32_t *__restrict__ sslot,
                              uint32_t *__restrict__ J) {
    uint32_t l = blockIdx.x;
    const uint32_t *p = pos + (size_t)l * S;
    __shared__ uint32_t mx;
    if (threadIdx.x == 0) mx = 0;
    __syncthreads();
    uint32_t lmx = 0;
    for (uint32_t e = threadIdx.x; e < S; e += blockDim.x) {
        uint32_t pe = p[e];
        uint32_t rank = 0;
        for (uint32_t f = 0; f < S; f++) {
            uint32_t pf = p[f];
            rank += (pf < pe) || (pf == pe && f < e);
        }
        spos[(size_t)l * S + rank] = pe;
        sslot[(size_t)l * S + rank] = e;
        lmx = max(lmx, pe + 1);
    }
    atomicMax(&mx, lmx);
    __syncthreads();
    if (threadIdx.x == 0) J[l] = mx;
}

// --------------------------------------------------------------- the walk --

// REC = true (walks of at most EMBED_REC_STEPS steps): every step's symbol
// is recorded in LDS (Lb bytes per lane) and the samples are read from the
// record through the sample positions when the keys are formed, so the walk
// itself never looks at the sample list.  REC = false: the walk stores each
// sampled symbol as it passes the sample's step (the positions sorted, one
// scalar read per sample).
constexpr uint32_t EMBED_REC_STEPS = 256;

template <int BW, bool RSTEP, bool REC>
__global__ void __launch_bounds__(64)
    k_embed(const uint32_t *__restrict__ packed, const uint64_t *__restrict__ offsets,
            uint64_t base, const uint32_t *__restrict__ len, const uint32_t *__restrict__ perm,
            uint32_t n, const uint32_t *__restrict__ Rstep, uint32_t Lpad,
            const uint32_t *__restrict__ Rwords, uint32_t nw, const uint32_t *__restrict__ spos,
            const uint32_t *__restrict__ sslot, const uint32_t *__restrict__ Jarr,
            const uint32_t *__restrict__ pos, uint32_t Lb, const uint64_t *__restrict__ v,
            uint32_t r, uint32_t z, uint32_t m, uint32_t sigma, uint32_t slot_words,
            uint64_t *__restrict__ keys, uint8_t *__restrict__ sig_out,
            uint32_t *__restrict__ dk_out, uint32_t *__restrict__ ids_out, uint32_t dk_shift) {
    constexpr uint32_t CPD = 32 / BW;
    constexpr uint32_t LOGBW = BW == 2 ? 1 : (BW == 4 ? 2 : 3);
    constexpr uint32_t LOGCPD = 5 - LOGBW;
    extern __shared__ uint32_t lds[];
    const uint32_t S = z * m;
    // REC: the record, [64][Lb]; otherwise the samples, [S][64]
    uint8_t *sig = (uint8_t *)lds;
    const uint32_t head = REC ? 64 * Lb : S * 64;
    uint32_t *slots = lds + ((head + 3) >> 2);           // [64][stride]
    const uint32_t stride = slot_words + 1;
    const uint32_t lane = threadIdx.x;
    const uint32_t chunk = blockIdx.x / r, l = blockIdx.x % r;
    const uint32_t rank = chunk * 64 + lane;
    const bool valid = rank < n;
    const uint32_t id = valid ? perm[rank] : 0;
    const uint32_t slen = valid ? len[id] : 0;
    const uint64_t s0 = valid ? offsets[id] - base : 0;
    const uint32_t J = Jarr[l];
    const uint32_t *sp = spos + (size_t)l * S;
    const uint32_t *ss = sslot + (size_t)l * S;
    const uint32_t *Rs = Rstep + (size_t)l * Lpad;
    const uint32_t *Rw = Rwords + (size_t)l * nw;
    uint32_t *myslot = slots + lane * stride;
    const uint32_t chunk_steps = (slot_words - 3) * CPD;

    uint32_t i = 0;   // characters consumed by this walk
    uint32_t ps = 0;  // position of character i inside the staged window
    uint32_t k = 0;   // next sample (wave-uniform)
    uint32_t np = (!REC && S) ? sp[0] : 0xFFFFFFFFu;
    uint8_t *rec = sig + lane * Lb;  // REC: this lane's record

    for (uint32_t cj = 0; cj < J; cj += chunk_steps) {
        // ---- stage the next window of every string of the wave into LDS
        __syncthreads();
        const bool live = i < slen;
        uint64_t gq = (s0 + i) >> LOGCPD;
        uint32_t p0 = (uint32_t)((s0 + i) & (CPD - 1));
        uint32_t nd = 0;
        if (live) {
            uint64_t need = ((uint64_t)p0 + (slen - i) + CPD - 1) / CPD + 1;
            nd = need < slot_words ? (uint32_t)need : slot_words;
        }
        ps = live ? p0 : 0;
        // every lane copies its own window: independent loads, eight in flight
        for (uint32_t t0 = 0; t0 < slot_words; t0 += 8) {
            uint32_t w[8];
#pragma unroll
            for (uint32_t i = 0; i < 8; i++) w[i] = (t0 + i < nd) ? packed[gq + t0 + i] : 0u;
#pragma unroll
            for (uint32_t i = 0; i < 8; i++)
                if (t0 + i < nd) myslot[t0 + i] = w[i];
        }
        __syncthreads();

        // ---- walk this chunk of steps, CPD steps per 32-bit code window
        const uint32_t jend = min(J, cj + chunk_steps);
        for (uint32_t j0 = cj; j0 < jend; j0 += CPD) {
            const uint32_t dq = ps >> LOGCPD, sh = (ps & (CPD - 1)) << LOGBW;
            const uint32_t win = __builtin_amdgcn_alignbit(myslot[dq + 1], myslot[dq], sh);
            uint32_t off = 0;
            if (REC) {
                // every step's symbol into the record (bottom once the
                // string is used up)
#pragma unroll
                for (uint32_t s = 0; s < CPD; s++) {
                    const uint32_t j = j0 + s;
                    if (j0 + CPD <= jend || j < jend) {
                        const uint32_t c = (win >> off) & ((1u << BW) - 1u);
                        rec[j] = (uint8_t)((i + (off >> LOGBW) < slen) ? c : sigma);
                        uint32_t b;
                        if (RSTEP) {
                            b = (Rs[j] >> (c & 31u)) & 1u;
                        } else {
                            uint32_t bi = j * sigma + c;
                            b = (Rw[bi >> 5] >> (bi & 31)) & 1u;
                        }
                        off += b << LOGBW;
                    }
                }
            } else if (np >= j0 + CPD && j0 + CPD <= jend) {
#pragma unroll
                for (uint32_t s = 0; s < CPD; s++) {
                    const uint32_t c = (win >> off) & ((1u << BW) - 1u);
                    uint32_t b;
                    if (RSTEP) {
                        b = (Rs[j0 + s] >> (c & 31u)) & 1u;
                    } else {
                        uint32_t bi = (j0 + s) * sigma + c;
                        b = (Rw[bi >> 5] >> (bi & 31)) & 1u;
                    }
                    off += b << LOGBW;
                }
            } else {
#pragma unroll
                for (uint32_t s = 0; s < CPD; s++) {
                    const uint32_t j = j0 + s;
                    if (j < jend) {
                        const uint32_t c = (win >> off) & ((1u << BW) - 1u);
                        while (np == j) {
                            uint32_t sym = (i + (off >> LOGBW) < slen) ? c : sigma;
                            sig[ss[k] * 64 + lane] = (uint8_t)sym;
                            k++;
                            np = k < S ? sp[k] : 0xFFFFFFFFu;
                        }
                        uint32_t b;
                        if (RSTEP) {
                            b = (Rs[j] >> (c & 31u)) & 1u;
                        } else {
                            uint32_t bi = j * sigma + c;
                            b = (Rw[bi >> 5] >> (bi & 31)) & 1u;
                        }
                        off += b << LOGBW;
                    }
                }
            }
            const uint32_t adv = off >> LOGBW;
            i += adv;
            ps += adv;
        }
    }

    // ---- two-level hash of the z signatures of this seed:
    //      key = sum_k u_k v_k mod 2^61-1, u_k = symbol + 1 <= 256.
    //      v_k is split into four 16-bit limbs (wave-uniform, scalar); each
    //      limb sum sum_k u_k * limb is exact in 32 bits for m <= 64
    //      (64 * 257 * 2^16 < 2^31), one full-rate 24-bit multiply-add per
    //      limb and sample; the limbs recombine once per key.
    if (!valid) return;
    for (uint32_t t = 0; t < z; t++) {
        const uint64_t *vt = v + ((size_t)l * z + t) * m;
        uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        const uint32_t *pt = pos + (size_t)l * S + t * m;
        for (uint32_t kk = 0; kk < m; kk++) {
            const uint32_t u =
                (uint32_t)(REC ? rec[pt[kk]] : sig[(t * m + kk) * 64 + lane]) + 1u;
            const uint64_t vv = vt[kk];
            s0 += __umul24(u, (uint32_t)vv & 0xFFFFu);
            s1 += __umul24(u, (uint32_t)(vv >> 16) & 0xFFFFu);
            s2 += __umul24(u, (uint32_t)(vv >> 32) & 0xFFFFu);
            s3 += __umul24(u, (uint32_t)(vv >> 48));
        }
        // s0 + s1 2^16 + s2 2^32 + s3 2^48 < 2^80, reduced with 2^61 == 1 (mod P)
        const unsigned __int128 x = (unsigned __int128)s0 + ((unsigned __int128)s1 << 16) +
                                    ((unsigned __int128)s2 << 32) + ((unsigned __int128)s3 << 48);
        uint64_t res = (uint64_t)(x & P61) + (uint64_t)(x >> 61);
        res = (res & P61) + (res >> 61);
        if (res >= P61) res -= P61;
        keys[((size_t)l * z + t) * n + id] = res;
        if (dk_out) {
            dk_out[((size_t)l * z + t) * n + rank] = (uint32_t)(res >> dk_shift);
            ids_out[((size_t)l * z + t) * n + rank] = id;
        }
        if (sig_out) {
            uint8_t *dst = sig_out + (((size_t)id * r + l) * z + t) * m;
            for (uint32_t kk = 0; kk < m; kk++)
                dst[kk] = REC ? rec[pt[kk]] : sig[(t * m + kk) * 64 + lane];
        }
    }
}

// Distortion diagnostic (Section 3.1; normalised Hamming distance under
// truncation, Section 6): thread (seed l, pair e, suffix pair ka, kb) walks
// both strings' CGK embeddings side by side for L steps and counts the steps
// whose symbols differ; the pair's value for seed l is the minimum over its
// suffix pairs (atomicMin into ham, which starts at all ones).  Threads are
// ordered seed-major so that a wave reads one seed's pi bits.  Once both
// pointers are past their strings every further step emits bottom twice.
template <bool RSTEP>
__global__ void k_embed_hamming(const uint8_t *__restrict__ codes,
                                const uint64_t *__restrict__ offsets, uint64_t base,
                                const uint32_t *__restrict__ len,
                                const uint64_t *__restrict__ pairs, uint64_t count, uint32_t r,
                                uint32_t kappa, uint32_t delta, const uint32_t *__restrict__ Rstep,
                                uint32_t Lpad, const uint32_t *__restrict__ Rwords, uint32_t nw,
                                uint32_t sigma, uint32_t L, uint32_t *__restrict__ ham) {
    const uint64_t kk = (uint64_t)kappa * kappa;
    const uint64_t tot = (uint64_t)r * count * kk;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < tot;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t l = (uint32_t)(g / (count * kk));
        const uint64_t rem = g - (uint64_t)l * count * kk;
        const uint64_t e = rem / kk;
        const uint32_t sp = (uint32_t)(rem - e * kk);
        const uint32_t ka = sp / kappa, kb = sp - ka * kappa;
        const uint64_t code = pairs[e];
        const uint32_t a = (uint32_t)(code >> 32), b = (uint32_t)code;
        const uint32_t fa = len[a], fb = len[b];
        const uint64_t wa = (uint64_t)ka * delta, wb = (uint64_t)kb * delta;
        const uint32_t sa = wa < fa ? (uint32_t)wa : fa, sb = wb < fb ? (uint32_t)wb : fb;
        const uint8_t *xa = codes + (offsets[a] - base) + sa;
        const uint8_t *xb = codes + (offsets[b] - base) + sb;
        const uint32_t la = fa - sa, lb = fb - sb;
        const uint32_t *Rs = Rstep + (size_t)l * Lpad;
        const uint32_t *Rw = Rwords + (size_t)l * nw;
        uint32_t ia = 0, ib = 0, h = 0;
        for (uint32_t j = 0; j < L; j++) {
            const bool in_a = ia < la, in_b = ib < lb;
            if (!in_a && !in_b) break;
            const uint32_t ca = in_a ? xa[ia] : sigma, cb = in_b ? xb[ib] : sigma;
            h += ca != cb ? 1u : 0u;
            if (RSTEP) {
                const uint32_t w = Rs[j];
                ia += in_a ? (w >> ca) & 1u : 0u;
                ib += in_b ? (w >> cb) & 1u : 0u;
            } else {
                const uint32_t ba = j * sigma + ca, bb = j * sigma + cb;
                ia += in_a ? (Rw[ba >> 5] >> (ba & 31)) & 1u : 0u;
                ib += in_b ? (Rw[bb >> 5] >> (bb & 31)) & 1u : 0u;
            }
        }
        atomicMin(&ham[e * r + l], h);
    }
}

inline uint32_t grid_for(ej_ctx *ctx, uint64_t work, uint32_t block) {
    uint64_t g = (work + block - 1) / block;
    uint64_t cap = (uint64_t)ctx->num_cu * 16;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return (uint32_t)g;
}

}  // namespace

void prepare(ej_ctx *ctx, const uint8_t *d_chars, const uint64_t *d_offsets, uint32_t n,
             uint32_t L_req, Prep &pp, const char *tag, const uint8_t *fixed_lut,
             uint32_t fixed_sigma, uint32_t fixed_L, bool need_perm) {
    std::string t(tag);
    pp.n = n;
    pp.d_offsets = d_offsets;
    pp.d_chars = d_chars;
    PrepInfo *d_info = ws<PrepInfo>(ctx, t + "_info", 1);
    pp.d_len = ws<uint32_t>(ctx, t + "_len", n + 1);
    hipLaunchKernelGGL(k_prep_info, dim3(1), dim3(64), 0, ctx->stream, d_offsets, n, d_info);
    EJ_CHECK_LAUNCH();
    if (n)
        hipLaunchKernelGGL(k_lengths, dim3(grid_for(ctx, n, 256)), dim3(256), 0, ctx->stream,
                           d_offsets, n, pp.d_len, d_info);
    EJ_CHECK_LAUNCH();
    // the byte presence bitmap in the same round trip as the offsets summary
    if (d_chars) {
        hipLaunchKernelGGL(k_presence, dim3((uint32_t)ctx->num_cu * 16), dim3(256), 0,
                           ctx->stream, d_chars, d_info);
        EJ_CHECK_LAUNCH();
    }
    PrepInfo info;
    read_back(ctx, d_info, sizeof(PrepInfo), &info);
    if (info.err & 1u) fail(EJ_EINVAL, "offsets are not non-decreasing");
    if (info.err & 2u) fail(EJ_EINVAL, "a string is longer than 2^31-1 bytes");
    if (info.offn < info.off0) fail(EJ_EINVAL, "offsets[n] < offsets[0]");
    pp.base = info.off0;
    pp.total = info.offn - info.off0;
    pp.maxlen = info.maxlen;
    pp.minlen = pp.n ? info.minlen : 0u;
    if (pp.total && !d_chars) fail(EJ_EINVAL, "null character buffer");
    uint32_t mask[8] = {0};
    memcpy(mask, info.mask, sizeof(mask));
    if (fixed_lut) {
        for (int b = 0; b < 256; b++)
            if (((mask[b >> 5] >> (b & 31)) & 1u) && fixed_lut[b] == 0xFF)
                fail(EJ_EALPHABET, "byte " + std::to_string(b) + " is outside the index alphabet");
        memcpy(pp.lut, fixed_lut, 256);
        pp.sigma = fixed_sigma;
    } else {
        uint32_t s = 0;
        for (int b = 0; b < 256; b++) {
            bool present = (mask[b >> 5] >> (b & 31)) & 1u;
            pp.lut[b] = present ? (uint8_t)s : 0xFF;
            if (present) s++;
        }
        if (s > 255) fail(EJ_EALPHABET, "all 256 byte values occur; the padding symbol needs one");
        pp.sigma = s;
    }
    // truncation (Section 4.1): ceil(average length) by default, at most 3N
    if (fixed_L) {
        pp.L = fixed_L;
    } else {
        uint64_t L = L_req;
        if (L == 0) L = n ? (pp.total + n - 1) / n : 1;
        if (L > 3ull * pp.maxlen) L = 3ull * pp.maxlen;
        if (L == 0) L = 1;
        if (L > 0x7FFFFFFFull) fail(EJ_EINVAL, "truncation length too large");
        pp.L = (uint32_t)L;
    }
    uint32_t sig_eff = pp.sigma ? pp.sigma : 1;
    pp.bw = sig_eff <= 4 ? 2 : (sig_eff <= 16 ? 4 : 8);
    // encodings
    uint8_t *d_lut = ws<uint8_t>(ctx, t + "_lut", 256);
    EJ_HIP(hipMemcpyAsync(d_lut, pp.lut, 256, hipMemcpyHostToDevice, ctx->stream));
    pp.d_codes = ws<uint8_t>(ctx, t + "_codes", ((pp.total + 3) & ~3ull) + 64);
    uint32_t cpd = 32 / pp.bw;
    uint64_t nwords = (pp.total + cpd - 1) / cpd;
    pp.d_packed = ws<uint32_t>(ctx, t + "_packed", nwords + 8);
    {
        dim3 g(grid_for(ctx, nwords + 8, 256));
        auto launch = [&](auto kern) {
            hipLaunchKernelGGL(kern, g, dim3(256), 0, ctx->stream, d_chars, pp.base, pp.total,
                               (const uint8_t *)d_lut, pp.d_codes, nwords, pp.d_packed);
            EJ_CHECK_LAUNCH();
        };
        if (pp.bw == 2)
            launch(k_encode_pack<2>);
        else if (pp.bw == 4)
            launch(k_encode_pack<4>);
        else
            launch(k_encode_pack<8>);
    }
    // length order (stable: ties keep input order)
    pp.d_perm = nullptr;
    if (need_perm && n) {
        uint32_t *lk = ws<uint32_t>(ctx, t + "_lenkey", n);
        uint32_t *iota = ws<uint32_t>(ctx, t + "_iota", n);
        uint32_t *lk2 = ws<uint32_t>(ctx, t + "_lenkey2", n);
        pp.d_perm = ws<uint32_t>(ctx, t + "_perm", n);
        EJ_HIP(hipMemcpyAsync(lk, pp.d_len, n * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                              ctx->stream));
        hipLaunchKernelGGL(k_iota, dim3(grid_for(ctx, n, 256)), dim3(256), 0, ctx->stream, iota, n);
        EJ_CHECK_LAUNCH();
        radix_sort_u32(ctx, lk, iota, lk2, pp.d_perm, 1, n, bits_for(pp.maxlen), 8);
    }
}

void draw_randomness(ej_ctx *ctx, const ej_params &p, uint32_t L, uint32_t sigma, Rand &rd,
                     const char *tag) {
    std::string t(tag);
    rd.r = p.r;
    rd.z = p.z;
    rd.m = p.m;
    rd.L = L;
    rd.sigma = sigma;
    rd.S = p.z * p.m;
    const uint32_t sig_eff = sigma ? sigma : 1;
    uint64_t nbits = (uint64_t)L * sig_eff;
    rd.nw = (uint32_t)((nbits + 31) / 32) + 16;
    rd.Lpad = ((L + 63) / 64) * 64 + 64;
    uint32_t T = p.r * p.z;
    rd.d_Rwords = ws<uint32_t>(ctx, t + "_Rwords", (size_t)p.r * rd.nw);
    rd.d_Rstep = ws<uint32_t>(ctx, t + "_Rstep", (size_t)p.r * rd.Lpad);
    rd.d_pos = ws<uint32_t>(ctx, t + "_pos", (size_t)T * p.m);
    rd.d_v = ws<uint64_t>(ctx, t + "_v", (size_t)T * p.m);
    rd.d_spos = ws<uint32_t>(ctx, t + "_spos", (size_t)T * p.m);
    rd.d_sslot = ws<uint32_t>(ctx, t + "_sslot", (size_t)T * p.m);
    rd.d_J = ws<uint32_t>(ctx, t + "_J", p.r);
    const Explicit &ex = ctx->ex;
    bool use_ex = ex.active && ex.r == p.r && ex.z == p.z && ex.m == p.m && ex.L == L &&
                  ex.sigma == sigma;
    if (use_ex) {
        // rows of the explicit words may be shorter than rd.nw; copy row-wise
        EJ_HIP(hipMemsetAsync(rd.d_Rwords, 0, (size_t)p.r * rd.nw * 4, ctx->stream));
        for (uint32_t l = 0; l < p.r; l++)
            EJ_HIP(hipMemcpyAsync(rd.d_Rwords + (size_t)l * rd.nw, ex.Rwords.data() + (size_t)l * ex.nw,
                                  (size_t)std::min(ex.nw, rd.nw) * 4, hipMemcpyHostToDevice,
                                  ctx->stream));
        EJ_HIP(hipMemcpyAsync(rd.d_pos, ex.pos.data(), ex.pos.size() * 4, hipMemcpyHostToDevice,
                              ctx->stream));
        if (!ex.v.empty())
            EJ_HIP(hipMemcpyAsync(rd.d_v, ex.v.data(), ex.v.size() * 8, hipMemcpyHostToDevice,
                                  ctx->stream));
        // explicit host arrays are pageable: wait before they can change
        sync(ctx);
    } else {
        hipLaunchKernelGGL(k_draw_R, dim3(grid_for(ctx, (uint64_t)p.r * rd.nw, 256)), dim3(256), 0,
                           ctx->stream, p.seed, p.r, rd.nw, rd.d_Rwords);
        EJ_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_draw_lsh, dim3(grid_for(ctx, (uint64_t)T * p.m, 256)), dim3(256), 0,
                       ctx->stream, p.seed, p.r, p.z, p.m, L, rd.d_pos, rd.d_v, use_ex ? 0 : 1,
                       (use_ex && !ex.v.empty()) ? 0 : 1);
    EJ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_rstep, dim3(grid_for(ctx, (uint64_t)p.r * rd.Lpad, 256)), dim3(256), 0,
                       ctx->stream, (const uint32_t *)rd.d_Rwords, rd.nw, p.r, rd.Lpad, L, sig_eff,
                       rd.d_Rstep);
    EJ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sample_sort, dim3(p.r), dim3(256), 0, ctx->stream,
                       (const uint32_t *)rd.d_pos, rd.S, rd.d_spos, rd.d_sslot, rd.d_J);
    EJ_CHECK_LAUNCH();
    rd.Jmax = L;
}

void embed_keys(ej_ctx *ctx, const Prep &pp, const Rand &rd, uint64_t *d_keys, uint8_t *d_sig,
                uint32_t *d_dk, uint32_t *d_rank_ids, uint32_t dk_shift) {
    if (pp.n == 0) return;
    const uint32_t S = rd.S;
    // short walks keep their whole record (Lb bytes per lane, Lb / 4 odd so
    // that the lanes' bytes of one step fall in different banks)
    const bool rec = rd.Jmax <= EMBED_REC_STEPS;
    uint32_t Lb = (rd.Jmax + 3) & ~3u;
    if (((Lb / 4) & 1u) == 0) Lb += 4;
    const uint32_t sigbytes = rec ? 64 * Lb : ((S * 64 + 3) / 4) * 4;
    // the walk is a dependent chain per lane: waves per CU hide its
    // latency, so by default the string windows are short (16 words: 64 to
    // 256 letters between restagings) and the LDS per wave is mostly the
    // samples (z * m bytes per lane)
    uint32_t budget = ctx->tune.embed_lds_budget;
    if (budget == 0) budget = sigbytes + 64 * 4 * 17;
    if (sigbytes + 64 * 4 * 12 > budget) budget = sigbytes + 64 * 4 * 64;
    if ((int)budget > ctx->lds_max) budget = (uint32_t)ctx->lds_max;
    if (sigbytes + 64 * 4 * 12 > budget)
        fail(EJ_EUNSUPPORTED, "z*m = " + std::to_string(S) + " samples per seed do not fit in LDS");
    uint32_t slot_words = (budget - sigbytes) / (64 * 4) - 1;
    // a window never needs more than the longest string plus slack
    uint32_t cpd = 32 / pp.bw;
    uint32_t need = (std::min(pp.maxlen, pp.L) + cpd - 1) / cpd + 4;
    if (slot_words > need) slot_words = std::max(need, 8u);
    size_t lds = sigbytes + (size_t)64 * (slot_words + 1) * 4;
    dim3 grid(rd.r * ceil_div(pp.n, 64)), block(64);
    const bool rstep = rd.sigma <= 32;
    auto launch = [&](auto kern) {
        if (lds > 65536)
            EJ_HIP(hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, grid, block, lds, ctx->stream, (const uint32_t *)pp.d_packed,
                           pp.d_offsets, pp.base, (const uint32_t *)pp.d_len,
                           (const uint32_t *)pp.d_perm, pp.n, (const uint32_t *)rd.d_Rstep, rd.Lpad,
                           (const uint32_t *)rd.d_Rwords, rd.nw, (const uint32_t *)rd.d_spos,
                           (const uint32_t *)rd.d_sslot, (const uint32_t *)rd.d_J,
                           (const uint32_t *)rd.d_pos, Lb, (const uint64_t *)rd.d_v, rd.r, rd.z,
                           rd.m, rd.sigma, slot_words, d_keys,
                           d_sig, d_dk, d_rank_ids, dk_shift);
        EJ_CHECK_LAUNCH();
    };
    if (rec) {
        if (pp.bw == 2)
            rstep ? launch(k_embed<2, true, true>) : launch(k_embed<2, false, true>);
        else if (pp.bw == 4)
            rstep ? launch(k_embed<4, true, true>) : launch(k_embed<4, false, true>);
        else
            rstep ? launch(k_embed<8, true, true>) : launch(k_embed<8, false, true>);
    } else {
        if (pp.bw == 2)
            rstep ? launch(k_embed<2, true, false>) : launch(k_embed<2, false, false>);
        else if (pp.bw == 4)
            rstep ? launch(k_embed<4, true, false>) : launch(k_embed<4, false, false>);
        else
            rstep ? launch(k_embed<8, true, false>) : launch(k_embed<8, false, false>);
    }
}

void embed_hamming(ej_ctx *ctx, const Prep &pp, const Rand &rd, const uint64_t *d_pairs,
                   uint64_t count, uint32_t kappa, uint32_t delta, uint32_t *d_ham) {
    if (count == 0) return;
    const uint64_t tot = (uint64_t)rd.r * count * kappa * kappa;
    EJ_HIP(hipMemsetAsync(d_ham, 0xFF, 4 * count * rd.r, ctx->stream));
    const uint32_t sig = rd.sigma ? rd.sigma : 1;
    auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid_for(ctx, tot, 256)), dim3(256), 0, ctx->stream,
                           (const uint8_t *)pp.d_codes, pp.d_offsets, pp.base,
                           (const uint32_t *)pp.d_len, d_pairs, count, rd.r, kappa, delta,
                           (const uint32_t *)rd.d_Rstep, rd.Lpad, (const uint32_t *)rd.d_Rwords,
                           rd.nw, sig, rd.L, d_ham);
        EJ_CHECK_LAUNCH();
    };
    if (sig <= 32)
        launch(k_embed_hamming<true>);
    else
        launch(k_embed_hamming<false>);
}

}  // namespace ej
