// Stage A5: threshold edit distance of candidate pairs (Section 3.3).
//
// Ukkonen's observation is that only a band of diagonals of the
// dynamic-programming table matters when the answer is compared with K.  For
// strings x (rows, the longer one) and y (columns), with d* = |x| - |y|, a
// path through diagonal d costs at least |d| + |d - d*|, so a path of cost
// <= K stays on the K + 1 diagonals lo..hi with lo = -floor((K - d*)/2) and
// hi = d* + floor((K - d*)/2).  The kernel evaluates that band with Myers'
// bit-vector recurrence (vertical and horizontal +1/-1 deltas as bit masks,
// one table column per step) in a diagonal-aligned form: bit k of the state
// always holds diagonal k + lo, so the band slides down one row per column
// by shifting the state right by one bit.
//
//  * Cells just outside the band are replaced by upper bounds (no move from
//    above the band's top row; a +1 vertical delta below its bottom row).
//    Every computed value is then >= the true value, and exact wherever an
//    optimal path of cost <= K passes, because such a path never leaves the
//    band.  The result min(value, K+1) therefore equals min(ED, K+1).
//  * Rows above row 0 are virtual rows with D[i][j] = j - i; they are
//    consistent with the recurrence, which removes all special cases at the
//    top-left corner.
//  * The value on diagonal d* (the final cell's) is tracked column by
//    column: along a diagonal the value grows by 0 or 1, and it stays put
//    exactly when the characters match or a horizontal or vertical -1 delta
//    enters the cell.  Cells of diagonal d* whose true value is <= K are
//    exact (their optimal paths obey the same diagonal bound), so a value
//    above K ends the pair early.
//
// GPU mapping: a pair owns NL lanes of a wave (32 band bits per lane, NL =
// ceil((K+2)/32)); a wave holds floor(64/NL) pairs.  The W-bit addition of
// Myers' step is a 32-bit add per lane plus a carry-lookahead across lanes
// done on two ballots with scalar arithmetic; the one-bit shift across lanes
// is a DPP wave_shl.  The match masks of the pattern (one bit array per
// symbol) live in LDS; the text is streamed from HBM one 32-column block
// ahead.  Verification runs in two passes: every pair for the first C1
// columns (most false candidates are rejected there), then the surviving
// pairs, compacted, from their saved state -- so that waves are not held by
// one long pair while the rest of their lanes idle.
#include <stdio.h>

#include <algorithm>

#include "ej_internal.h"

namespace ej {

namespace {

constexpr uint32_t NO_LIMIT = 0xFFFFFFFFu;
constexpr uint32_t DECIDED = 0xFFFFFFFFu;

// How a pair's lanes are laid out in the wave, which decides how the
// one-bit shift and the carries cross lanes:
//   LANES_ONE  one lane per pair: no cross-lane traffic at all;
//   LANES_ROW  16 lanes per pair = one DPP row: row_shl gives the top lane 0;
//   LANES_WAVE 64 lanes per pair: wave_shl gives lane 63 zero and the carry
//              out of lane 63 falls off the 64-bit scalar add;
//   LANES_ANY  any other width: wave_shl plus a mask, carries cut per pair.
enum { LANES_ONE = 0, LANES_ROW = 1, LANES_WAVE = 2, LANES_ANY = 3 };

// Lanes per pair: fixed by the layout except for LANES_ANY, so that the
// per-block index arithmetic folds to constants in the common layouts.
template <int MODE>
__device__ inline uint32_t lanes_of(uint32_t nl) {
    return MODE == LANES_ONE ? 1u : MODE == LANES_ROW ? 16u : MODE == LANES_WAVE ? 64u : nl;
}

// s = a + b; the carry-out of every lane lands in one wave-wide mask.
__device__ inline uint32_t add_carry_mask(uint32_t a, uint32_t b, uint64_t &carry) {
    uint32_t s;
    asm("v_add_co_u32 %0, %1, %2, %3" : "=v"(s), "=s"(carry) : "v"(a), "v"(b));
    return s;
}

// s = a + b + (bit `lane` of cin); carry-outs of every lane in cout.
__device__ inline uint32_t add_carry_chain(uint32_t a, uint32_t b, uint64_t cin, uint64_t &cout) {
    uint32_t s;
    asm("v_addc_co_u32 %0, %1, %2, %3, %4" : "=v"(s), "=s"(cout) : "v"(a), "v"(b), "s"(cin));
    return s;
}

// s = a + (bit `lane` of the wave-wide mask cin): one add with the carry-in
// taken straight from the scalar mask.
__device__ inline uint32_t add_carry_in(uint32_t a, uint64_t cin) {
    uint32_t s;
    uint64_t unused;
    asm("v_addc_co_u32 %0, %1, %2, 0, %3" : "=v"(s), "=s"(unused) : "v"(a), "s"(cin));
    return s;
}

// s = a + (bit `lane` of cin), with the carry-out of every lane in cout.
__device__ inline uint32_t add_carry_in_out(uint32_t a, uint64_t cin, uint64_t &cout) {
    uint32_t s;
    asm("v_addc_co_u32 %0, %1, %2, 0, %3" : "=v"(s), "=s"(cout) : "v"(a), "s"(cin));
    return s;
}

// The verified-column counter: each lane sums the columns of the pairs it
// decided, and a wave adds once when it leaves (one atomic per wave instead of
// one per pair, which contended on the counter's line).
__device__ inline void add_columns(unsigned long long *columns, unsigned long long v) {
    if (!columns) return;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63u) == 0 && v) atomicAdd(columns, v);
}

// popcount(x) + acc in one v_bcnt.
__device__ inline uint32_t popc_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

template <int MODE>
__device__ inline uint32_t from_next_lane(uint32_t x, uint32_t keep) {
    if (MODE == LANES_ROW)  // row_shl:1, lanes 15/31/47/63 read 0
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x101, 0xf, 0xf, true);
    const uint32_t y = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x130, 0xf, 0xf, true);
    return MODE == LANES_WAVE ? y : (y & keep);
}

// Words of one pair's match-mask tile in LDS: sigma rows of `stride` words,
// padded so that consecutive tiles start 16 banks apart.  The rows' strides
// are multiples of 32 words, so without the pad the pairs of a wave would
// read their ring slots from the same banks in every column (4-way bank
// conflicts at 4 pairs per wave); with it, 2-way, the least that 64 lanes
// reading 64 words from 32 banks can have.
__host__ __device__ inline uint32_t tile_words_for(uint32_t sigma, uint32_t stride) {
    const uint32_t w = sigma * stride;
    return w + ((16u - (w & 31u)) & 31u);
}

// 32 columns of Myers' step in the diagonal-aligned band.  FAST counts the
// tracked diagonal with a masked popcount (no pair's text ends inside the
// block); otherwise one bit per column is collected into acc.
// The match word of column jb+1+s is read from LDS inside the step (text
// symbol s of tw selects the symbol's bit array; the lane's two words at
// `slot` are funnel-shifted by s), which keeps the live registers low.
// Addresses are LDS byte offsets: symbol c's words start at c * stride4
// (a 24-bit multiply of the symbol byte) and the lane's word at slot4.
template <int MODE, bool FAST>
__device__ inline void myers_block(const uint8_t *peq, uint32_t stride4, uint32_t slot4,
                                   const uint32_t tw[8], uint32_t &Pv, uint32_t &Mv, uint32_t &Z,
                                   uint32_t &acc, uint32_t kmask, uint32_t kbit, uint64_t notlast,
                                   uint32_t keep) {
#pragma unroll
    for (uint32_t s = 0; s < 32; s++) {
        const uint32_t c = (tw[s >> 2] >> (8 * (s & 3))) & 0xFFu;
        const uint32_t *pa = (const uint32_t *)(peq + (__umul24(c, stride4) + slot4));
        const uint32_t eq = __builtin_amdgcn_alignbit(pa[1], pa[0], s);
        const uint32_t Xv = eq | Mv;
        uint32_t sum;
        if (MODE == LANES_ONE) {
            sum = (eq & Pv) + Pv;
        } else {
            uint64_t G;
            sum = add_carry_mask(eq & Pv, Pv, G);
            uint64_t P = __builtin_amdgcn_ballot_w64(sum == 0xFFFFFFFFu);
            if (MODE != LANES_WAVE) {
                G &= notlast;
                P &= notlast;
            }
            const uint64_t cin = ((G | P) + G) ^ P;
            sum = add_carry_in(sum, cin);
        }
        const uint32_t Xh = (sum ^ Pv) | eq;
        const uint32_t Ph = Mv | ~(Xh | Pv);
        const uint32_t Mh = Pv & Xh;
        const uint32_t nx = MODE == LANES_ONE ? 0u : from_next_lane<MODE>(Xv, keep);
        const uint32_t Xv1 = __builtin_amdgcn_alignbit(nx, Xv, 1);
        Pv = Mh | ~(Xv1 | Ph);
        Mv = Ph & Xv1;
        if (FAST)
            Z = popc_acc((Xv1 | Mh) & kmask, Z);
        else
            acc |= (((Xv1 | Mh) >> kbit) & 1u) << s;
    }
}

// myers_block with WPL band words per lane (2 or 4; words WPL*l ..
// WPL*l + WPL - 1 of the pair's band in lane l): the lane's sum carries
// between its words inside the lane, and the lookahead between lanes
// (ballots, scalar add) and the shift's word from the next lane are paid once
// per 32*WPL bits.  km[q] selects the tracked diagonal's bit in word q of the
// owner lane (zero elsewhere).
template <int MODE, bool FAST, int WPL>
__device__ inline void myers_blockw(const uint8_t *peq, uint32_t stride4, uint32_t slot4,
                                    const uint32_t tw[8], uint32_t (&Pv)[WPL],
                                    uint32_t (&Mv)[WPL], uint32_t &Z, uint32_t &acc,
                                    const uint32_t (&km)[WPL], uint64_t notlast, uint32_t keep) {
#pragma unroll
    for (uint32_t s = 0; s < 32; s++) {
        const uint32_t c = (tw[s >> 2] >> (8 * (s & 3))) & 0xFFu;
        const uint32_t *pa = (const uint32_t *)(peq + (__umul24(c, stride4) + slot4));
        uint32_t mw[WPL + 1], eq[WPL], X[WPL], sum[WPL];
#pragma unroll
        for (int q = 0; q <= WPL; q++) mw[q] = pa[q];
#pragma unroll
        for (int q = 0; q < WPL; q++) {
            eq[q] = __builtin_amdgcn_alignbit(mw[q + 1], mw[q], s);
            X[q] = eq[q] | Mv[q];
        }
        uint64_t cy;
        sum[0] = add_carry_mask(eq[0] & Pv[0], Pv[0], cy);
#pragma unroll
        for (int q = 1; q < WPL; q++) sum[q] = add_carry_chain(eq[q] & Pv[q], Pv[q], cy, cy);
        if (MODE != LANES_ONE) {
            uint32_t all = sum[0];
#pragma unroll
            for (int q = 1; q < WPL; q++) all &= sum[q];
            uint64_t G = cy;
            uint64_t P = __builtin_amdgcn_ballot_w64(all == 0xFFFFFFFFu);
            if (MODE != LANES_WAVE) {
                G &= notlast;
                P &= notlast;
            }
            const uint64_t cin = ((G | P) + G) ^ P;
            sum[0] = add_carry_in_out(sum[0], cin, cy);
#pragma unroll
            for (int q = 1; q < WPL - 1; q++) sum[q] = add_carry_in_out(sum[q], cy, cy);
            sum[WPL - 1] = add_carry_in(sum[WPL - 1], cy);
        }
        const uint32_t nx = MODE == LANES_ONE ? 0u : from_next_lane<MODE>(X[0], keep);
        uint32_t d = 0;
#pragma unroll
        for (int q = 0; q < WPL; q++) {
            const uint32_t Xh = (sum[q] ^ Pv[q]) | eq[q];
            const uint32_t Ph = Mv[q] | ~(Xh | Pv[q]);
            const uint32_t Mh = Pv[q] & Xh;
            const uint32_t Xs = __builtin_amdgcn_alignbit(q + 1 < WPL ? X[q + 1] : nx, X[q], 1);
            Pv[q] = Mh | ~(Xs | Ph);
            Mv[q] = Ph & Xs;
            d |= (Xs | Mh) & km[q];
        }
        if (FAST)
            Z = popc_acc(d, Z);
        else
            acc |= (d != 0u ? 1u : 0u) << s;
    }
}

// The 32 text symbols of columns jb+1 .. jb+32 (bytes y[jb .. jb+31]) as 8
// little-endian dwords, or zeros once jb >= nn.  Bytes past position nn are
// the next strings' codes or the array's zeroed padding -- valid symbols
// either way; the columns they feed are past the end of the text and never
// counted.  Reads stay within y[0 .. nn+35] (the code arrays carry 64 bytes
// of padding).
__device__ inline void load_text_block(const uint8_t *y, uint32_t nn, uint32_t jb, uint32_t tw[8]) {
#pragma unroll
    for (int q = 0; q < 8; q++) tw[q] = 0;
    if (jb >= nn) return;
    const uintptr_t a = (uintptr_t)(y + jb);
    const uint32_t *base = (const uint32_t *)(a & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(a & 3) * 8;
    uint32_t w[9];
#pragma unroll
    for (int q = 0; q < 9; q++) w[q] = base[q];
#pragma unroll
    for (int q = 0; q < 8; q++) tw[q] = __builtin_amdgcn_alignbit(w[q + 1], w[q], sh);
}

// One string set as the kernels see it: symbol codes (offsets relative to
// base) and the precomputed match masks of every string.
struct StrSet {
    const uint8_t *codes;
    const uint64_t *off;
    uint64_t base;
    const uint32_t *mw;    // mask words
    const uint64_t *moff;  // [n] first mask word of each string
};

struct PairView {
    const uint8_t *xp, *yp;
    const uint32_t *mw;            // pattern's masks: symbol c at mw + c * W
    uint32_t W;                    // mask words per symbol of the pattern
    uint32_t m, nn, Kp, dstar, O;  // O = -lo = floor((Kp - d*)/2)
    bool skip;
};

__device__ inline PairView view_pair(const StrSet &A, const StrSet &B, const uint64_t *pairs,
                                     const uint32_t *Kq, uint32_t K, uint64_t pidx, bool act) {
    PairView v;
    v.xp = A.codes;
    v.yp = A.codes;
    v.mw = A.mw;
    v.W = 0;
    v.m = 0;
    v.nn = 0;
    v.Kp = K;
    if (act) {
        uint64_t code = pairs[pidx];
        uint32_t a = (uint32_t)(code >> 32), b = (uint32_t)code;
        uint64_t oa = A.off[a], ob = B.off[b];
        uint32_t la = (uint32_t)(A.off[a + 1] - oa), lb = (uint32_t)(B.off[b + 1] - ob);
        const uint8_t *pa = A.codes + (oa - A.base), *pb = B.codes + (ob - B.base);
        if (Kq) v.Kp = Kq[pidx];
        if (la >= lb) {
            v.xp = pa; v.m = la; v.yp = pb; v.nn = lb;
            v.mw = A.mw + A.moff[a];
        } else {
            v.xp = pb; v.m = lb; v.yp = pa; v.nn = la;
            v.mw = B.mw + B.moff[b];
        }
        v.W = (v.m + 31) / 32;
    }
    v.skip = !act || v.m - v.nn > v.Kp;
    if (v.skip) {
        v.m = 0;
        v.nn = 0;
        v.W = 0;
    }
    // a skipped pair keeps d* = 0 so that one lane of its tile owns the
    // (constant) result K_p + 1
    v.dstar = v.m - v.nn;
    v.O = v.skip ? 0u : (v.Kp - v.dstar) / 2;
    return v;
}

// Word `wabs` of the band's match mask for symbol c: bit b is pattern row
// 32*wabs + b - O (1-based), i.e. pattern index p = 32*wabs + b - O - 1,
// funnel-shifted out of the pattern's precomputed masks; indexes below 0 or
// past the pattern read as zero.
__device__ inline uint32_t mask_word(const PairView &v, uint32_t c, uint32_t wabs) {
    const int32_t p0 = 32 * (int32_t)wabs - (int32_t)v.O - 1;
    const int32_t q = p0 >> 5;  // floor(p0 / 32)
    const uint32_t sh = (uint32_t)p0 & 31u;
    const uint32_t *mc = v.mw + (size_t)c * v.W;
    const uint32_t lo = (uint32_t)q < v.W ? mc[q] : 0u;
    const uint32_t hi = (uint32_t)(q + 1) < v.W ? mc[q + 1] : 0u;
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// Match-mask words w0 .. w0+nw-1 of every symbol into one tile's LDS region
// `pq`, shared among the tile's NL lanes (lane l of the tile).
template <bool RING>
__device__ inline void fill_tile(uint32_t *pq, const PairView &v, uint32_t l, uint32_t NL,
                                 uint32_t sigma, uint32_t stride, uint32_t RW, uint32_t wpp,
                                 uint32_t w0, uint32_t nw) {
    for (uint32_t c = 0; c < sigma; c++)
        for (uint32_t w = l; w < nw; w += NL) {
            const uint32_t word = mask_word(v, c, w0 + w);
            if (RING) {
                const uint32_t sl = (w0 + w) & (RW - 1);
                pq[c * stride + sl] = word;
                pq[c * stride + sl + RW] = word;
            } else if (w0 + w < wpp) {
                pq[c * stride + w0 + w] = word;
            }
        }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// k_verify's tile: the full layout as in fill_tile, or a ring of RW slots
// (word w at slot w % RW) whose first WPL slots are repeated after the last
// (stride RW + WPL), so that the WPL + 1 words a lane reads are always
// adjacent.
template <bool RING, int WPL>
__device__ inline void fill_tile_w(uint32_t *pq, const PairView &v, uint32_t l, uint32_t NL,
                                   uint32_t sigma, uint32_t stride, uint32_t RW, uint32_t wpp,
                                   uint32_t w0, uint32_t nw) {
    for (uint32_t c = 0; c < sigma; c++)
        for (uint32_t w = l; w < nw; w += NL) {
            const uint32_t word = mask_word(v, c, w0 + w);
            if (RING) {
                const uint32_t sl = (w0 + w) % RW;
                pq[c * stride + sl] = word;
                if (sl < WPL) pq[c * stride + sl + RW] = word;
            } else if (w0 + w < wpp) {
                pq[c * stride + w0 + w] = word;
            }
        }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Match masks of a pair live in LDS in one of two layouts:
//   full (RING = false): word w of symbol c at c*stride + w, stride = wpp,
//        the whole pattern;
//   ring (RING = true):  only the NL+1 words the band touches at a time,
//        word w at slots w % RW and w % RW + RW (stride = 2*RW) so that two
//        consecutive words are always adjacent; the word entering the band
//        is computed from the pattern once per 32-column block.
// Bit b of word w is pattern row 32w + b - O (1-based; rows outside
// 1..m never match).
//
// One pass over a list of pairs.  Pass 1 (resume == 0) starts every pair at
// column 0 and stops at column jlim; the owner lane writes aux[pidx] = Z for
// a pair still undecided there (its Pv/Mv go to `state`) and DECIDED for the
// others.  Pass 2 (resume == 1) takes the pairs listed in `list`, restores
// their state and runs them to the end.  WPL band words per lane (1, 2 or
// 4): lane l of a pair holds words WPL*l .. WPL*l + WPL - 1, NL_arg is the
// lanes per pair.  The ring here (fill_tile_w) has RW = wpp = NW + 1 slots:
// a block reads words jb/32 .. jb/32 + NW, and the word entering after it
// takes the slot of word jb/32, which no lane reads again.
template <int MODE, bool RING, int WPL>
__global__ void __launch_bounds__(64)
    k_verify(StrSet A, StrSet B, const uint64_t *__restrict__ pairs, uint64_t count_arg,
             const uint64_t *__restrict__ count_dev, const uint32_t *__restrict__ list,
             uint32_t K, const uint32_t *__restrict__ Kq, uint32_t sigma, uint32_t NL_arg,
             uint32_t tpw, uint32_t wpp, uint32_t jbeg, uint32_t jlim, int resume,
             uint32_t *__restrict__ state, uint32_t *__restrict__ aux,
             int32_t *__restrict__ dist, unsigned long long *__restrict__ columns) {
    extern __shared__ uint32_t lds[];
    unsigned long long colsum = 0;  // text columns of the pairs decided here
    const uint32_t NL = lanes_of<MODE>(NL_arg);
    const uint32_t NW = NL * WPL;  // band words of a pair
    constexpr uint32_t LWB = WPL == 4 ? 7 : WPL == 2 ? 6 : 5;  // log2 of a lane's bits
    // pass 2, and a join sized on the device, take the pair count from the
    // device (a grid sized for all pairs; never more than count_arg)
    const uint64_t count = count_dev ? min(*count_dev, count_arg) : count_arg;
    const uint32_t lane = threadIdx.x;
    const uint32_t tile = lane / NL, l = lane - tile * NL;
    const bool in_tile = tile < tpw;
    const uint32_t RW = wpp;                          // ring: words per ring
    const uint32_t stride = RING ? RW + WPL : wpp;    // words per symbol
    const uint32_t tile_words = tile_words_for(sigma, stride);
    uint64_t last = 0;  // top lane of every pair, and lanes outside pairs
    for (uint32_t q = 0; q < 64; q++)
        if ((q / NL) >= tpw || (q % NL) == NL - 1) last |= 1ull << q;
    const uint64_t notlast = ~last;
    const uint32_t keep = (l == NL - 1 || !in_tile) ? 0u : 0xFFFFFFFFu;
    uint32_t *pq_mine = lds + (in_tile ? tile : 0) * tile_words;
    const uint8_t *peq8 = (const uint8_t *)pq_mine;

    for (uint64_t g = blockIdx.x; g * tpw < count; g += gridDim.x) {
        const uint64_t k = g * tpw + tile;  // index into the (listed) pairs
        const bool act = in_tile && k < count;
        const uint64_t pidx = act ? (list ? (uint64_t)list[k] : k) : 0;
        const PairView v = view_pair(A, B, pairs, Kq, K, pidx, act);
        __syncthreads();
        // ---- match masks of the words the first block needs (ring) or of
        //      the whole pattern (full), every tile its own
        if (in_tile)
            fill_tile_w<RING, WPL>(pq_mine, v, l, NL, sigma, stride, RW, wpp,
                                   RING ? (jbeg >> 5) : 0u, RING ? NW + 1 : wpp);
        __syncthreads();

        // ---- state at column jbeg
        const uint32_t kstar = v.O + v.dstar;
        const bool owner = in_tile && (kstar >> LWB) == l;
        const uint32_t kbit = kstar & 31;
        // the tracked diagonal's word inside the owner lane
        const uint32_t kw = (kstar >> 5) & (WPL - 1);
        uint32_t Pv[WPL], Mv[WPL], Z = 0;
        if (resume) {
#pragma unroll
            for (int q = 0; q < WPL; q++) {
                Pv[q] = act ? state[(pidx * NL + l) * 2 * WPL + 2 * q] : 0u;
                Mv[q] = act ? state[(pidx * NL + l) * 2 * WPL + 2 * q + 1] : 0u;
            }
            if (owner && act) Z = aux[pidx];
        } else {
            // D[i][0] = |i|: bit k holds row k - O, rows <= 0 have delta -1
#pragma unroll
            for (int q = 0; q < WPL; q++) {
                const int lo = 32 * (int)(WPL * l + q);
                const int Oi = (int)v.O;
                if (Oi >= lo + 31)
                    Mv[q] = ~0u;
                else if (Oi < lo)
                    Mv[q] = 0u;
                else
                    Mv[q] = (1u << (Oi - lo + 1)) - 1u;
                Pv[q] = ~Mv[q];
            }
        }
        uint32_t nmax = v.nn;
        for (int d = 32; d >= 1; d >>= 1) nmax = max(nmax, (uint32_t)__shfl_xor((int)nmax, d, 64));
        const uint32_t jend = min(nmax, jlim);
        uint32_t jdone = jbeg;
        // the owner's own stopping column: the wave runs on until its last
        // pair is decided, but only the columns a pair needed are counted
        uint32_t jstop = NO_LIMIT;
        uint32_t tw[8], tn[8];
        load_text_block(v.yp, v.nn, jbeg, tw);
        uint32_t sb = RING ? (jbeg >> 5) % RW : 0u;  // ring: the slot of word jb/32
        for (uint32_t jb = jbeg; jb < jend; jb += 32) {
            load_text_block(v.yp, v.nn, jb + 32, tn);
            const uint32_t wn = (jb >> 5) + NW + 1;  // ring: the word entering next
            const uint32_t w0 = (jb >> 5) + WPL * l;   // the lane's first band word
            uint32_t slot = sb + WPL * l;               // WPL * l < RW
            if (slot >= RW) slot -= RW;
            const uint32_t slot4 = 4 * (RING ? slot : w0);
            // columns past the end of a pair's text do not count; a block
            // where no text ends takes the masked-popcount path
            const bool ends_here = in_tile && v.nn > jb && v.nn < jb + 32;
            if (__builtin_amdgcn_ballot_w64(ends_here) == 0) {
                const uint32_t km = (owner && jb + 32 <= v.nn) ? (1u << kbit) : 0u;
                uint32_t unused = 0;
                if constexpr (WPL > 1) {
                    uint32_t kq[WPL];
#pragma unroll
                    for (int q = 0; q < WPL; q++) kq[q] = kw == (uint32_t)q ? km : 0u;
                    myers_blockw<MODE, true, WPL>(peq8, 4 * stride, slot4, tw, Pv, Mv, Z, unused,
                                                  kq, notlast, keep);
                } else
                    myers_block<MODE, true>(peq8, 4 * stride, slot4, tw, Pv[0], Mv[0], Z, unused,
                                            km, kbit, notlast, keep);
            } else {
                uint32_t acc = 0;
                if constexpr (WPL > 1) {
                    const uint32_t km = owner ? (1u << kbit) : 0u;
                    uint32_t kq[WPL];
#pragma unroll
                    for (int q = 0; q < WPL; q++) kq[q] = kw == (uint32_t)q ? km : 0u;
                    myers_blockw<MODE, false, WPL>(peq8, 4 * stride, slot4, tw, Pv, Mv, Z, acc,
                                                   kq, notlast, keep);
                } else {
                    myers_block<MODE, false>(peq8, 4 * stride, slot4, tw, Pv[0], Mv[0], Z, acc, 0u,
                                             kbit, notlast, keep);
                }
                const uint32_t ncol = v.nn > jb ? min(v.nn - jb, 32u) : 0u;
                const uint32_t cmask = ncol >= 32 ? 0xFFFFFFFFu : ((1u << ncol) - 1u);
                if (owner) Z += (uint32_t)__builtin_popcount(acc & cmask);
            }
            if (RING && in_tile) {
                // the entering word, lane c of the tile for symbol c; the slot
                // it takes held word wn - RW = jb/32, which no lane reads any
                // more
                for (uint32_t c = l; c < sigma; c += NL) {
                    const uint32_t word = mask_word(v, c, wn);
                    pq_mine[c * stride + sb] = word;
                    if (sb < WPL) pq_mine[c * stride + sb + RW] = word;
                }
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
            }
            if (RING) sb = sb + 1 == RW ? 0u : sb + 1;
            jdone = jb + 32;
#pragma unroll
            for (int q = 0; q < 8; q++) tw[q] = tn[q];
            const uint32_t cols = min(jdone, v.nn);
            const bool live = owner && !v.skip && v.dstar + cols - Z <= v.Kp && jdone < v.nn;
            if (owner && !live && jstop == NO_LIMIT) jstop = jdone;
            if (__builtin_amdgcn_ballot_w64(live) == 0) break;
        }
        const uint32_t cols = min(jdone, v.nn);
        const uint32_t Vd = v.dstar + cols - Z;
        // Z (hence the decision) lives in the owner lane; every lane of the
        // tile learns it from a ballot
        const bool und_owner =
            owner && act && !v.skip && Vd <= v.Kp && jdone < v.nn && jlim != NO_LIMIT;
        const uint64_t und_mask = __builtin_amdgcn_ballot_w64(und_owner);
        const uint32_t owner_lane = tile * NL + (kstar >> LWB);
        const bool undecided = in_tile && ((und_mask >> (owner_lane & 63)) & 1ull);
        if (act && undecided) {
            // pass 1 stops here: keep the state of the pair for pass 2
#pragma unroll
            for (int q = 0; q < WPL; q++) {
                state[(pidx * NL + l) * 2 * WPL + 2 * q] = Pv[q];
                state[(pidx * NL + l) * 2 * WPL + 2 * q + 1] = Mv[q];
            }
        }
        if (owner && act) {
            if (undecided) {
                aux[pidx] = Z;
            } else {
                uint32_t res = v.skip ? v.Kp + 1 : Vd;
                if (res > v.Kp + 1) res = v.Kp + 1;
                dist[pidx] = (int32_t)res;
                if (aux && !resume) aux[pidx] = DECIDED;
            }
            const uint32_t need = min(min(jdone, jstop), v.nn);
            colsum += (unsigned long long)(need - min(jbeg, need));
        }
    }
    add_columns(columns, colsum);
}

// Persistent form.  The grid stays resident and every tile (the NL lanes of
// one pair) takes the next pair from a device-wide counter as soon as its
// current pair is decided, so a wave never idles on its longest pair and
// nothing is saved between passes.  Pairs decided without any column (length
// gap above the threshold, empty text) are written when taken.  A wave
// leaves once the counter has passed `count` and none of its tiles holds a
// pair; every tile takes at most `count` pairs, so every wave exits.  The
// k-th pair taken is order[k] (or k): the order only schedules, results go
// to dist[pair].
template <int MODE, bool RING>
__global__ void __launch_bounds__(64)
    k_verify_queue(StrSet A, StrSet B, const uint64_t *__restrict__ pairs, uint32_t count,
                   const uint64_t *__restrict__ count_dev, const uint32_t *__restrict__ order,
                   uint32_t K,
                   const uint32_t *__restrict__ Kq, uint32_t sigma, uint32_t NL_arg, uint32_t tpw,
                   uint32_t wpp, uint32_t *__restrict__ next, int32_t *__restrict__ dist,
                   unsigned long long *__restrict__ columns) {
    extern __shared__ uint32_t lds[];
    unsigned long long colsum = 0;  // text columns of the pairs decided here
    const uint32_t NL = lanes_of<MODE>(NL_arg);
    // a count on the device (a join sized on the device): at most `count`
    if (count_dev) count = (uint32_t)min<uint64_t>(*count_dev, count);
    const uint32_t lane = threadIdx.x;
    const uint32_t tile = lane / NL, l = lane - tile * NL;
    const bool in_tile = tile < tpw;
    const uint32_t RW = wpp;
    const uint32_t stride = RING ? 2 * RW : wpp;
    const uint32_t tile_words = tile_words_for(sigma, stride);
    uint64_t last = 0;
    for (uint32_t q = 0; q < 64; q++)
        if ((q / NL) >= tpw || (q % NL) == NL - 1) last |= 1ull << q;
    const uint64_t notlast = ~last;
    const uint32_t keep = (l == NL - 1 || !in_tile) ? 0u : 0xFFFFFFFFu;
    uint32_t *pq_mine = lds + (in_tile ? tile : 0) * tile_words;
    const uint8_t *peq8 = (const uint8_t *)pq_mine;

    PairView v = view_pair(A, B, pairs, Kq, K, 0, false);
    uint32_t pidx = 0;
    bool active = in_tile;  // may still hold or take pairs
    bool need = in_tile;    // holds no pair
    bool owner = false;
    uint32_t jb = 0, Pv = 0, Mv = 0, Z = 0, kstar = 0, kbit = 0;
    uint32_t tw[8];
#pragma unroll
    for (int q = 0; q < 8; q++) tw[q] = 0;

    for (;;) {
        // ---- tiles without a pair take the next one
        for (;;) {
            if (__builtin_amdgcn_ballot_w64(need && l == 0) == 0) break;
            uint32_t got = 0xFFFFFFFFu;
            if (need && l == 0) got = atomicAdd(next, 1u);
            got = (uint32_t)__shfl((int)got, (int)(tile * NL), 64);
            bool fresh = false;
            if (need) {
                if (got >= count) {
                    need = false;
                    active = false;
                    owner = false;
                    v.m = 0;
                    v.nn = 0;
                    v.W = 0;
                } else {
                    pidx = order ? order[got] : got;
                    v = view_pair(A, B, pairs, Kq, K, pidx, true);
                    kstar = v.O + v.dstar;
                    owner = (kstar >> 5) == l;
                    kbit = kstar & 31;
                    jb = 0;
                    Z = 0;
                    // D[i][0] = |i|: bit k holds row k - O, rows <= 0 have delta -1
                    const int lo = 32 * (int)l;
                    const int Oi = (int)v.O;
                    Mv = Oi >= lo + 31 ? ~0u : (Oi < lo ? 0u : (1u << (Oi - lo + 1)) - 1u);
                    Pv = ~Mv;
                    if (v.skip || v.nn == 0) {
                        // decided without a column: length gap > K_p, or ED = |x|
                        if (owner) {
                            const uint32_t res = v.skip ? v.Kp + 1 : min(v.dstar, v.Kp + 1);
                            dist[pidx] = (int32_t)res;
                        }
                    } else {
                        need = false;
                        fresh = true;
                    }
                }
            }
            if (fresh) {
                fill_tile<RING>(pq_mine, v, l, NL, sigma, stride, RW, wpp, 0u,
                                RING ? NL + 1 : wpp);
                load_text_block(v.yp, v.nn, 0, tw);
            }
        }
        if (__builtin_amdgcn_ballot_w64(active) == 0) break;

        // ---- one 32-column block of every tile that holds a pair
        uint32_t tn[8];
        load_text_block(v.yp, v.nn, jb + 32, tn);
        const uint32_t wn = (jb >> 5) + NL + 1;  // ring: the word entering next
        const uint32_t slot4 = 4 * (RING ? (((jb >> 5) + l) & (RW - 1)) : ((jb >> 5) + l));
        const bool ends_here = active && v.nn > jb && v.nn < jb + 32;
        if (__builtin_amdgcn_ballot_w64(ends_here) == 0) {
            const uint32_t km = (owner && jb + 32 <= v.nn) ? (1u << kbit) : 0u;
            uint32_t unused = 0;
            myers_block<MODE, true>(peq8, 4 * stride, slot4, tw, Pv, Mv, Z, unused, km, kbit,
                                    notlast, keep);
        } else {
            uint32_t acc = 0;
            myers_block<MODE, false>(peq8, 4 * stride, slot4, tw, Pv, Mv, Z, acc, 0u, kbit,
                                     notlast, keep);
            const uint32_t ncol = v.nn > jb ? min(v.nn - jb, 32u) : 0u;
            const uint32_t cmask = ncol >= 32 ? 0xFFFFFFFFu : ((1u << ncol) - 1u);
            if (owner) Z += (uint32_t)__builtin_popcount(acc & cmask);
        }
        if (RING && active) {
            // the entering word, lane c of the tile for symbol c
            const uint32_t sl = wn & (RW - 1);
            for (uint32_t c = l; c < sigma; c += NL) {
                const uint32_t word = mask_word(v, c, wn);
                pq_mine[c * stride + sl] = word;
                pq_mine[c * stride + sl + RW] = word;
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        if (active) jb += 32;
#pragma unroll
        for (int q = 0; q < 8; q++) tw[q] = tn[q];

        // ---- decisions live in the owner lane; the tile learns them by ballot
        const uint32_t cols = min(jb, v.nn);
        const uint32_t Vd = v.dstar + cols - Z;
        const bool fin_owner = owner && active && !(Vd <= v.Kp && jb < v.nn);
        const uint64_t fin = __builtin_amdgcn_ballot_w64(fin_owner);
        const uint32_t owner_lane = tile * NL + (kstar >> 5);
        const bool tile_fin = in_tile && active && ((fin >> (owner_lane & 63)) & 1ull);
        if (fin_owner) {
            dist[pidx] = (int32_t)min(Vd, v.Kp + 1);
            colsum += (unsigned long long)cols;
        }
        if (tile_fin) {
            need = true;
            owner = false;
        }
    }
    add_columns(columns, colsum);
}

// ---------------------------------------------------------------------------
// Lane form: one pair per lane.  The band's NW words live in the lane's own
// registers, so the W-bit addition is a chain of add-with-carry instructions
// and the one-bit shift a funnel shift between neighbouring registers -- no
// ballots and no cross-lane moves, about ten VALU instructions per 32 band
// cells and column.
//
//  * Each lane keeps in LDS, one row per symbol, the match-mask words of the
//    NW+1 band words its next 32 columns read; after every block the rows
//    move down one word and the entering word is taken from the pattern's
//    precomputed masks.
//  * Row `sigma` is all ones: the symbol of padding columns after the end of
//    the text.  In a column where every cell matches, every diagonal keeps
//    its value (the match move keeps it and no diagonal ever decreases), so
//    the whole state stays fixed.  A pair whose text ends inside a block
//    therefore runs the whole block, and its state at the block end is its
//    state at the last text column.
//  * The value on diagonal d* is not counted column by column.  The kernel
//    counts the top diagonal instead (band bit 0: one fixed register, 0 or 1
//    added per column as for any diagonal) and, at block ends, reads the
//    value on d* as the top value plus the vertical deltas of bits 1..k*.
//  * Pairs come from a device-wide counter, one per lane.  Lanes whose pair is
//    decided take the next one before the following block, and the whole wave
//    fills the mask windows of the pairs just taken.
template <int NW>
__device__ inline void lane_state_init(uint32_t O, uint32_t (&Pv)[NW], uint32_t (&Mv)[NW]) {
    // D[i][0] = |i|: bit k holds row k - O, rows <= 0 have delta -1
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const int d = (int)O - 32 * w;
        const uint32_t mv = d >= 31 ? 0xFFFFFFFFu : (d < 0 ? 0u : (2u << d) - 1u);
        Mv[w] = mv;
        Pv[w] = ~mv;
    }
}

// Text of columns jb+1 .. jb+32 with the columns past nn set to the
// match-all symbol `pad`.
__device__ inline void lane_text_block(const uint8_t *y, uint32_t nn, uint32_t jb, uint32_t pad,
                                       uint32_t tw[8]) {
    load_text_block(y, nn, jb, tw);
    const uint32_t r = nn > jb ? nn - jb : 0u;
    const uint32_t fill = pad * 0x01010101u;
#pragma unroll
    for (uint32_t q = 0; q < 8; q++) {
        const uint32_t v = r > 4 * q ? r - 4 * q : 0u;
        const uint32_t keep = v >= 4 ? 0xFFFFFFFFu : ((1u << (8 * v)) - 1u);
        tw[q] = (tw[q] & keep) | (fill & ~keep);
    }
}

// 32 columns of one pair per lane.  Row c of the lane's window holds the
// match-mask words of band words jb/32 .. jb/32+NW for symbol c.  The words
// of column s+1 are read while column s is computed; a scheduling barrier
// per column keeps the compiler from hoisting the reads of every column of
// the block at once (which would take hundreds of registers).
template <int NW>
__device__ inline void lane_block(const uint32_t *win, const uint32_t tw[8], uint32_t (&Pv)[NW],
                                  uint32_t (&Mv)[NW], uint32_t &Zt) {
    const uint8_t *w8 = (const uint8_t *)win;
    uint32_t cur[NW + 1], nxt[NW + 1];
    {
        const uint32_t *src = (const uint32_t *)(w8 + __umul24(tw[0] & 0xFFu, 4u * (NW + 1)));
#pragma unroll
        for (int w = 0; w <= NW; w++) cur[w] = src[w];
    }
#pragma unroll
    for (uint32_t s = 0; s < 32; s++) {
        if (s < 31) {
            const uint32_t c = (tw[(s + 1) >> 2] >> (8 * ((s + 1) & 3))) & 0xFFu;
            const uint32_t *src = (const uint32_t *)(w8 + __umul24(c, 4u * (NW + 1)));
#pragma unroll
            for (int w = 0; w <= NW; w++) nxt[w] = src[w];
        }
        uint32_t Xv[NW + 1], Ph[NW], Mh[NW];
        uint64_t cy = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const uint32_t eq = s == 0 ? cur[w] : __builtin_amdgcn_alignbit(cur[w + 1], cur[w], s);
            Xv[w] = eq | Mv[w];
            uint32_t sum;
            if (NW == 1)
                sum = (eq & Pv[w]) + Pv[w];
            else if (w == 0)
                sum = add_carry_mask(eq & Pv[w], Pv[w], cy);
            else
                sum = add_carry_chain(eq & Pv[w], Pv[w], cy, cy);
            const uint32_t Xh = (sum ^ Pv[w]) | eq;
            Ph[w] = Mv[w] | ~(Xh | Pv[w]);
            Mh[w] = Pv[w] & Xh;
        }
        Xv[NW] = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const uint32_t Xv1 = __builtin_amdgcn_alignbit(Xv[w + 1], Xv[w], 1);
            if (w == 0) Zt = popc_acc((Xv1 | Mh[0]) & 1u, Zt);
            Pv[w] = Mh[w] | ~(Xv1 | Ph[w]);
            Mv[w] = Ph[w] & Xv1;
        }
        // the state is materialised every column: left free, the compiler
        // re-associates the bit operations across columns and keeps every
        // column's intermediates alive to the end of the block
#pragma unroll
        for (int w = 0; w < NW; w++) asm volatile("" : "+v"(Pv[w]), "+v"(Mv[w]));
#pragma unroll
        for (int w = 0; w <= NW; w++) cur[w] = nxt[w];
        __builtin_amdgcn_sched_barrier(0);
    }
}

__device__ inline uint32_t readlane_u32(uint32_t x, uint32_t L) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)L);
}

template <int NW, int SIGMAX>
__global__ void __launch_bounds__(64)
    k_verify_lane(StrSet A, StrSet B, const uint64_t *__restrict__ pairs, uint32_t count,
                  const uint64_t *__restrict__ count_dev, const uint32_t *__restrict__ order,
                  uint32_t K, const uint32_t *__restrict__ Kq, uint32_t sigma, uint32_t region,
                  uint32_t *__restrict__ next, int32_t *__restrict__ dist,
                  unsigned long long *__restrict__ columns) {
    constexpr uint32_t RS = NW + 1;  // words per symbol row of a window
    extern __shared__ uint32_t lds[];
    unsigned long long colsum = 0;  // text columns of the pairs decided here
    if (count_dev) count = (uint32_t)min<uint64_t>(*count_dev, count);
    const uint32_t lane = threadIdx.x;
    uint32_t *win = lds + lane * region;
#pragma unroll
    for (uint32_t w = 0; w < RS; w++) win[sigma * RS + w] = 0xFFFFFFFFu;

    PairView v = view_pair(A, B, pairs, Kq, K, 0, false);
    uint32_t pidx = 0, jb = 0, Zt = 0, kstar = 0;
    uint32_t Pv[NW], Mv[NW], tw[8];
#pragma unroll
    for (int w = 0; w < NW; w++) Pv[w] = Mv[w] = 0;
#pragma unroll
    for (int q = 0; q < 8; q++) tw[q] = 0;
    bool has = false;     // holds an undecided pair
    bool drained = false; // the counter has passed `count` for this lane

    for (;;) {
        // ---- lanes without a pair take the next ones; pairs decided without
        //      any column (length gap above the threshold, empty text) are
        //      written at once
        bool fresh = false;
        for (;;) {
            const bool need = !has && !drained;
            const uint64_t nm = __builtin_amdgcn_ballot_w64(need);
            if (nm == 0) break;
            const uint32_t leader = (uint32_t)__builtin_ctzll(nm);
            uint32_t got = 0;
            if (lane == leader) got = atomicAdd(next, (uint32_t)__popcll(nm));
            got = readlane_u32(got, leader);
            if (need) {
                const uint32_t k = got + (uint32_t)__popcll(nm & ((1ull << lane) - 1ull));
                if (k >= count) {
                    drained = true;
                } else {
                    pidx = order ? order[k] : k;
                    v = view_pair(A, B, pairs, Kq, K, pidx, true);
                    if (v.skip || v.nn == 0) {
                        dist[pidx] = (int32_t)(v.skip ? v.Kp + 1 : min(v.dstar, v.Kp + 1));
                    } else {
                        has = true;
                        fresh = true;
                        jb = 0;
                        Zt = 0;
                        kstar = v.O + v.dstar;
                        lane_state_init<NW>(v.O, Pv, Mv);
                        lane_text_block(v.yp, v.nn, 0, sigma, tw);
                    }
                }
            }
        }
        if (__builtin_amdgcn_ballot_w64(has) == 0) break;
        // ---- the windows of the pairs just taken
        if (SIGMAX <= 4) {
            // small alphabets: the whole wave fills each fresh lane's window
            // in turn (a handful of words per lane)
            uint64_t fm = __builtin_amdgcn_ballot_w64(fresh);
            while (fm) {
                const uint32_t L = (uint32_t)__builtin_ctzll(fm);
                fm &= fm - 1;
                PairView u = v;
                const uint64_t mp = (uint64_t)(uintptr_t)v.mw;
                u.mw = (const uint32_t *)(uintptr_t)(
                    ((uint64_t)readlane_u32((uint32_t)(mp >> 32), L) << 32) |
                    readlane_u32((uint32_t)mp, L));
                u.W = readlane_u32(v.W, L);
                u.O = readlane_u32(v.O, L);
                uint32_t *wl = lds + L * region;
                for (uint32_t t = lane; t < sigma * RS; t += 64) {
                    const uint32_t c = t / RS, w = t - c * RS;
                    wl[c * RS + w] = mask_word(u, c, w);
                }
            }
            // other lanes wrote these windows: the barrier orders their
            // writes before the owners' reads
            __syncthreads();
        } else if (fresh) {
            // larger alphabets: every fresh lane fills its own sigma rows at
            // once (independent loads, in parallel over the fresh lanes,
            // where a wave-wide fill would take one global latency per lane).
            // Window word w of a row is the funnel shift of pattern mask words
            // q0 + w and q0 + w + 1 (as mask_word), so a row takes RS + 1
            // loads; the last one is kept for the next block's entering word
            const int32_t p0 = -(int32_t)v.O - 1;
            const int32_t q0 = p0 >> 5;  // floor
            const uint32_t sh = (uint32_t)p0 & 31u;
            for (uint32_t c = 0; c < sigma; c++) {
                const uint32_t *mc = v.mw + (size_t)c * v.W;
                uint32_t t[RS + 1];
#pragma unroll
                for (uint32_t i = 0; i <= RS; i++) {
                    const int32_t q = q0 + (int32_t)i;
                    t[i] = (uint32_t)q < v.W ? mc[q] : 0u;
                }
#pragma unroll
                for (uint32_t w = 0; w < RS; w++)
                    win[c * RS + w] = __builtin_amdgcn_alignbit(t[w + 1], t[w], sh);
                win[(sigma + 1) * RS + c] = t[RS];
            }
        }

        // ---- one block of 32 columns; the next block's text and entering
        //      mask words are fetched first (none once the text ends in this
        //      block).  Larger alphabets keep the entering word's low source
        //      word from the previous block (stored after the rows), so a
        //      symbol costs one load per block
        uint32_t tn[8];
        lane_text_block(v.yp, has ? v.nn : 0u, jb + 32, sigma, tn);
        const uint32_t wn = (jb >> 5) + RS;
        const bool more = has && jb + 32 < v.nn;
        uint32_t nwd[SIGMAX];
        if (SIGMAX <= 4) {
#pragma unroll
            for (uint32_t c = 0; c < (uint32_t)SIGMAX; c++)
                nwd[c] = (more && c < sigma) ? mask_word(v, c, wn) : 0u;
        } else {
            const int32_t p0 = 32 * (int32_t)wn - (int32_t)v.O - 1;
            const int32_t q = (p0 >> 5) + 1;  // the high source word
            const uint32_t sh = (uint32_t)p0 & 31u;
#pragma unroll
            for (uint32_t c = 0; c < (uint32_t)SIGMAX; c++) {
                nwd[c] = 0u;
                if (more && c < sigma) {
                    const uint32_t hi = (uint32_t)q < v.W ? v.mw[(size_t)c * v.W + q] : 0u;
                    uint32_t *keep_lo = win + (sigma + 1) * RS + c;
                    nwd[c] = __builtin_amdgcn_alignbit(hi, *keep_lo, sh);
                    *keep_lo = hi;
                }
            }
        }
        lane_block<NW>(win, tw, Pv, Mv, Zt);
#pragma unroll
        for (uint32_t c = 0; c < (uint32_t)SIGMAX; c++) {
            if (c < sigma) {
                uint32_t *row = win + c * RS;
                uint32_t t[RS];
#pragma unroll
                for (uint32_t w = 1; w < RS; w++) t[w] = row[w];
#pragma unroll
                for (uint32_t w = 1; w < RS; w++) row[w - 1] = t[w];
                row[NW] = nwd[c];
            }
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        jb += 32;
#pragma unroll
        for (int q = 0; q < 8; q++) tw[q] = tn[q];

        // ---- decisions: the value on d* is the top value plus the vertical
        //      deltas of bits 1..k*
        if (has) {
            uint32_t P = 0, M = 0;
#pragma unroll
            for (int w = 0; w < NW; w++) {
                const int d = (int)kstar - 32 * w;
                uint32_t mk = d >= 31 ? 0xFFFFFFFFu : (d < 0 ? 0u : (2u << d) - 1u);
                if (w == 0) mk &= ~1u;
                P = popc_acc(Pv[w] & mk, P);
                M = popc_acc(Mv[w] & mk, M);
            }
            const uint32_t Vd = v.O + jb - Zt + P - M;
            if (Vd > v.Kp || jb >= v.nn) {
                dist[pidx] = (int32_t)min(Vd, v.Kp + 1);
                colsum += (unsigned long long)min(jb, v.nn);
                has = false;
            }
        }
    }
    add_columns(columns, colsum);
}

// ---------------------------------------------------------------------------
// Form grouped by pattern ("verify_mode" 3).  The candidates are ordered by
// their pattern (the longer string of the pair, as view_pair takes it) and
// cut into chunks of at most 64 pairs of one pattern.  A wave takes a chunk:
// the whole wave copies the pattern's precomputed match masks into LDS once
// (coalesced: a pattern's masks are contiguous), then each lane runs one pair
// of the chunk, its band in registers as in the lane form.  No lane has a
// window of its own to fill from scattered loads and shift block by block:
// band word w at column s of block jb is the funnel shift of pattern mask
// words q and q + 1, q = floor((jb + s - O - 1) / 32) + w (mask_word's bits),
// read from the shared rows, which carry `lead` zero words before the pattern
// and NW + 2 after it.  Worth it when strings have many candidate partners
// (the mask copy is paid once per chunk instead of once per pair) and for
// large alphabets (a few KB of LDS per wave instead of a window per lane).
//
// Chunks: key = pattern of pair k, with bit PB set when the pattern is
// longer than `lim` letters (pairs past a count on the device get the key
// 0xFFFFFFFF), sorted on PB + 1 bits; a chunk starts where the key changes
// and every 64 pairs within a run of one key.  The chunks of short patterns
// thus come first and run with LDS rows sized for `lim` letters (many waves
// per CU); the few long ones follow in a launch of their own.

__global__ void k_grp_keys(const uint64_t *__restrict__ off, const uint64_t *__restrict__ pairs,
                           uint64_t count, const uint64_t *__restrict__ count_dev, uint32_t PB,
                           uint64_t lim, uint32_t *__restrict__ key,
                           uint32_t *__restrict__ val) {
    const uint64_t live = count_dev ? min(*count_dev, count) : count;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count;
         k += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t pat = 0xFFFFFFFFu;
        if (k < live) {
            const uint64_t code = pairs[k];
            const uint32_t a = (uint32_t)(code >> 32), b = (uint32_t)code;
            const uint64_t la = off[a + 1] - off[a], lb = off[b + 1] - off[b];
            pat = la >= lb ? a : b;  // view_pair's pattern
            if ((la >= lb ? la : lb) > lim) pat |= 1u << PB;
        }
        key[k] = pat;
        val[k] = (uint32_t)k;
    }
}

// Run starts of the sorted keys, into a table indexed by the key's class
// and pattern (n slots per class); every key of a run reads the same slot.
__device__ inline uint32_t grp_slot(uint32_t key, uint32_t PB, uint32_t n) {
    return PB >= 32 ? key : (key & ((1u << PB) - 1u)) + ((key >> PB) & 1u) * n;
}

__global__ void k_grp_run_starts(const uint32_t *__restrict__ key, uint64_t count,
                                 const uint64_t *__restrict__ count_dev, uint32_t PB, uint32_t n,
                                 uint32_t *__restrict__ rstart) {
    const uint64_t live = count_dev ? min(*count_dev, count) : count;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < live;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = key[k];
        if (k == 0 || key[k - 1] != x) rstart[grp_slot(x, PB, n)] = (uint32_t)k;
    }
}

__global__ void k_grp_chunk_flags(const uint32_t *__restrict__ key, uint64_t count,
                                  const uint64_t *__restrict__ count_dev, uint32_t PB, uint32_t n,
                                  const uint32_t *__restrict__ rstart,
                                  uint32_t *__restrict__ flags) {
    const uint64_t live = count_dev ? min(*count_dev, count) : count;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count;
         k += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t f = 0;
        if (k < live) f = ((k - rstart[grp_slot(key[k], PB, n)]) & 63u) == 0 ? 1u : 0u;
        flags[k] = f;
    }
}

__global__ void k_grp_chunk_starts(const uint32_t *__restrict__ flags,
                                   const uint32_t *__restrict__ pos, uint64_t count,
                                   const uint64_t *__restrict__ count_dev,
                                   const uint64_t *__restrict__ nchunks,
                                   uint32_t *__restrict__ start) {
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count;
         k += (uint64_t)gridDim.x * blockDim.x)
        if (flags[k]) start[pos[k]] = (uint32_t)k;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        start[*nchunks] = (uint32_t)(count_dev ? min(*count_dev, count) : count);
}

// The first chunk of a long pattern (bit PB of its first key; PB >= 32:
// none), by bisection over the chunks: range[0] = 0, range[1] = that chunk,
// range[2] = chunks.
__global__ void k_grp_split(const uint32_t *__restrict__ key, const uint32_t *__restrict__ start,
                            const uint64_t *__restrict__ nchunks, uint32_t PB,
                            uint64_t *__restrict__ range) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint64_t nch = *nchunks;
    uint64_t lo = PB >= 32 ? nch : 0, hi = nch;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if ((key[start[mid]] >> PB) & 1u)
            hi = mid;
        else
            lo = mid + 1;
    }
    range[0] = 0;
    range[1] = lo;
    range[2] = nch;
}

// 32 columns of one pair per lane, the pattern's rows shared in LDS: row c
// at rows + c * S (lead zero words, then the pattern's words).  b0 = jb - O - 1
// (the pattern bit of band bit 0 at the block's first column).
template <int NW>
__device__ inline void grp_block(const uint32_t *rows, uint32_t S, int32_t b0,
                                 const uint32_t tw[8], uint32_t (&Pv)[NW], uint32_t (&Mv)[NW],
                                 uint32_t &Zt) {
    uint32_t cur[NW + 1], nxt[NW + 1];
    auto fetch = [&](uint32_t s, uint32_t (&o)[NW + 1]) {
        const uint32_t c = (tw[s >> 2] >> (8 * (s & 3))) & 0xFFu;
        const int32_t p = b0 + (int32_t)s;
        const uint32_t *src = rows + __umul24(c, S) + (p >> 5);
#pragma unroll
        for (int w = 0; w <= NW; w++) o[w] = src[w];
    };
    fetch(0, cur);
#pragma unroll
    for (uint32_t s = 0; s < 32; s++) {
        if (s < 31) fetch(s + 1, nxt);
        const uint32_t sh = (uint32_t)(b0 + (int32_t)s) & 31u;
        uint32_t Xv[NW + 1], Ph[NW], Mh[NW];
        uint64_t cy = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const uint32_t eq = __builtin_amdgcn_alignbit(cur[w + 1], cur[w], sh);
            Xv[w] = eq | Mv[w];
            uint32_t sum;
            if (NW == 1)
                sum = (eq & Pv[w]) + Pv[w];
            else if (w == 0)
                sum = add_carry_mask(eq & Pv[w], Pv[w], cy);
            else
                sum = add_carry_chain(eq & Pv[w], Pv[w], cy, cy);
            const uint32_t Xh = (sum ^ Pv[w]) | eq;
            Ph[w] = Mv[w] | ~(Xh | Pv[w]);
            Mh[w] = Pv[w] & Xh;
        }
        Xv[NW] = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const uint32_t Xv1 = __builtin_amdgcn_alignbit(Xv[w + 1], Xv[w], 1);
            if (w == 0) Zt = popc_acc((Xv1 | Mh[0]) & 1u, Zt);
            Pv[w] = Mh[w] | ~(Xv1 | Ph[w]);
            Mv[w] = Ph[w] & Xv1;
        }
#pragma unroll
        for (int w = 0; w < NW; w++) asm volatile("" : "+v"(Pv[w]), "+v"(Mv[w]));
#pragma unroll
        for (int w = 0; w <= NW; w++) cur[w] = nxt[w];
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int NW>
__global__ void __launch_bounds__(64)
    k_verify_grp(StrSet A, const uint64_t *__restrict__ pairs, const uint32_t *__restrict__ order,
                 const uint32_t *__restrict__ cstart, const uint64_t *__restrict__ crange,
                 uint32_t K, const uint32_t *__restrict__ Kq, uint32_t sigma, uint32_t S,
                 uint32_t lead, uint32_t *__restrict__ next, int32_t *__restrict__ dist,
                 unsigned long long *__restrict__ columns) {
    extern __shared__ uint32_t rows[];  // (sigma + 1) rows of S words
    unsigned long long colsum = 0;  // text columns of the pairs decided here
    const uint32_t lane = threadIdx.x;
    // chunks [crange[0], crange[1])
    const uint32_t c0 = (uint32_t)crange[0], nch = (uint32_t)crange[1];
    for (;;) {
        uint32_t ch = 0;
        if (lane == 0) ch = c0 + atomicAdd(next, 1u);
        ch = readlane_u32(ch, 0);
        if (ch >= nch) break;
        const uint32_t cs = cstart[ch], ce = cstart[ch + 1];
        const bool act = cs + lane < ce;
        const uint32_t pidx = act ? order[cs + lane] : 0u;
        PairView v = view_pair(A, A, pairs, Kq, K, pidx, act);
        // the chunk's pattern (every pair of the chunk has it), from its first pair
        const uint64_t c0 = pairs[order[cs]];
        const uint32_t a0 = (uint32_t)(c0 >> 32), b0i = (uint32_t)c0;
        const uint64_t la0 = A.off[a0 + 1] - A.off[a0], lb0 = A.off[b0i + 1] - A.off[b0i];
        const uint32_t pat = la0 >= lb0 ? a0 : b0i;
        const uint32_t m = (uint32_t)(la0 >= lb0 ? la0 : lb0);
        const uint32_t W = (m + 31) / 32;
        const uint32_t *mw = A.mw + A.moff[pat];
        const uint32_t used = lead + W + NW + 2;  // words of each row this pattern needs
        // the previous chunk's lanes are done with the rows
        __syncthreads();
        for (uint32_t t = lane; t < (sigma + 1) * used; t += 64) {
            const uint32_t c = t / used, i = t - c * used;
            uint32_t x = 0xFFFFFFFFu;  // the padding symbol matches everything
            if (c < sigma) x = (i >= lead && i - lead < W) ? mw[(size_t)c * W + (i - lead)] : 0u;
            rows[c * S + i] = x;
        }
        __syncthreads();
        bool has = false;
        uint32_t Pv[NW], Mv[NW], tw[8], Zt = 0, kstar = 0, jb = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) Pv[w] = Mv[w] = 0;
        if (act) {
            if (v.skip || v.nn == 0) {
                dist[pidx] = (int32_t)(v.skip ? v.Kp + 1 : min(v.dstar, v.Kp + 1));
            } else {
                has = true;
                kstar = v.O + v.dstar;
                lane_state_init<NW>(v.O, Pv, Mv);
            }
        }
        lane_text_block(v.yp, has ? v.nn : 0u, 0, sigma, tw);
        while (__builtin_amdgcn_ballot_w64(has)) {
            uint32_t tn[8];
            lane_text_block(v.yp, has ? v.nn : 0u, jb + 32, sigma, tn);
            // lanes without a pair run on the padding row (all ones): their
            // state stays fixed and nothing of it is read
            grp_block<NW>(rows + lead, S, (int32_t)jb - (int32_t)v.O - 1, tw, Pv, Mv, Zt);
            jb += 32;
#pragma unroll
            for (int q = 0; q < 8; q++) tw[q] = tn[q];
            if (has) {
                uint32_t P = 0, M = 0;
#pragma unroll
                for (int w = 0; w < NW; w++) {
                    const int d = (int)kstar - 32 * w;
                    uint32_t mk = d >= 31 ? 0xFFFFFFFFu : (d < 0 ? 0u : (2u << d) - 1u);
                    if (w == 0) mk &= ~1u;
                    P = popc_acc(Pv[w] & mk, P);
                    M = popc_acc(Mv[w] & mk, M);
                }
                const uint32_t Vd = v.O + jb - Zt + P - M;
                if (Vd > v.Kp || jb >= v.nn) {
                    dist[pidx] = (int32_t)min(Vd, v.Kp + 1);
                    colsum += (unsigned long long)min(jb, v.nn);
                    has = false;
                }
            }
        }
    }
    add_columns(columns, colsum);
}

using GrpKernel = void (*)(StrSet, const uint64_t *, const uint32_t *, const uint32_t *,
                           const uint64_t *, uint32_t, const uint32_t *, uint32_t, uint32_t,
                           uint32_t, uint32_t *, int32_t *, unsigned long long *);

GrpKernel grp_kernel(uint32_t nw) {
    switch (nw) {
        case 1: return k_verify_grp<1>;
        case 2: return k_verify_grp<2>;
        case 3: return k_verify_grp<3>;
        case 4: return k_verify_grp<4>;
        case 5: return k_verify_grp<5>;
        case 6: return k_verify_grp<6>;
        case 7: return k_verify_grp<7>;
        case 8: return k_verify_grp<8>;
        case 9: return k_verify_grp<9>;
        case 10: return k_verify_grp<10>;
        case 11: return k_verify_grp<11>;
        case 12: return k_verify_grp<12>;
        case 13: return k_verify_grp<13>;
        case 14: return k_verify_grp<14>;
        case 15: return k_verify_grp<15>;
        case 16: return k_verify_grp<16>;
        default: return nullptr;
    }
}

// ---------------------------------------------------------------------------
// Split form: KL lanes per pair (KL = 2, 4, 8 or 16, one DPP row at most),
// each holding WPL consecutive words of the band in registers.  Inside a lane
// the addition is an add-with-carry chain and the shift a funnel shift; only
// the lane boundaries need the carry-lookahead (two ballots and scalar
// arithmetic, then the carry-in rippled through the lane's words) and one DPP
// move for the shift.  The lane form's windows, padding symbol, top-diagonal
// count and pair counter carry over, with one window per pair that its KL
// lanes share.  Compared with one pair per lane, a pair's columns take KL
// times fewer steps one after the other, which matters when there are few
// pairs per lane of the grid and they differ much in length.

// s = a + (bit `lane` of cin); carry-outs of every lane in cout.
__device__ inline uint32_t add_carry_ripple(uint32_t a, uint64_t cin, uint64_t &cout) {
    uint32_t s;
    asm("v_addc_co_u32 %0, %1, %2, 0, %3" : "=v"(s), "=s"(cout) : "v"(a), "s"(cin));
    return s;
}

// Dwords q0 .. q0+nq-1 (nq <= TQ) of the text of columns jb+1 .. jb+32, the
// columns past nn set to the match-all symbol `pad`.  Reads stay within
// y[0 .. nn+35], as for load_text_block.
template <int TQ>
__device__ inline void text_part(const uint8_t *y, uint32_t nn, uint32_t jb, uint32_t pad,
                                 uint32_t q0, uint32_t nq, uint32_t (&out)[TQ]) {
    const uint32_t fill = pad * 0x01010101u;
#pragma unroll
    for (int i = 0; i < TQ; i++) out[i] = fill;
    if (jb >= nn || q0 >= 8) return;
    const uintptr_t a = (uintptr_t)(y + jb);
    const uint32_t *base = (const uint32_t *)(a & ~(uintptr_t)3) + q0;
    const uint32_t sh = (uint32_t)(a & 3) * 8;
    uint32_t w[TQ + 1];
#pragma unroll
    for (int i = 0; i <= TQ; i++) w[i] = (uint32_t)i <= nq ? base[i] : 0u;
    const uint32_t r = nn - jb;
#pragma unroll
    for (int i = 0; i < TQ; i++) {
        const uint32_t q = q0 + i;
        const uint32_t v = r > 4 * q ? r - 4 * q : 0u;
        const uint32_t keep = v >= 4 ? 0xFFFFFFFFu : ((1u << (8 * v)) - 1u);
        out[i] = (__builtin_amdgcn_alignbit(w[i + 1], w[i], sh) & keep) | (fill & ~keep);
    }
}

// The WPL+1 window words of a lane: its WPL words in as few 16- or 8-byte
// LDS reads as they allow (rows and lane slices are 16-byte aligned when WPL
// is a multiple of 4), then the first word of the next lane.
template <int WPL>
__device__ inline void window_words(const uint32_t *src, uint32_t (&o)[WPL + 1]) {
    if constexpr (WPL % 4 == 0) {
#pragma unroll
        for (int i = 0; i < WPL / 4; i++) {
            const uint4 q = ((const uint4 *)src)[i];
            o[4 * i] = q.x;
            o[4 * i + 1] = q.y;
            o[4 * i + 2] = q.z;
            o[4 * i + 3] = q.w;
        }
    } else if constexpr (WPL % 2 == 0) {
#pragma unroll
        for (int i = 0; i < WPL / 2; i++) {
            const uint2 q = ((const uint2 *)src)[i];
            o[2 * i] = q.x;
            o[2 * i + 1] = q.y;
        }
    } else {
#pragma unroll
        for (int w = 0; w < WPL; w++) o[w] = src[w];
    }
    o[WPL] = src[WPL];
}

// 32 columns of a pair whose band is split over its tile's lanes.  `wl` is
// the lane's first window word, `txt` the tile's 32 text symbols in LDS.  The
// symbol of column s+2 and the words of column s+1 are read while column s is
// computed; a scheduling barrier per column bounds the registers.
template <int WPL>
__device__ inline void split_block(const uint32_t *wl, uint32_t rs4, const uint8_t *txt,
                                   uint32_t (&Pv)[WPL], uint32_t (&Mv)[WPL], uint32_t &Zt,
                                   uint64_t notlast, uint32_t keep) {
    const uint8_t *w8 = (const uint8_t *)wl;
    uint32_t cur[WPL + 1], nxt[WPL + 1];
    window_words<WPL>((const uint32_t *)(w8 + __umul24((uint32_t)txt[0], rs4)), cur);
    uint32_t cn = txt[1];
#pragma unroll
    for (uint32_t s = 0; s < 32; s++) {
        if (s < 31) {
            window_words<WPL>((const uint32_t *)(w8 + __umul24(cn, rs4)), nxt);
            if (s < 30) cn = txt[s + 2];
        }
        uint32_t eq[WPL], sum[WPL], Xv[WPL + 1], Ph[WPL], Mh[WPL];
        uint64_t cy = 0;
        uint32_t all = 0xFFFFFFFFu;
#pragma unroll
        for (int w = 0; w < WPL; w++) {
            eq[w] = s == 0 ? cur[w] : __builtin_amdgcn_alignbit(cur[w + 1], cur[w], s);
            Xv[w] = eq[w] | Mv[w];
            if (w == 0)
                sum[w] = add_carry_mask(eq[w] & Pv[w], Pv[w], cy);
            else
                sum[w] = add_carry_chain(eq[w] & Pv[w], Pv[w], cy, cy);
            all &= sum[w];
        }
        // carries across the pair's lanes: G = carry out of the lane, P = the
        // lane's words are all ones (a carry in passes through)
        uint64_t G = cy & notlast;
        uint64_t P = __builtin_amdgcn_ballot_w64(all == 0xFFFFFFFFu) & notlast;
        const uint64_t cin = ((G | P) + G) ^ P;
        uint64_t rc = cin;
#pragma unroll
        for (int w = 0; w < WPL; w++) sum[w] = add_carry_ripple(sum[w], rc, rc);
#pragma unroll
        for (int w = 0; w < WPL; w++) {
            const uint32_t Xh = (sum[w] ^ Pv[w]) | eq[w];
            Ph[w] = Mv[w] | ~(Xh | Pv[w]);
            Mh[w] = Pv[w] & Xh;
        }
        // word 0 of the next lane of the pair (row_shl:1; zero above the band)
        Xv[WPL] = (uint32_t)__builtin_amdgcn_mov_dpp((int)Xv[0], 0x101, 0xf, 0xf, true) & keep;
#pragma unroll
        for (int w = 0; w < WPL; w++) {
            const uint32_t Xv1 = __builtin_amdgcn_alignbit(Xv[w + 1], Xv[w], 1);
            if (w == 0) Zt = popc_acc((Xv1 | Mh[0]) & 1u, Zt);
            Pv[w] = Mh[w] | ~(Xv1 | Ph[w]);
            Mv[w] = Ph[w] & Xv1;
        }
#pragma unroll
        for (int w = 0; w < WPL; w++) asm volatile("" : "+v"(Pv[w]), "+v"(Mv[w]));
#pragma unroll
        for (int w = 0; w <= WPL; w++) cur[w] = nxt[w];
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Region of one tile: (sigma + 1) symbol rows of RS words (NW + 1 rounded up
// to a multiple of 4, so that rows start 16-byte aligned), then 8 words of
// text (the current block's 32 symbols); regions are multiples of 4 words.  Up to 4 words per lane the kernel
// is held to 80 registers, so that 6 waves share a SIMD: then a medium-sized
// join's long pairs all find a tile at once instead of some tiles running two
// of them one after the other.
template <int WPL, int SIGMAX>
__global__ void __launch_bounds__(64, WPL <= 4 ? 6 : 1)
    k_verify_split(StrSet A, StrSet B, const uint64_t *__restrict__ pairs, uint32_t count,
                   const uint64_t *__restrict__ count_dev, const uint32_t *__restrict__ order,
                   uint32_t K, const uint32_t *__restrict__ Kq, uint32_t sigma, uint32_t KL,
                   uint32_t region, uint32_t *__restrict__ next, int32_t *__restrict__ dist,
                   unsigned long long *__restrict__ columns) {
    extern __shared__ uint32_t lds[];
    unsigned long long colsum = 0;  // text columns of the pairs decided here
    if (count_dev) count = (uint32_t)min<uint64_t>(*count_dev, count);
    constexpr int TQ = 4;  // text dwords per lane, at most (8 / KL, KL >= 2)
    const uint32_t lane = threadIdx.x;
    const uint32_t tile = lane / KL, l = lane - tile * KL;
    const uint32_t head = tile * KL;  // lane 0 of the tile
    const uint32_t NW = WPL * KL;     // band words of a pair
    const uint32_t RS = (NW + 4) & ~3u;  // words per symbol row of a window
    const uint32_t nq = KL >= 8 ? 1u : 8u / KL;  // text dwords of this lane
    const uint32_t q0 = l * nq;                  // (none when q0 >= 8)
    uint32_t *win = lds + tile * region;
    uint32_t *txtw = win + (sigma + 1) * RS;
    const uint8_t *txt = (const uint8_t *)txtw;
    uint64_t last = 0;
    for (uint32_t q = 0; q < 64; q++)
        if (q % KL == KL - 1) last |= 1ull << q;
    const uint64_t notlast = ~last;
    const uint32_t keep = l == KL - 1 ? 0u : 0xFFFFFFFFu;
    for (uint32_t w = l; w < RS; w += KL) win[sigma * RS + w] = 0xFFFFFFFFu;

    PairView v = view_pair(A, B, pairs, Kq, K, 0, false);
    uint32_t pidx = 0, jb = 0, Zt = 0, kstar = 0;
    uint32_t Pv[WPL], Mv[WPL], tp[TQ];
#pragma unroll
    for (int w = 0; w < WPL; w++) Pv[w] = Mv[w] = 0;
    bool has = false, drained = false;  // per tile, equal in its lanes

    for (;;) {
        // ---- tiles without a pair take the next ones (lane 0 of the tile
        //      asks, the tile learns the index by shuffle)
        bool fresh = false;
        for (;;) {
            const bool need = !has && !drained;
            const uint64_t nm = __builtin_amdgcn_ballot_w64(need && l == 0);
            if (nm == 0) break;
            const uint32_t leader = (uint32_t)__builtin_ctzll(nm);
            uint32_t got = 0;
            if (lane == leader) got = atomicAdd(next, (uint32_t)__popcll(nm));
            got = readlane_u32(got, leader);
            uint32_t k = got + (uint32_t)__popcll(nm & ((1ull << lane) - 1ull));
            k = (uint32_t)__shfl((int)k, (int)head, 64);
            if (need) {
                if (k >= count) {
                    drained = true;
                } else {
                    pidx = order ? order[k] : k;
                    v = view_pair(A, B, pairs, Kq, K, pidx, true);
                    if (v.skip || v.nn == 0) {
                        if (l == 0)
                            dist[pidx] = (int32_t)(v.skip ? v.Kp + 1 : min(v.dstar, v.Kp + 1));
                    } else {
                        has = true;
                        fresh = true;
                        jb = 0;
                        Zt = 0;
                        kstar = v.O + v.dstar;
                        // D[i][0] = |i|: bit k holds row k - O, rows <= 0 have delta -1
#pragma unroll
                        for (int w = 0; w < WPL; w++) {
                            const int d = (int)v.O - 32 * (int)(l * WPL + w);
                            const uint32_t mv =
                                d >= 31 ? 0xFFFFFFFFu : (d < 0 ? 0u : (2u << d) - 1u);
                            Mv[w] = mv;
                            Pv[w] = ~mv;
                        }
                        text_part<TQ>(v.yp, v.nn, 0, sigma, q0, nq, tp);
#pragma unroll
                        for (int i = 0; i < TQ; i++)
                            if ((uint32_t)i < nq && q0 + i < 8) txtw[q0 + i] = tp[i];
                    }
                }
            }
        }
        if (__builtin_amdgcn_ballot_w64(has) == 0) break;
        // ---- the windows of the pairs just taken, filled by the whole wave
        uint64_t fm = __builtin_amdgcn_ballot_w64(fresh && l == 0);
        while (fm) {
            const uint32_t L = (uint32_t)__builtin_ctzll(fm);
            fm &= fm - 1;
            PairView u = v;
            const uint64_t mp = (uint64_t)(uintptr_t)v.mw;
            u.mw = (const uint32_t *)(uintptr_t)(((uint64_t)readlane_u32((uint32_t)(mp >> 32), L)
                                                  << 32) |
                                                 readlane_u32((uint32_t)mp, L));
            u.W = readlane_u32(v.W, L);
            u.O = readlane_u32(v.O, L);
            uint32_t *wt = lds + (L / KL) * region;
            for (uint32_t t = lane; t < sigma * RS; t += 64) {
                const uint32_t c = t / RS, w = t - c * RS;
                wt[c * RS + w] = mask_word(u, c, w);
            }
        }
        __syncthreads();

        // ---- one block of 32 columns; this lane's part of the next block's
        //      text and the entering mask words (symbol c by lane c mod KL)
        //      are fetched first
        text_part<TQ>(v.yp, has ? v.nn : 0u, jb + 32, sigma, q0, nq, tp);
        const uint32_t wn = (jb >> 5) + NW + 1;  // band word entering the window
        uint32_t nwd[SIGMAX];
#pragma unroll
        for (uint32_t c = 0; c < (uint32_t)SIGMAX; c++)
            nwd[c] = (has && c < sigma && c % KL == l) ? mask_word(v, c, wn) : 0u;
        split_block<WPL>(win + l * WPL, 4 * RS, txt, Pv, Mv, Zt, notlast, keep);
        // shift the window down one word: every lane moves its own words,
        // reading all before any lane writes; then the next block's text
        uint32_t mv[SIGMAX][WPL];
#pragma unroll
        for (uint32_t c = 0; c < (uint32_t)SIGMAX; c++)
#pragma unroll
            for (uint32_t w = 0; w < (uint32_t)WPL; w++)
                mv[c][w] = c < sigma ? win[c * RS + l * WPL + w + 1] : 0u;
        __syncthreads();
#pragma unroll
        for (uint32_t c = 0; c < (uint32_t)SIGMAX; c++) {
            if (c < sigma) {
#pragma unroll
                for (uint32_t w = 0; w < (uint32_t)WPL; w++) win[c * RS + l * WPL + w] = mv[c][w];
                if (c % KL == l) win[c * RS + NW] = nwd[c];
            }
        }
#pragma unroll
        for (int i = 0; i < TQ; i++)
            if ((uint32_t)i < nq && q0 + i < 8) txtw[q0 + i] = tp[i];
        __syncthreads();
        jb += 32;

        // ---- decisions: the value on d* is the top value (lane 0 of the
        //      tile) plus the vertical deltas of bits 1..k* (all lanes)
        int32_t D = 0;
#pragma unroll
        for (int w = 0; w < WPL; w++) {
            const int d = (int)kstar - 32 * (int)(l * WPL + w);
            uint32_t mk = d >= 31 ? 0xFFFFFFFFu : (d < 0 ? 0u : (2u << d) - 1u);
            if (w == 0 && l == 0) mk &= ~1u;
            D += __builtin_popcount(Pv[w] & mk) - __builtin_popcount(Mv[w] & mk);
        }
        for (uint32_t o = 1; o < KL; o <<= 1) D += __shfl_xor(D, (int)o, 64);
        const uint32_t Z0 = (uint32_t)__shfl((int)Zt, (int)head, 64);
        if (has) {
            const uint32_t Vd = (uint32_t)((int32_t)(v.O + jb - Z0) + D);
            if (Vd > v.Kp || jb >= v.nn) {
                if (l == 0) {
                    dist[pidx] = (int32_t)min(Vd, v.Kp + 1);
                    colsum += (unsigned long long)min(jb, v.nn);
                }
                has = false;
            }
        }
    }
    add_columns(columns, colsum);
}

// Mask words of every string: sigma * ceil(len / 32).
__global__ void k_mask_sizes(const uint64_t *__restrict__ off, uint32_t n, uint32_t sigma,
                             uint64_t *__restrict__ sz) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        const uint64_t len = off[s + 1] - off[s];
        sz[s] = (uint64_t)sigma * ((len + 31) / 32);
    }
}

// Match masks, one wave per string, lane w building word w of every symbol:
// the 32 codes of the word are compared with the symbol four at a time (a
// byte is zero after the xor iff it matches).
__global__ void k_build_masks(const uint8_t *__restrict__ codes, const uint64_t *__restrict__ off,
                              uint64_t base, uint32_t n, uint32_t sigma,
                              const uint64_t *__restrict__ moff, uint32_t *__restrict__ words) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t s = wave; s < n; s += nwaves) {
        const uint64_t o = off[s] - base;
        const uint32_t len = (uint32_t)(off[s + 1] - off[s]);
        const uint32_t W = (len + 31) / 32;
        uint32_t *dst = words + moff[s];
        for (uint32_t w = lane; w < W; w += 64) {
            // codes x[32w .. 32w+31]: reads stay within the array's 64-byte padding
            const uintptr_t a = (uintptr_t)(codes + o + 32ull * w);
            const uint32_t *b4 = (const uint32_t *)(a & ~(uintptr_t)3);
            const uint32_t sh = (uint32_t)(a & 3) * 8;
            uint32_t d[9], t[8];
#pragma unroll
            for (int q = 0; q < 9; q++) d[q] = b4[q];
#pragma unroll
            for (int q = 0; q < 8; q++) t[q] = __builtin_amdgcn_alignbit(d[q + 1], d[q], sh);
            const uint32_t valid = len - 32 * w;
            const uint32_t vmask = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
            for (uint32_t c = 0; c < sigma; c++) {
                const uint32_t rep = c * 0x01010101u;
                uint32_t word = 0;
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const uint32_t x = t[q] ^ rep;
                    // bit 7 of a byte of z is set iff that byte of x is zero
                    const uint32_t z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
                    const uint32_t nib = ((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) |
                                         ((z >> 28) & 8u);
                    word |= nib << (4 * q);
                }
                dst[(uint64_t)c * W + w] = word & vmask;
            }
        }
    }
}

// Match masks for alphabets up to MASK_LDS_SIGMA symbols, one thread per
// mask word: thread i builds word w of string s (its words are numbered
// from moff[s] / sigma, found by bisection; an empty string shares its
// offset with the next one, and the last string at or below the word's
// offset owns it) for every symbol at once.  Each of the word's 32 codes
// sets its bit in a lane-private LDS word of its symbol; the sigma words
// are then written out (consecutive threads: consecutive words of a row).
// moff[n] holds the total.
constexpr uint32_t MASK_LDS_SIGMA = 64;

__global__ void __launch_bounds__(64)
    k_build_masks_lds(const uint8_t *__restrict__ codes, const uint64_t *__restrict__ off,
                      uint64_t base, uint32_t n, uint32_t sigma,
                      const uint64_t *__restrict__ moff, uint32_t *__restrict__ words) {
    extern __shared__ uint32_t acc[];  // [sigma][64]
    const uint32_t lane = threadIdx.x;
    const uint64_t tw = moff[n] / sigma;
    for (uint64_t i = (uint64_t)blockIdx.x * 64 + lane; i < tw; i += (uint64_t)gridDim.x * 64) {
        const uint64_t at = i * sigma;
        uint32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo + 1) / 2;
            if (moff[mid] <= at)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint32_t s = lo;
        const uint64_t o = off[s] - base;
        const uint32_t len = (uint32_t)(off[s + 1] - off[s]);
        const uint32_t W = (len + 31) / 32;
        const uint32_t w = (uint32_t)(i - moff[s] / sigma);
        for (uint32_t c = 0; c < sigma; c++) acc[c * 64 + lane] = 0u;
        // codes x[32w .. 32w+31]: reads stay within the array's 64-byte padding
        const uintptr_t a = (uintptr_t)(codes + o + 32ull * w);
        const uint32_t *b4 = (const uint32_t *)(a & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(a & 3) * 8;
        uint32_t d[9], t[8];
#pragma unroll
        for (int q = 0; q < 9; q++) d[q] = b4[q];
#pragma unroll
        for (int q = 0; q < 8; q++) t[q] = __builtin_amdgcn_alignbit(d[q + 1], d[q], sh);
        const uint32_t valid = min(len - 32 * w, 32u);
#pragma unroll
        for (uint32_t q = 0; q < 32; q++) {
            const uint32_t c = (t[q >> 2] >> (8 * (q & 3))) & 0xFFu;
            if (q < valid) atomicOr(&acc[c * 64 + lane], 1u << q);
        }
        uint32_t *dst = words + moff[s];
        for (uint32_t c = 0; c < sigma; c++) dst[(uint64_t)c * W + w] = acc[c * 64 + lane];
    }
}

__global__ void k_zero_u32(uint32_t *__restrict__ p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

__global__ void k_max_u32(const uint32_t *__restrict__ a, uint64_t n, uint32_t *__restrict__ out) {
    uint32_t mx = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        mx = max(mx, a[i]);
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, mx);
}

// flags[k] = 1 for the pairs pass 1 left undecided
__global__ void k_alive_flags(const uint32_t *__restrict__ aux, uint64_t count,
                              const uint64_t *__restrict__ count_dev,
                              uint32_t *__restrict__ flags) {
    // pairs past a count on the device were never verified: not alive
    const uint64_t live = count_dev ? min(*count_dev, count) : count;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < count;
         e += (uint64_t)gridDim.x * blockDim.x)
        flags[e] = (e < live && aux[e] != DECIDED) ? 1u : 0u;
}

__global__ void k_alive_list(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos,
                             uint64_t count, uint32_t *__restrict__ list) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < count;
         e += (uint64_t)gridDim.x * blockDim.x)
        if (flags[e]) list[pos[e]] = (uint32_t)e;
}

// Lane form limits: bands of up to 16 words (K <= 510) in registers, and
// alphabets of up to 4 symbols (the windows of 64 lanes stay within LDS at a
// few waves per CU).  With one lane per pair and bands of up to 8 words
// (K <= 254), alphabets of up to 32 symbols: a lane's window of 33 rows of at
// most 9 words, 76 KB per wave at the most (33 KB at K = 100 over 25 letters).
constexpr uint32_t LANE_MAX_WORDS = 16;
constexpr uint32_t LANE_MAX_SIGMA = 4;
constexpr uint32_t LANE_WIDE_WORDS = 8;
constexpr uint32_t LANE_WIDE_SIGMA = 32;

using LaneKernel = void (*)(StrSet, StrSet, const uint64_t *, uint32_t, const uint64_t *,
                            const uint32_t *, uint32_t, const uint32_t *, uint32_t, uint32_t,
                            uint32_t *, int32_t *, unsigned long long *);

LaneKernel lane_kernel(uint32_t nw) {
    switch (nw) {
        case 1: return k_verify_lane<1, LANE_MAX_SIGMA>;
        case 2: return k_verify_lane<2, LANE_MAX_SIGMA>;
        case 3: return k_verify_lane<3, LANE_MAX_SIGMA>;
        case 4: return k_verify_lane<4, LANE_MAX_SIGMA>;
        case 5: return k_verify_lane<5, LANE_MAX_SIGMA>;
        case 6: return k_verify_lane<6, LANE_MAX_SIGMA>;
        case 7: return k_verify_lane<7, LANE_MAX_SIGMA>;
        case 8: return k_verify_lane<8, LANE_MAX_SIGMA>;
        case 9: return k_verify_lane<9, LANE_MAX_SIGMA>;
        case 10: return k_verify_lane<10, LANE_MAX_SIGMA>;
        case 11: return k_verify_lane<11, LANE_MAX_SIGMA>;
        case 12: return k_verify_lane<12, LANE_MAX_SIGMA>;
        case 13: return k_verify_lane<13, LANE_MAX_SIGMA>;
        case 14: return k_verify_lane<14, LANE_MAX_SIGMA>;
        case 15: return k_verify_lane<15, LANE_MAX_SIGMA>;
        case 16: return k_verify_lane<16, LANE_MAX_SIGMA>;
        default: return nullptr;
    }
}

using SplitKernel = void (*)(StrSet, StrSet, const uint64_t *, uint32_t, const uint64_t *,
                             const uint32_t *, uint32_t, const uint32_t *, uint32_t, uint32_t,
                             uint32_t, uint32_t *, int32_t *, unsigned long long *);
constexpr uint32_t SPLIT_MAX_WPL = 8;

LaneKernel lane_kernel_wide(uint32_t nw) {
    switch (nw) {
        case 1: return k_verify_lane<1, LANE_WIDE_SIGMA>;
        case 2: return k_verify_lane<2, LANE_WIDE_SIGMA>;
        case 3: return k_verify_lane<3, LANE_WIDE_SIGMA>;
        case 4: return k_verify_lane<4, LANE_WIDE_SIGMA>;
        case 5: return k_verify_lane<5, LANE_WIDE_SIGMA>;
        case 6: return k_verify_lane<6, LANE_WIDE_SIGMA>;
        case 7: return k_verify_lane<7, LANE_WIDE_SIGMA>;
        case 8: return k_verify_lane<8, LANE_WIDE_SIGMA>;
        default: return nullptr;
    }
}

SplitKernel split_kernel(uint32_t wpl) {
    switch (wpl) {
        case 1: return k_verify_split<1, LANE_MAX_SIGMA>;
        case 2: return k_verify_split<2, LANE_MAX_SIGMA>;
        case 3: return k_verify_split<3, LANE_MAX_SIGMA>;
        case 4: return k_verify_split<4, LANE_MAX_SIGMA>;
        case 5: return k_verify_split<5, LANE_MAX_SIGMA>;
        case 6: return k_verify_split<6, LANE_MAX_SIGMA>;
        case 7: return k_verify_split<7, LANE_MAX_SIGMA>;
        case 8: return k_verify_split<8, LANE_MAX_SIGMA>;
        default: return nullptr;
    }
}

// Words per lane window: (sigma + 1) rows of NW + 1 words, padded to an odd
// count so that the 64 lanes' windows start in distinct LDS banks.
// Words per lane of the lane form: (sigma + 1) rows of nw + 1 window words
// (the symbols and the all-ones padding row); alphabets above 4 symbols keep
// one more word per symbol after the rows (the low source word of the next
// entering mask word).  Odd, so that lanes fall on different banks.
inline uint32_t lane_region(uint32_t nw, uint32_t sigma) {
    const uint32_t r = (sigma + 1) * (nw + 1) + (sigma > 4 ? sigma : 0u);
    return r | 1u;
}

// Sort keys of the pass-2 list (11 bits, one radix pass): pairs with longer
// texts first (key 0x7FE - columns/32, texts beyond 65,472 columns share key
// 0), entries past the number of survivors last (0x7FF).  The order only
// schedules the work.
__global__ void k_alive_keys(StrSet A, StrSet B, const uint64_t *__restrict__ pairs,
                             const uint32_t *__restrict__ list, const uint64_t *__restrict__ nalive,
                             uint64_t count, uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    const uint64_t na = *nalive;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count;
         k += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t kk = 0x7FFu, v = 0;
        if (k < na) {
            v = list[k];
            const uint64_t code = pairs[v];
            const uint32_t a = (uint32_t)(code >> 32), b = (uint32_t)code;
            const uint64_t la = A.off[a + 1] - A.off[a], lb = B.off[b + 1] - B.off[b];
            const uint64_t blocks = (la < lb ? la : lb) >> 5;
            kk = 0x7FEu - (uint32_t)(blocks < 0x7FEu ? blocks : 0x7FEu);
        }
        key[k] = kk;
        val[k] = v;
    }
}

// Sort keys of the first pass: longest text first in 32-column blocks,
// clamped at cap_blocks (the columns the pass runs: texts at least that long
// all tie and keep their order, the k-th being pair order[k], or k);
// entries past a count on the device sort last.  val = the pair's index.
__global__ void k_len_keys(StrSet A, StrSet B, const uint64_t *__restrict__ pairs, uint64_t count,
                           const uint64_t *__restrict__ count_dev,
                           const uint32_t *__restrict__ order, uint32_t cap_blocks,
                           uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    const uint64_t live = count_dev ? min(*count_dev, count) : count;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count;
         k += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t kk = 0x7FFu;
        const uint32_t v = order ? order[k] : (uint32_t)k;
        if (k < live) {
            const uint64_t code = pairs[v];
            const uint32_t a = (uint32_t)(code >> 32), b = (uint32_t)code;
            const uint64_t la = A.off[a + 1] - A.off[a], lb = B.off[b + 1] - B.off[b];
            const uint64_t blocks = ((la < lb ? la : lb) + 31) >> 5;
            kk = 0x7FEu - (uint32_t)(blocks < cap_blocks ? blocks : cap_blocks);
        }
        key[k] = kk;
        val[k] = v;
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

uint32_t verify_lanes_for(uint32_t K) {
    uint64_t nl = (K + 2ull + 31) / 32;
    return nl <= 64 ? (uint32_t)nl : 0u;
}

void build_masks(ej_ctx *ctx, const uint8_t *d_codes, const uint64_t *d_offsets, uint64_t base,
                 uint32_t n, uint64_t total, uint32_t sigma, RowMasks &rm, const char *tag,
                 uint32_t *own_words, uint64_t *own_off) {
    std::string t(tag);
    uint64_t *off = own_off ? own_off : ws<uint64_t>(ctx, t + "_moff", (uint64_t)n + 1);
    uint32_t *words =
        own_words ? own_words : ws<uint32_t>(ctx, t + "_mwords", mask_words_bound(total, n, sigma));
    rm.words = words;
    rm.off = off;
    rm.n = n;
    if (n == 0) return;
    uint64_t *sz = ws<uint64_t>(ctx, t + "_msz", (uint64_t)n + 1);
    hipLaunchKernelGGL(k_mask_sizes, dim3(grid_for(ctx, n, 256)), dim3(256), 0, ctx->stream,
                       d_offsets, n, sigma, sz);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u64(ctx, sz, off, n, off + n);
    if (sigma >= 1 && sigma <= MASK_LDS_SIGMA) {
        // at most total / 32 + n words per symbol
        const uint64_t tw = total / 32 + n;
        const uint64_t grid = std::min<uint64_t>((tw + 63) / 64, (uint64_t)ctx->num_cu * 32);
        hipLaunchKernelGGL(k_build_masks_lds, dim3((uint32_t)grid), dim3(64),
                           (size_t)sigma * 64 * 4, ctx->stream, d_codes, d_offsets, base, n,
                           sigma, (const uint64_t *)off, words);
    } else {
        hipLaunchKernelGGL(k_build_masks, dim3(grid_for(ctx, (uint64_t)n * 64, 256)), dim3(256),
                           0, ctx->stream, d_codes, d_offsets, base, n, sigma,
                           (const uint64_t *)off, words);
    }
    EJ_CHECK_LAUNCH();
}

void verify(ej_ctx *ctx, const uint8_t *d_codes, const uint64_t *d_offsets, uint64_t base,
            uint32_t sigma, uint32_t maxlen, const RowMasks &masks, const uint64_t *d_pairs,
            uint64_t count, uint32_t K, const uint32_t *d_Kq, int32_t *d_dist,
            const uint8_t *d_codes_b, const uint64_t *d_offsets_b, uint64_t base_b,
            uint32_t maxlen_b, const RowMasks *masks_b, unsigned long long *d_columns,
            const uint32_t *d_order, const uint64_t *d_count, uint32_t minlen) {
    if (count == 0) return;
    if (count >= 0xFFFFFFFFull) fail(EJ_EUNSUPPORTED, "more than 2^32 pairs in one verification");
    uint32_t Kmax = K;
    if (d_Kq) {
        uint32_t *d_mx = ws<uint32_t>(ctx, "verify_kmax", 1);
        EJ_HIP(hipMemsetAsync(d_mx, 0, 4, ctx->stream));
        hipLaunchKernelGGL(k_max_u32, dim3(grid_for(ctx, count, 256)), dim3(256), 0, ctx->stream,
                           d_Kq, count, d_mx);
        EJ_CHECK_LAUNCH();
        read_back(ctx, d_mx, 4, &Kmax);
    }
    const uint32_t NL = verify_lanes_for(Kmax);
    if (NL == 0)
        fail(EJ_EUNSUPPORTED,
             "threshold " + std::to_string(Kmax) + " exceeds 2046 (band > 2048 bits)");
    const bool self_set = d_codes_b == nullptr;  // the pairs are of one string set
    if (!d_codes_b) {
        d_codes_b = d_codes;
        d_offsets_b = d_offsets;
        base_b = base;
        maxlen_b = maxlen;
        masks_b = &masks;
    }
    const StrSet A{d_codes, d_offsets, base, masks.words, masks.off};
    const StrSet B{d_codes_b, d_offsets_b, base_b, masks_b->words, masks_b->off};
    const uint32_t sig = sigma ? sigma : 1;
    const uint32_t W = 32 * NL;
    const uint32_t mtext = std::min(maxlen, maxlen_b);
    // full layout: Eq reads reach word (ncols-1)/32 + NL; pattern bits reach
    // ncols + K
    uint32_t wpp_full = (mtext + W + 64) / 32 + 2;
    wpp_full = (wpp_full + 1) & ~1u;
    // ring layout: NL+1 live words, one more being filled
    uint32_t RW = 1;
    while (RW < NL + 2) RW <<= 1;
    const uint32_t ring_mode = ctx->tune.verify_ring;
    const bool ring = ring_mode != 0 && NL >= 2 && (ring_mode == 2 || 2 * RW < wpp_full);
    const uint32_t wpp = ring ? RW : wpp_full;
    const uint32_t tile_bytes = tile_words_for(sig, ring ? 2 * RW : wpp_full) * 4;
    uint32_t tpw = 64 / NL;
    uint32_t budget = ctx->tune.verify_lds_budget;
    if ((int)budget > ctx->lds_max) budget = (uint32_t)ctx->lds_max;
    if (tile_bytes > budget) budget = (uint32_t)ctx->lds_max;
    if (tile_bytes > budget)
        fail(EJ_EUNSUPPORTED, "strings too long for the LDS-resident match masks (" +
                                  std::to_string(tile_bytes) + " bytes per pair)");
    tpw = std::min(tpw, budget / tile_bytes);
    const size_t lds = (size_t)tpw * tile_bytes;
    const int mode = NL == 1 ? LANES_ONE : NL == 16 ? LANES_ROW : NL == 64 ? LANES_WAVE : LANES_ANY;
    Timers &tk = ctx->timers;
    auto kmark = [&]() {
        if (tk.on && tk.nkv < 4) EJ_HIP(hipEventRecord(tk.kv[tk.nkv++], ctx->stream));
    };
    // grouped by pattern: the candidates' patterns share LDS rows per chunk
    if (ctx->tune.verify_mode == 3 && self_set && NL <= LANE_MAX_WORDS && masks.n > 0) {
        const uint32_t lead = (Kmax / 2 + 1 + 31) / 32;
        const uint32_t Wfull = (maxlen + 31) / 32;
        const uint32_t S = lead + Wfull + NL + 2;
        const size_t glds = (size_t)(sig + 1) * S * 4;
        if (glds <= (size_t)ctx->lds_max) {
            ctx->last_verify_form = 4;
            const uint32_t n = masks.n;
            uint32_t *gkey = ws<uint32_t>(ctx, "vg_key", count);
            uint32_t *gval = ws<uint32_t>(ctx, "vg_val", count);
            uint32_t *gkey2 = ws<uint32_t>(ctx, "vg_key2", count);
            uint32_t *gorder = ws<uint32_t>(ctx, "vg_order", count);
            uint32_t *cflag = ws<uint32_t>(ctx, "vg_cflag", count);
            uint32_t *cpos = ws<uint32_t>(ctx, "vg_cpos", count);
            uint32_t *cstart = ws<uint32_t>(ctx, "vg_cstart", count + 1);
            uint64_t *d_nch = ws<uint64_t>(ctx, "vg_nchunks", 1);
            uint64_t *crange = ws<uint64_t>(ctx, "vg_crange", 3);
            uint32_t *next = ws<uint32_t>(ctx, "vg_next", 2);
            const GrpKernel gk = grp_kernel(NL);
            const uint32_t want = std::max(1u, ctx->tune.verify_blocks_per_cu);
            // waves per CU for `lds` bytes per wave (at most `want`)
            auto resident = [&](size_t lds) {
                if (lds > 65536)
                    EJ_HIP(hipFuncSetAttribute((const void *)gk,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds));
                int occ = 0;
                EJ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gk, 64, lds));
                return std::max(1u, std::min((uint32_t)std::max(occ, 1), want));
            };
            // rows sized for the whole set hold fewer waves per CU than asked
            // for: patterns up to `lim` letters then take rows of Ws words
            // (as many as `want` waves per CU leave room for), the longer
            // ones the full rows, in a second launch
            const uint32_t per_cu = resident(glds);
            int lds_cu = 0;
            EJ_HIP(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                         ctx->device));
            const uint64_t row_bytes = (uint64_t)(sig + 1) * 4;
            const uint64_t fit = (uint64_t)std::max(lds_cu, 0) / want / row_bytes;
            const uint32_t Ws =
                fit > lead + NL + 2 ? (uint32_t)std::min<uint64_t>(fit - lead - NL - 2, Wfull)
                                    : 0u;
            // pattern indexes are below n: PB bits hold them and the padding
            // key's all-ones field
            const uint32_t PB = std::max(1u, bits_for(n));
            const bool split = per_cu < want && Ws >= 1 && Ws < Wfull && PB < 32;
            uint32_t *rstart = ws<uint32_t>(ctx, "vg_rstart", split ? 2ull * n : n);
            const uint32_t Ss = split ? lead + Ws + NL + 2 : S;
            const size_t glds_s = (size_t)(sig + 1) * Ss * 4;
            const uint32_t per_cu_s = split ? resident(glds_s) : per_cu;
            const uint64_t lim = split ? 32ull * Ws : ~0ull;
            const uint64_t grid_s =
                std::min<uint64_t>((count + 63) / 64, (uint64_t)ctx->num_cu * per_cu_s);
            const uint64_t grid_l =
                std::min<uint64_t>((count + 63) / 64, (uint64_t)ctx->num_cu * per_cu);
            // pairs ordered by (length class, pattern), cut into chunks (no
            // host round trip)
            const uint32_t KB = split ? PB : 32u;  // the class bit (32: none)
            hipLaunchKernelGGL(k_grp_keys, dim3(grid_for(ctx, count, 256)), dim3(256), 0,
                               ctx->stream, A.off, d_pairs, count, d_count, split ? PB : 0u, lim,
                               gkey, gval);
            EJ_CHECK_LAUNCH();
            radix_sort_u32(ctx, gkey, gval, gkey2, gorder, 1, (uint32_t)count,
                           split ? PB + 1 : PB, ctx->tune.radix_bits);
            hipLaunchKernelGGL(k_grp_run_starts, dim3(grid_for(ctx, count, 256)), dim3(256), 0,
                               ctx->stream, (const uint32_t *)gkey2, count, d_count, KB, n,
                               rstart);
            EJ_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_grp_chunk_flags, dim3(grid_for(ctx, count, 256)), dim3(256), 0,
                               ctx->stream, (const uint32_t *)gkey2, count, d_count, KB, n,
                               (const uint32_t *)rstart, cflag);
            EJ_CHECK_LAUNCH();
            scan_exclusive_u32(ctx, cflag, cpos, count, d_nch);
            hipLaunchKernelGGL(k_grp_chunk_starts, dim3(grid_for(ctx, count, 256)), dim3(256),
                               0, ctx->stream, (const uint32_t *)cflag, (const uint32_t *)cpos,
                               count, d_count, (const uint64_t *)d_nch, cstart);
            EJ_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_grp_split, dim3(1), dim3(64), 0, ctx->stream,
                               (const uint32_t *)gkey2, (const uint32_t *)cstart,
                               (const uint64_t *)d_nch, KB, crange);
            EJ_CHECK_LAUNCH();
            char key[448];
            snprintf(key, sizeof(key),
                     "verify_grp %u %p %p %llu %p %p %p %p %p %p %u %p %u %u %u %u %p %p %p "
                     "%llu %llu %zu %zu %d %llu",
                     NL, (const void *)d_codes, (const void *)d_offsets, (unsigned long long)base,
                     (const void *)A.mw, (const void *)A.moff, (const void *)d_pairs,
                     (const void *)gorder, (const void *)cstart, (const void *)crange, K,
                     (const void *)d_Kq, sig, S, Ss, lead, (void *)next, (void *)d_dist,
                     (void *)d_columns, (unsigned long long)grid_s, (unsigned long long)grid_l,
                     glds, glds_s, (int)split, (unsigned long long)ctx->ws_gen);
            if (split && tk.on) tk.more++;  // two launches between the events
            kmark();
            run_captured(ctx, key, [&] {
                hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, ctx->stream, next);
                EJ_CHECK_LAUNCH();
                hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, ctx->stream, next + 1);
                EJ_CHECK_LAUNCH();
                // short patterns: chunks [crange[0], crange[1]); without the
                // split every chunk is there (no key has the class bit)
                hipLaunchKernelGGL(gk, dim3((uint32_t)(split ? grid_s : grid_l)), dim3(64),
                                   split ? glds_s : glds, ctx->stream, A, d_pairs,
                                   (const uint32_t *)gorder, (const uint32_t *)cstart,
                                   (const uint64_t *)crange, K, d_Kq, sig, split ? Ss : S, lead,
                                   next, d_dist, d_columns);
                EJ_CHECK_LAUNCH();
                if (split) {
                    // long patterns: chunks [crange[1], crange[2])
                    hipLaunchKernelGGL(gk, dim3((uint32_t)grid_l), dim3(64), glds, ctx->stream,
                                       A, d_pairs, (const uint32_t *)gorder,
                                       (const uint32_t *)cstart, (const uint64_t *)(crange + 1),
                                       K, d_Kq, sig, S, lead, next + 1, d_dist, d_columns);
                    EJ_CHECK_LAUNCH();
                }
            });
            kmark();
            return;
        }
    }
    // the lane family: KL lanes per pair (1: the whole band in one lane)
    uint32_t KL = ctx->tune.verify_split;
    // (the split lanes take alphabets of up to 4 symbols; larger ones use one
    // lane per pair up to 8 band words)
    if (KL == 0)
        KL = (NL <= 4 || (sig > LANE_MAX_SIGMA && NL <= LANE_WIDE_WORDS)) ? 1u : NL <= 8 ? 2u : 4u;
    while (KL > 1 && KL / 2 >= NL) KL /= 2;  // no lane without a word of the band
    const uint32_t WPL = (NL + KL - 1) / KL;
    const uint32_t NWf = KL * WPL;
    const bool lane_ok = KL == 1 ? NL <= LANE_MAX_WORDS : WPL <= SPLIT_MAX_WPL;
    // alphabets above 4 symbols: one lane per pair with up to 8 band words
    const bool wide = sig > LANE_MAX_SIGMA && KL == 1 && NWf <= LANE_WIDE_WORDS &&
                      sig <= LANE_WIDE_SIGMA;
    if (ctx->tune.verify_mode == 2 && lane_ok && (sig <= LANE_MAX_SIGMA || wide) &&
        (int)((64 / KL) * ((sig + 1) * (NWf + 4) + 12) * 4) <= ctx->lds_max) {
        // lane form: KL lanes per pair, a device-wide pair counter
        ctx->last_verify_form = KL == 1 ? 2 : 3;
        const LaneKernel lk = wide ? lane_kernel_wide(NWf) : lane_kernel(NWf);
        const void *kf = KL == 1 ? (const void *)lk : (const void *)split_kernel(WPL);
        // split tiles: rows of NW+1 words rounded up to a multiple of 4, then
        // the text block (8 words)
        const uint32_t region =
            KL == 1 ? lane_region(NWf, sig) : ((sig + 1) * ((NWf + 4) & ~3u) + 8 + 3) & ~3u;
        const size_t llds = (size_t)(64 / KL) * region * 4;
        if (llds > 65536)
            EJ_HIP(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)llds));
        int occ = 0;
        EJ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kf, 64, llds));
        if (occ < 1) occ = 1;
        const uint32_t per_cu = std::max(1u, std::min((uint32_t)occ, ctx->tune.verify_blocks_per_cu));
        const uint64_t grid =
            std::min<uint64_t>((count * KL + 63) / 64, (uint64_t)ctx->num_cu * per_cu);
        uint32_t *next = ws<uint32_t>(ctx, "verify_next", 1);
        char key[512];
        snprintf(key, sizeof(key),
                 "verify_lane %u %u %p %p %llu %p %p %p %p %llu %p %p %p %u %p %p %u %p %u %u %p "
                 "%p %p %llu %zu %llu",
                 NWf, KL, (const void *)d_codes, (const void *)d_offsets, (unsigned long long)base,
                 (const void *)A.mw, (const void *)A.moff, (const void *)d_codes_b,
                 (const void *)d_offsets_b, (unsigned long long)base_b, (const void *)B.mw,
                 (const void *)B.moff, (const void *)d_pairs, (unsigned)count,
                 (const void *)d_count, (const void *)d_order, K, (const void *)d_Kq, sig, region,
                 (void *)next,
                 (void *)d_dist, (void *)d_columns, (unsigned long long)grid, llds,
                 (unsigned long long)ctx->ws_gen);
        kmark();
        run_captured(ctx, key, [&] {
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, ctx->stream, next);
            EJ_CHECK_LAUNCH();
            if (KL == 1)
                hipLaunchKernelGGL(lk, dim3((uint32_t)grid), dim3(64), llds,
                                   ctx->stream, A, B, d_pairs, (uint32_t)count, d_count, d_order,
                                   K, d_Kq, sig, region, next, d_dist, d_columns);
            else
                hipLaunchKernelGGL(split_kernel(WPL), dim3((uint32_t)grid), dim3(64), llds,
                                   ctx->stream, A, B, d_pairs, (uint32_t)count, d_count, d_order,
                                   K, d_Kq, sig, KL, region, next, d_dist, d_columns);
            EJ_CHECK_LAUNCH();
        });
        kmark();
        return;
    }
    if (ctx->tune.verify_mode >= 1) {
        // persistent form: one resident grid, a device-wide pair counter
        ctx->last_verify_form = 1;
        auto qkern = mode == LANES_ONE    ? k_verify_queue<LANES_ONE, false>
                     : mode == LANES_ROW  ? (ring ? k_verify_queue<LANES_ROW, true>
                                                  : k_verify_queue<LANES_ROW, false>)
                     : mode == LANES_WAVE ? (ring ? k_verify_queue<LANES_WAVE, true>
                                                  : k_verify_queue<LANES_WAVE, false>)
                     : (ring ? k_verify_queue<LANES_ANY, true> : k_verify_queue<LANES_ANY, false>);
        if (lds > 65536)
            EJ_HIP(hipFuncSetAttribute((const void *)qkern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        int occ = 0;
        EJ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, qkern, 64, lds));
        if (occ < 1) occ = 1;
        const uint64_t ngroups = (count + tpw - 1) / tpw;
        const uint64_t grid = std::min<uint64_t>(ngroups, (uint64_t)ctx->num_cu * occ);
        uint32_t *next = ws<uint32_t>(ctx, "verify_next", 1);
        // the counter reset and the persistent launch: one captured graph in
        // graph mode (keyed by every launch argument and the workspace
        // generation, so that no buffer of a cached graph has moved)
        char key[512];
        snprintf(key, sizeof(key),
                 "verify_queue %d %d %p %p %llu %p %p %p %p %llu %p %p %p %u %p %p %u %p %u %u %u "
                 "%u %p %p %p %llu %zu %llu",
                 mode, (int)ring, (const void *)d_codes, (const void *)d_offsets,
                 (unsigned long long)base, (const void *)A.mw, (const void *)A.moff,
                 (const void *)d_codes_b, (const void *)d_offsets_b, (unsigned long long)base_b,
                 (const void *)B.mw, (const void *)B.moff, (const void *)d_pairs, (unsigned)count,
                 (const void *)d_count, (const void *)d_order, K, (const void *)d_Kq, sig, NL, tpw,
                 wpp, (void *)next,
                 (void *)d_dist, (void *)d_columns, (unsigned long long)grid, lds,
                 (unsigned long long)ctx->ws_gen);
        kmark();
        run_captured(ctx, key, [&] {
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, ctx->stream, next);
            EJ_CHECK_LAUNCH();
            hipLaunchKernelGGL(qkern, dim3((uint32_t)grid), dim3(64), lds, ctx->stream, A, B,
                               d_pairs, (uint32_t)count, d_count, d_order, K, d_Kq, sig, NL, tpw,
                               wpp, next, d_dist, d_columns);
            EJ_CHECK_LAUNCH();
        });
        kmark();
        return;
    }
    ctx->last_verify_form = 0;
    const uint32_t C1 = ctx->tune.verify_pass1_cols & ~31u;
    const bool two_pass = C1 > 0 && C1 < mtext;
    // WPL band words per lane (knob verify_wpl: 1, 2 or 4, lowered until the
    // band has at least 2 WPL words): fewer lanes per pair, so the lookahead
    // between lanes, the shift's word from the next lane and the symbol's
    // address are paid once per 32 WPL bits.  The ring holds exactly the
    // NW + 1 words a block reads (RW = NW + 1), its first WPL slots repeated
    // after the last.
    uint32_t Wv = ctx->tune.verify_wpl >= 4 ? 4u : ctx->tune.verify_wpl >= 2 ? 2u : 1u;
    while (Wv > 1 && NL < 2 * Wv) Wv /= 2;
    const uint32_t vNL = (NL + Wv - 1) / Wv, NWv = vNL * Wv;
    uint32_t wppf = (mtext + 32 * NWv + 64) / 32 + 2;
    wppf = (wppf + 1) & ~1u;
    const uint32_t RWv = NWv + 1;
    const bool vring = ring_mode != 0 && vNL >= 2 && (ring_mode == 2 || RWv + Wv < wppf);
    const uint32_t vwpp = vring ? RWv : wppf;
    const uint32_t tb = tile_words_for(sig, vring ? RWv + Wv : wppf) * 4;
    uint32_t vbudget = ctx->tune.verify_lds_budget;
    if ((int)vbudget > ctx->lds_max) vbudget = (uint32_t)ctx->lds_max;
    if (tb > vbudget) vbudget = (uint32_t)ctx->lds_max;
    if (tb > vbudget)
        fail(EJ_EUNSUPPORTED, "strings too long for the LDS-resident match masks (" +
                                  std::to_string(tb) + " bytes per pair)");
    const uint32_t vtpw = std::min(64u / vNL, vbudget / tb);
    const size_t vlds = (size_t)vtpw * tb;
    const int vmode =
        vNL == 1 ? LANES_ONE : vNL == 16 ? LANES_ROW : vNL == 64 ? LANES_WAVE : LANES_ANY;
    using VKern = decltype(&k_verify<LANES_ANY, true, 1>);
    VKern vkern;
    if (Wv == 1)
        vkern = vmode == LANES_ONE    ? k_verify<LANES_ONE, false, 1>
                : vmode == LANES_ROW  ? (vring ? k_verify<LANES_ROW, true, 1>
                                               : k_verify<LANES_ROW, false, 1>)
                : vmode == LANES_WAVE ? (vring ? k_verify<LANES_WAVE, true, 1>
                                               : k_verify<LANES_WAVE, false, 1>)
                                      : (vring ? k_verify<LANES_ANY, true, 1>
                                               : k_verify<LANES_ANY, false, 1>);
    else if (Wv == 2)
        vkern = vmode == LANES_ROW ? (vring ? k_verify<LANES_ROW, true, 2>
                                            : k_verify<LANES_ROW, false, 2>)
                                   : (vring ? k_verify<LANES_ANY, true, 2>
                                            : k_verify<LANES_ANY, false, 2>);
    else
        vkern = vmode == LANES_ROW ? (vring ? k_verify<LANES_ROW, true, 4>
                                            : k_verify<LANES_ROW, false, 4>)
                                   : (vring ? k_verify<LANES_ANY, true, 4>
                                            : k_verify<LANES_ANY, false, 4>);
    if (vlds > 65536)
        EJ_HIP(hipFuncSetAttribute((const void *)vkern,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)vlds));
    if (Wv > 1) ctx->last_verify_form = 5;
    uint32_t *state = nullptr, *aux = nullptr;
    if (two_pass) {
        // Pv and Mv of every band word of every pair
        state = ws<uint32_t>(ctx, "verify_state", count * vNL * 2 * Wv);
        aux = ws<uint32_t>(ctx, "verify_aux", count);
    }
    const uint64_t cap = (uint64_t)ctx->num_cu * ctx->tune.verify_blocks_per_cu;
    // sort buffers of the passes' orders, taken when a sort runs
    uint32_t *lkey = nullptr, *lkey2 = nullptr, *lval = nullptr, *list = nullptr;
    auto sort_buffers = [&] {
        if (list) return;
        lkey = ws<uint32_t>(ctx, "verify_lkey", count);
        lkey2 = ws<uint32_t>(ctx, "verify_lkey2", count);
        lval = ws<uint32_t>(ctx, "verify_lval", count);
        list = ws<uint32_t>(ctx, "verify_list", count);
    };
    // the first pass in order of text length, longest first and clamped at
    // the columns it runs, so that a wave's pairs end about together (a wave
    // runs until its last pair is decided); skipped when every text outlasts
    // it (minlen: a lower bound on the texts, 0 if unknown).  Within a
    // length, and when there is no length sort, in d_order (most frequent
    // pairs first: pairs likely within K, which run to their end, share waves)
    const uint32_t run1 = two_pass ? C1 : 32u * 0x7FEu;
    const uint32_t *list1 = d_order;
    if (ctx->tune.verify_len_order && minlen < std::min(run1, mtext)) {
        sort_buffers();
        hipLaunchKernelGGL(k_len_keys, dim3(grid_for(ctx, count, 256)), dim3(256), 0,
                           ctx->stream, A, B, d_pairs, count, d_count, d_order, run1 >> 5, lkey,
                           lval);
        EJ_CHECK_LAUNCH();
        radix_sort_u32(ctx, lkey, lval, lkey2, list, 1, (uint32_t)count, 11, 11);
        list1 = list;
    }
    {
        kmark();
        uint64_t ngroups = (count + vtpw - 1) / vtpw;
        uint64_t grid = std::min<uint64_t>(ngroups, cap);
        hipLaunchKernelGGL(vkern, dim3((uint32_t)grid), dim3(64), vlds, ctx->stream, A, B, d_pairs,
                           count, d_count, list1, K, d_Kq,
                           sig, vNL, vtpw, vwpp, 0u,
                           two_pass ? C1 : NO_LIMIT, 0, state, aux, d_dist, d_columns);
        EJ_CHECK_LAUNCH();
        kmark();
    }
    if (!two_pass) return;
    sort_buffers();
    uint32_t *flags = ws<uint32_t>(ctx, "verify_flags", count);
    uint32_t *pos = ws<uint32_t>(ctx, "verify_pos", count);
    uint64_t *d_nalive = ws<uint64_t>(ctx, "verify_nalive", 1);
    hipLaunchKernelGGL(k_alive_flags, dim3(grid_for(ctx, count, 256)), dim3(256), 0, ctx->stream,
                       (const uint32_t *)aux, count, d_count, flags);
    EJ_CHECK_LAUNCH();
    scan_exclusive_u32(ctx, flags, pos, count, d_nalive);
    // no host round trip: the list and pass 2 are sized for all pairs and
    // pass 2 reads the number of undecided pairs from the device
    uint32_t *list0 = ws<uint32_t>(ctx, "verify_list0", count);
    hipLaunchKernelGGL(k_alive_list, dim3(grid_for(ctx, count, 256)), dim3(256), 0, ctx->stream,
                       (const uint32_t *)flags, (const uint32_t *)pos, count, list0);
    EJ_CHECK_LAUNCH();
    // longest texts first, so that each wave's pairs run about as long as
    // one another and the longest start early (the first pass's list is no
    // longer read: pass 1 has finished on this stream)
    hipLaunchKernelGGL(k_alive_keys, dim3(grid_for(ctx, count, 256)), dim3(256), 0, ctx->stream,
                       A, B, d_pairs, (const uint32_t *)list0, (const uint64_t *)d_nalive, count,
                       lkey, lval);
    EJ_CHECK_LAUNCH();
    radix_sort_u32(ctx, lkey, lval, lkey2, list, 1, (uint32_t)count, 11, 11);
    uint64_t ngroups = (count + vtpw - 1) / vtpw;
    uint64_t grid = std::min<uint64_t>(ngroups, cap);
    kmark();
    hipLaunchKernelGGL(vkern, dim3((uint32_t)grid), dim3(64), vlds, ctx->stream, A, B, d_pairs,
                       count, (const uint64_t *)d_nalive, (const uint32_t *)list, K, d_Kq, sig,
                       vNL, vtpw, vwpp, C1, NO_LIMIT, 1,
                       state, aux, d_dist, d_columns);
    EJ_CHECK_LAUNCH();
    kmark();
}

}  // namespace ej
