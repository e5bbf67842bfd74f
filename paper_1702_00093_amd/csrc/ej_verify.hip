// Stage A5: threshold edit distance of candidate pairs (Section 3.3).
//
// Ukkonen's observation is that only the 2K+1 diagonals |i - j| <= K of the
// dynamic-programming table matter when the answer is compared with K.  The
// kernel evaluates that band with Myers' bit-vector recurrence (vertical and
// horizontal +1/-1 deltas as bit masks, one column of the table per step),
// in a diagonal-aligned form: bit k of the state always holds diagonal
// k - Kb, so the band slides down one row per column by shifting the state
// right by one bit.
//
//  * Cells just outside the band are replaced by upper bounds (the row above
//    the band grows by +1 to the right, the row below the band by +1
//    downwards).  Every computed value is then >= the true value, and exact
//    wherever the true value is <= Kb, because such a cell is reached by an
//    optimal path that never leaves the band.  The result min(value, K+1)
//    therefore equals min(ED, K+1).
//  * Rows above row 0 are virtual rows with D[i][j] = j - i; they are
//    consistent with the recurrence, which removes all special cases at the
//    top-left corner.
//  * The value on the diagonal of the final cell, d* = |x| - |y|, is tracked
//    column by column: along a diagonal the value grows by 0 or 1, and it
//    stays put exactly when the characters match or a horizontal or
//    vertical -1 delta enters the cell.  Text columns past the end of a
//    shorter text match everything (a padding character whose match mask is
//    all ones), so finished pairs keep their value while the rest of the
//    wave continues.  A value above K ends the pair early.
//
// GPU mapping: a pair owns NL lanes of a wave (32 band bits per lane, NL =
// ceil((2K+2)/32)); a wave holds floor(64/NL) pairs.  The W-bit addition of
// Myers' step is a 32-bit add per lane plus a carry-lookahead across lanes
// done on two ballots with scalar arithmetic; the one-bit shift across lanes
// is a DPP wave_shl.  The match masks of the pattern (one bit array per
// symbol, the "Peq" table) and the text live in LDS.
#include <algorithm>

#include "ej_internal.h"

namespace ej {

namespace {

__device__ inline uint32_t dpp_from_next_lane(uint32_t x) {
    // lane i receives x of lane i+1 (lane 63 receives 0)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xf, 0xf, false);
}

__global__ void __launch_bounds__(64)
    k_verify(const uint8_t *__restrict__ codes_a, const uint64_t *__restrict__ off_a,
             uint64_t base_a, const uint8_t *__restrict__ codes_b,
             const uint64_t *__restrict__ off_b, uint64_t base_b,
             const uint64_t *__restrict__ pairs, uint64_t count, uint32_t K,
             const uint32_t *__restrict__ Kq, uint32_t sigma, uint32_t NL, uint32_t tpw,
             uint32_t wpp, uint32_t tstride, uint32_t tile_words, int32_t *__restrict__ dist) {
    extern __shared__ uint32_t lds[];
    const uint32_t lane = threadIdx.x;
    const uint32_t tile = lane / NL, l = lane - tile * NL;
    const bool in_tile = tile < tpw;
    const uint32_t Kb = 16 * NL - 1;  // band half-width: 32*NL >= 2*Kb + 2
    uint64_t last = 0;
    for (uint32_t q = 0; q < 64; q++)
        if ((q / NL) >= tpw || (q % NL) == NL - 1) last |= 1ull << q;
    const uint32_t keep = (l == NL - 1 || !in_tile) ? 0u : 0xFFFFFFFFu;
    uint32_t *tb = lds + (in_tile ? tile : 0) * tile_words;

    // padding symbol: matches every row
    for (uint32_t t = 0; t < tpw; t++)
        for (uint32_t w = lane; w < wpp; w += 64) lds[t * tile_words + sigma * wpp + w] = ~0u;

    for (uint64_t g = blockIdx.x; g * tpw < count; g += gridDim.x) {
        const uint64_t pidx = g * tpw + tile;
        const bool act = in_tile && pidx < count;
        uint32_t m = 0, nn = 0, Kp = K;
        const uint8_t *xp = codes_a, *yp = codes_a;
        if (act) {
            uint64_t code = pairs[pidx];
            uint32_t a = (uint32_t)(code >> 32), b = (uint32_t)code;
            uint64_t oa = off_a[a], ob = off_b[b];
            uint32_t la = (uint32_t)(off_a[a + 1] - oa), lb = (uint32_t)(off_b[b + 1] - ob);
            const uint8_t *pa = codes_a + (oa - base_a), *pb = codes_b + (ob - base_b);
            if (Kq) Kp = Kq[pidx];
            if (la >= lb) {
                xp = pa; m = la; yp = pb; nn = lb;
            } else {
                xp = pb; m = lb; yp = pa; nn = la;
            }
        }
        const bool skip = !act || m - nn > Kp;
        if (skip) {
            m = 0;
            nn = 0;
        }
        // a skipped pair keeps d* = 0 so that one lane of its tile owns the
        // (constant) result K_p + 1
        const uint32_t dstar = m - nn;
        __syncthreads();
        // ---- match masks of each pattern and the text of each pair -> LDS
        for (uint32_t t = 0; t < tpw; t++) {
            const uint32_t mt = readlane_u32(m, t * NL);
            const uint32_t nt = readlane_u32(nn, t * NL);
            const uint64_t xa = readlane_u64((uint64_t)(uintptr_t)xp, t * NL);
            const uint64_t ya = readlane_u64((uint64_t)(uintptr_t)yp, t * NL);
            const uint8_t *xt = (const uint8_t *)(uintptr_t)xa;
            const uint8_t *yt = (const uint8_t *)(uintptr_t)ya;
            uint32_t *pq = lds + t * tile_words;
            // bit index of pattern row i (1-based) is i + Kb
            for (uint32_t q = 0; q < wpp / 2; q++) {
                const int row = (int)(64 * q + lane) - (int)Kb;
                uint32_t c = 0xFFFFFFFFu;
                if (row >= 1 && row <= (int)mt) c = xt[row - 1];
                for (uint32_t ch = 0; ch < sigma; ch++) {
                    uint64_t msk = __builtin_amdgcn_ballot_w64(c == ch);
                    if (lane == 0) pq[ch * wpp + 2 * q] = (uint32_t)msk;
                    if (lane == 1) pq[ch * wpp + 2 * q + 1] = (uint32_t)(msk >> 32);
                }
            }
            uint8_t *tx = (uint8_t *)(pq + (sigma + 1) * wpp);
            for (uint32_t u = lane; u < tstride; u += 64) tx[u] = u < nt ? yt[u] : (uint8_t)sigma;
        }
        __syncthreads();

        uint32_t nmax = nn;
        for (int d = 32; d >= 1; d >>= 1) nmax = max(nmax, (uint32_t)__shfl_xor((int)nmax, d, 64));

        // ---- column 0: D[i][0] = |i|; bit k holds row k - Kb
        const int lo = 32 * (int)l;
        uint32_t Mv;
        if ((int)Kb >= lo + 31)
            Mv = ~0u;
        else if ((int)Kb < lo)
            Mv = 0u;
        else
            Mv = (1u << ((int)Kb - lo + 1)) - 1u;
        uint32_t Pv = ~Mv;
        const uint32_t kstar = Kb + dstar;
        const bool owner = in_tile && (kstar >> 5) == l;
        const uint32_t kmask = owner ? (1u << (kstar & 31)) : 0u;
        uint32_t Z = 0;  // columns in which the tracked diagonal did not grow
        const uint32_t *peq = tb;
        const uint32_t *txt = tb + (sigma + 1) * wpp;
        uint32_t jdone = 0;
        for (uint32_t jb = 0; jb < nmax; jb += 32) {
            uint32_t Eq[32];
            const uint32_t wbase = (jb >> 5) + l;
            uint32_t tw = 0;
#pragma unroll
            for (uint32_t s = 0; s < 32; s++) {
                if ((s & 3) == 0) tw = txt[(jb + s) >> 2];
                const uint32_t c = (tw >> (8 * (s & 3))) & 0xFFu;
                const uint32_t *pa = peq + c * wpp + wbase;
                Eq[s] = __builtin_amdgcn_alignbit(pa[1], pa[0], s);
            }
#pragma unroll
            for (uint32_t s = 0; s < 32; s++) {
                const uint32_t eq = Eq[s];
                const uint32_t Xv = eq | Mv;
                uint32_t sum = (eq & Pv) + Pv;
                const uint64_t G = __builtin_amdgcn_ballot_w64(sum < Pv);
                const uint64_t P = __builtin_amdgcn_ballot_w64(sum == 0xFFFFFFFFu);
                const uint64_t U = (G | P) & ~last, V = G & ~last;
                const uint64_t cin = (U + V) ^ U ^ V;
                sum += __builtin_amdgcn_inverse_ballot_w64(cin) ? 1u : 0u;
                const uint32_t Xh = (sum ^ Pv) | eq;
                const uint32_t Ph = Mv | ~(Xh | Pv);
                const uint32_t Mh = Pv & Xh;
                const uint32_t nx = dpp_from_next_lane(Xv) & keep;
                const uint32_t Xv1 = __builtin_amdgcn_alignbit(nx, Xv, 1);
                Pv = Mh | ~(Xv1 | Ph);
                Mv = Ph & Xv1;
                Z += __builtin_popcount((Xv1 | Mh) & kmask);
            }
            jdone = jb + 32;
            const uint32_t Vd = dstar + jdone - Z;
            const bool live = owner && !skip && Vd <= Kp && jdone < nn;
            if (__builtin_amdgcn_ballot_w64(live) == 0) break;
        }
        if (owner && act) {
            uint32_t res = skip ? Kp + 1 : dstar + jdone - Z;
            if (res > Kp + 1) res = Kp + 1;
            dist[pidx] = (int32_t)res;
        }
    }
}

__global__ void k_max_u32(const uint32_t *__restrict__ a, uint64_t n, uint32_t *__restrict__ out) {
    uint32_t mx = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        mx = max(mx, a[i]);
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, mx);
}

}  // namespace

uint32_t verify_lanes_for(uint32_t K) {
    uint64_t nl = (2ull * K + 2 + 31) / 32;
    if (nl == 0) nl = 1;
    return nl <= 64 ? (uint32_t)nl : 0u;
}

void verify(ej_ctx *ctx, const uint8_t *d_codes, const uint64_t *d_offsets, uint64_t base,
            uint32_t sigma, uint32_t maxlen, const uint64_t *d_pairs, uint64_t count, uint32_t K,
            const uint32_t *d_Kq, int32_t *d_dist, const uint8_t *d_codes_b,
            const uint64_t *d_offsets_b, uint64_t base_b, uint32_t maxlen_b) {
    if (count == 0) return;
    uint32_t Kmax = K;
    if (d_Kq) {
        uint32_t *d_mx = ws<uint32_t>(ctx, "verify_kmax", 1);
        EJ_HIP(hipMemsetAsync(d_mx, 0, 4, ctx->stream));
        uint64_t g = std::min<uint64_t>((count + 255) / 256, (uint64_t)ctx->num_cu * 8);
        hipLaunchKernelGGL(k_max_u32, dim3((uint32_t)g), dim3(256), 0, ctx->stream, d_Kq, count,
                           d_mx);
        EJ_CHECK_LAUNCH();
        read_back(ctx, d_mx, 4, &Kmax);
    }
    const uint32_t NL = verify_lanes_for(Kmax);
    if (NL == 0)
        fail(EJ_EUNSUPPORTED, "threshold " + std::to_string(Kmax) + " exceeds 1022 (band > 2048 bits)");
    if (!d_codes_b) {
        d_codes_b = d_codes;
        d_offsets_b = d_offsets;
        base_b = base;
        maxlen_b = maxlen;
    }
    const uint32_t W = 32 * NL;
    const uint32_t mx = std::max(maxlen, maxlen_b);
    const uint32_t mtext = std::min(maxlen, maxlen_b);
    uint32_t wpp = (mx + W + 95) / 32;
    wpp = (wpp + 1) & ~1u;
    const uint32_t tstride = ((mtext + 31) / 32) * 32 + 32;
    const uint32_t tile_words = (sigma + 1) * wpp + tstride / 4;
    const uint32_t tile_bytes = tile_words * 4;
    uint32_t tpw = 64 / NL;
    uint32_t budget = 48 * 1024;
    if ((int)budget > ctx->lds_max) budget = (uint32_t)ctx->lds_max;
    if (tile_bytes > budget) budget = (uint32_t)ctx->lds_max;
    if (tile_bytes > budget)
        fail(EJ_EUNSUPPORTED, "strings too long for the LDS-resident verification tile (" +
                                  std::to_string(tile_bytes) + " bytes)");
    tpw = std::min(tpw, budget / tile_bytes);
    size_t lds = (size_t)tpw * tile_bytes;
    uint64_t ngroups = (count + tpw - 1) / tpw;
    uint64_t grid = std::min<uint64_t>(ngroups, (uint64_t)ctx->num_cu * 16);
    if (lds > 65536)
        EJ_HIP(hipFuncSetAttribute((const void *)k_verify,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_verify, dim3((uint32_t)grid), dim3(64), lds, ctx->stream, d_codes,
                       d_offsets, base, d_codes_b, d_offsets_b, base_b, d_pairs, count, K, d_Kq,
                       sigma, NL, tpw, wpp, tstride, tile_words, d_dist);
    EJ_CHECK_LAUNCH();
}

}  // namespace ej
