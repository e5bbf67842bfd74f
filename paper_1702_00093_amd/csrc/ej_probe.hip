// Peak probe for the integer VALU roofline.
//
// Verification (bit-parallel edit distance) is bound by 32-bit integer
// vector instructions, so its roofline needs the rate at which the chip
// issues them.  The probe runs eight independent dependency chains per lane
// (enough ILP with several waves per SIMD to hide the instruction latency)
// of one instruction class -- or of the mix that dominates verification:
// 32-bit adds, 3-input logic (v_bitop3 on gfx950) and funnel shifts
// (v_alignbit) in turn -- with no memory traffic except one store per lane
// at the end.  Every operand is a register or an inline constant (a 32-bit
// literal lengthens the instruction and changes its rate, and verification's
// instructions carry none).  Each chain step is exactly one VALU instruction
// (register-only inline assembly for the single classes, which the compiler
// would otherwise fold; ISA checked: 4 unrolled steps x 8 chains x 3 steps =
// 96 VALU instructions per iteration plus the loop counter's scalar add and
// branch), so the achieved rate is
//   waves x iterations x 96 x 64 lanes / kernel time  [lane-ops/s].
#include "ej_internal.h"

namespace ej {

namespace {

constexpr uint32_t PROBE_BLOCK = 256;
constexpr uint32_t PROBE_CHAINS = 8;
constexpr uint32_t PROBE_UNROLL = 4;
constexpr uint32_t PROBE_OPS_PER_STEP = 3;
constexpr uint32_t PROBE_NMIX = 15;

// One chain step of instruction class MIX (1..14), a single VALU instruction:
//   1 v_add_u32            2 v_xor_b32            3 v_bitop3_b32
//   4 v_alignbit_b32       5 v_add_co_u32 (carry-out to a scalar mask)
//   6 v_addc_co_u32 (carry in and out through a scalar mask, one carry chain
//     per dependency chain, as in a multi-word add)
//   7 v_cmp_eq_u32 (to VCC; the chain value passes through unchanged)
//   8 v_mov_b32 with DPP wave_shl:1 (a one-lane shift across the wave)
//   9 v_bcnt_u32_b32       10 v_add3_u32          11 v_cndmask_b32 on a
//     scalar mask that the loop never writes
//   12 v_or3_b32           13 v_and_or_b32        14 v_mul_u32_u24 with an
//     SDWA byte select (a symbol byte times a row stride)
template <int MIX>
__device__ inline uint32_t probe_step(uint32_t x, uint32_t k0, uint32_t k1, uint32_t k2,
                                      uint64_t m, uint64_t &cy) {
    uint32_t r = x;
    if (MIX == 1) {
        asm volatile("v_add_u32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(k0));
    } else if (MIX == 2) {
        asm volatile("v_xor_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(k1));
    } else if (MIX == 3) {
        asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xde" : "=v"(r) : "v"(x), "v"(k1), "v"(k2));
    } else if (MIX == 4) {
        asm volatile("v_alignbit_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(k1), "v"(k2));
    } else if (MIX == 5) {
        uint64_t carry;
        asm volatile("v_add_co_u32 %0, %1, %2, %3" : "=v"(r), "=s"(carry) : "v"(x), "v"(k0));
    } else if (MIX == 6) {
        asm volatile("v_addc_co_u32 %0, %1, %2, %3, %4"
                     : "=v"(r), "=s"(cy) : "v"(x), "v"(k0), "s"(cy));
    } else if (MIX == 7) {
        asm volatile("v_cmp_eq_u32 vcc, %0, %1" : : "v"(x), "v"(k0) : "vcc");
    } else if (MIX == 8) {
        asm volatile("v_mov_b32_dpp %0, %1 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                     : "=v"(r) : "v"(x));
    } else if (MIX == 9) {
        asm volatile("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(k0));
    } else if (MIX == 10) {
        asm volatile("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(k0), "v"(k1));
    } else if (MIX == 11) {
        asm volatile("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(k1), "v"(x), "s"(m));
    } else if (MIX == 12) {
        asm volatile("v_or3_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(k1), "v"(k2));
    } else if (MIX == 13) {
        asm volatile("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(k1), "v"(k2));
    } else {
        asm volatile(
            "v_mul_u32_u24_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD "
            "src0_sel:BYTE_1 src1_sel:DWORD"
            : "=v"(r) : "v"(x), "v"(k0));
    }
    return r;
}

template <int MIX>
__global__ void __launch_bounds__(PROBE_BLOCK)
    k_probe_valu(uint32_t iters, uint32_t salt, uint32_t *__restrict__ out) {
    uint32_t a[PROBE_CHAINS];
    uint64_t cy[PROBE_CHAINS];
    const uint32_t t = blockIdx.x * PROBE_BLOCK + threadIdx.x;
#pragma unroll
    for (uint32_t c = 0; c < PROBE_CHAINS; c++) {
        a[c] = t * (2 * c + 1) + c;
        cy[c] = 0;
    }
    // loop-invariant operands that the compiler cannot fold (kernel argument)
    const uint32_t k0 = salt, k1 = salt * 0x9E3779B9u, k2 = salt ^ 0x5bd1e995u;
    const uint64_t m = 0x5555555555555555ull * salt;
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (uint32_t u = 0; u < PROBE_UNROLL; u++) {
            if (MIX == 0) {
                // add, 3-input logic, funnel shift in turn, chains interleaved
#pragma unroll
                for (uint32_t c = 0; c < PROBE_CHAINS; c++) a[c] = probe_step<1>(a[c], k0, k1, k2, m, cy[c]);
#pragma unroll
                for (uint32_t c = 0; c < PROBE_CHAINS; c++) a[c] = probe_step<3>(a[c], k0, k1, k2, m, cy[c]);
#pragma unroll
                for (uint32_t c = 0; c < PROBE_CHAINS; c++) a[c] = probe_step<4>(a[c], k0, k1, k2, m, cy[c]);
            } else {
                // chains interleaved: consecutive instructions are independent
#pragma unroll
                for (uint32_t o = 0; o < PROBE_OPS_PER_STEP; o++)
#pragma unroll
                    for (uint32_t c = 0; c < PROBE_CHAINS; c++)
                        a[c] = probe_step<MIX>(a[c], k0, k1, k2, m, cy[c]);
            }
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (uint32_t c = 0; c < PROBE_CHAINS; c++) s ^= a[c] ^ (uint32_t)cy[c];
    out[t] = s;
}

}  // namespace

}  // namespace ej

using namespace ej;

extern "C" {

ej_status ej_probe_valu(ej_ctx *ctx, uint32_t mix, uint32_t iters, uint32_t blocks_per_cu,
                        double *lane_ops, float *ms) {
    if (!lane_ops || !ms || iters == 0 || blocks_per_cu == 0 || blocks_per_cu > 64 ||
        mix >= PROBE_NMIX)
        return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        const uint32_t blocks = (uint32_t)ctx->num_cu * blocks_per_cu;
        uint32_t *out = ws<uint32_t>(ctx, "probe_out", (uint64_t)blocks * PROBE_BLOCK);
        hipEvent_t e0 = ctx->timers.ev[6], e1 = ctx->timers.ev[7];
        using Kern = void (*)(uint32_t, uint32_t, uint32_t *);
        const Kern kerns[PROBE_NMIX] = {
            k_probe_valu<0>,  k_probe_valu<1>,  k_probe_valu<2>,  k_probe_valu<3>,
            k_probe_valu<4>,  k_probe_valu<5>,  k_probe_valu<6>,  k_probe_valu<7>,
            k_probe_valu<8>,  k_probe_valu<9>,  k_probe_valu<10>, k_probe_valu<11>,
            k_probe_valu<12>, k_probe_valu<13>, k_probe_valu<14>};
        const Kern kern = kerns[mix];
        // one untimed launch warms the clocks and the code object
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(PROBE_BLOCK), 0, ctx->stream, iters / 8 + 1,
                           3u, out);
        EJ_CHECK_LAUNCH();
        EJ_HIP(hipEventRecord(e0, ctx->stream));
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(PROBE_BLOCK), 0, ctx->stream, iters, 5u, out);
        EJ_CHECK_LAUNCH();
        EJ_HIP(hipEventRecord(e1, ctx->stream));
        sync(ctx);
        float t = 0.f;
        EJ_HIP(hipEventElapsedTime(&t, e0, e1));
        *ms = t;
        const double ops = (double)blocks * PROBE_BLOCK * iters * PROBE_UNROLL * PROBE_CHAINS *
                           PROBE_OPS_PER_STEP;
        *lane_ops = t > 0.f ? ops / (t * 1e-3) : 0.0;
    });
}

}  // extern "C"
