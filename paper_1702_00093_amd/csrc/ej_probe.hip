// Peak probe for the integer VALU roofline.
//
// Verification (bit-parallel edit distance) is bound by 32-bit integer
// vector instructions, so its roofline needs the rate at which the chip
// issues them.  The probe runs eight independent dependency chains per lane
// (enough ILP with several waves per SIMD to hide the 4-8 cycle latency) of
// one instruction mix -- by default the instructions that dominate
// verification: 32-bit adds, 3-input logic (v_bitop3 on gfx950) and funnel
// shifts (v_alignbit); or one instruction class alone -- with no memory
// traffic except one store per lane at the end.  Each chain step is exactly
// one VALU instruction in the compiled loop (ISA checked: 4 unrolled steps x
// 8 chains x 3 instructions = 96 VALU instructions per iteration plus the
// loop counter's scalar add and branch), so the achieved rate is
//   waves x iterations x 96 x 64 lanes / kernel time  [lane-ops/s].
#include "ej_internal.h"

namespace ej {

namespace {

constexpr uint32_t PROBE_BLOCK = 256;
constexpr uint32_t PROBE_CHAINS = 8;
constexpr uint32_t PROBE_UNROLL = 4;
constexpr uint32_t PROBE_OPS_PER_STEP = 3;  // add, 3-input logic, funnel shift

// One chain step of instruction mix MIX (each a single VALU instruction in the
// compiled loop; checked in the ISA):
//   0: the verification mix -- add, 3-input logic, funnel shift in turn
//   1: 32-bit add (VOP2)
//   2: 2-input logic, xor (VOP2)
//   3: 3-input logic (v_bitop3)
//   4: funnel shift (v_alignbit)
//   5: add with the carry-out to a scalar mask (v_add_co_u32, VOP3)
// One chain step of instruction mix MIX, a single VALU instruction (checked
// in the ISA).  The single-class mixes are written as register-only inline
// assembly, since the compiler would otherwise fold repeated adds, xors or
// rotations of one value into one instruction:
//   0: the verification mix -- add, 3-input logic, funnel shift in turn
//   1: 32-bit add (v_add_u32, VOP2)
//   2: 2-input logic (v_xor_b32, VOP2)
//   3: 3-input logic (v_bitop3_b32)
//   4: funnel shift (v_alignbit_b32)
//   5: add with the carry-out to a scalar mask (v_add_co_u32, VOP3)
template <int MIX>
__device__ inline uint32_t probe_step(uint32_t x, uint32_t k0, uint32_t k1, uint32_t k2) {
    uint32_t r;
    if (MIX == 1) {
        asm volatile("v_add_u32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(k0));
    } else if (MIX == 2) {
        asm volatile("v_xor_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(k1));
    } else if (MIX == 3) {
        r = (x & k1) | (~x & k2) ^ (x & 0x0F0F0F0Fu);
    } else if (MIX == 4) {
        asm volatile("v_alignbit_b32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(k1), "v"(k2));
    } else {
        uint64_t carry;
        asm volatile("v_add_co_u32 %0, %1, %2, %3" : "=v"(r), "=s"(carry) : "v"(x), "v"(k0));
    }
    return r;
}

template <int MIX>
__global__ void __launch_bounds__(PROBE_BLOCK)
    k_probe_valu(uint32_t iters, uint32_t salt, uint32_t *__restrict__ out) {
    uint32_t a[PROBE_CHAINS];
    const uint32_t t = blockIdx.x * PROBE_BLOCK + threadIdx.x;
#pragma unroll
    for (uint32_t c = 0; c < PROBE_CHAINS; c++) a[c] = t * (2 * c + 1) + c;
    // loop-invariant operands that the compiler cannot fold (kernel argument)
    const uint32_t k0 = salt, k1 = salt * 0x9E3779B9u, k2 = salt ^ 0x5bd1e995u;
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (uint32_t u = 0; u < PROBE_UNROLL; u++) {
#pragma unroll
            for (uint32_t c = 0; c < PROBE_CHAINS; c++) {
                if (MIX == 0) {
                    uint32_t x = a[c] + k0;                          // v_add_u32
                    x = (x & k1) | (~x & k2) ^ (x & 0x0F0F0F0Fu);    // v_bitop3_b32
                    a[c] = __builtin_amdgcn_alignbit(x, x, 7 + c);    // v_alignbit_b32
                }
            }
            if (MIX != 0) {
                // chains interleaved: consecutive instructions are independent
#pragma unroll
                for (uint32_t o = 0; o < PROBE_OPS_PER_STEP; o++)
#pragma unroll
                    for (uint32_t c = 0; c < PROBE_CHAINS; c++)
                        a[c] = probe_step<MIX>(a[c], k0, k1, k2);
            }
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (uint32_t c = 0; c < PROBE_CHAINS; c++) s ^= a[c];
    out[t] = s;
}

}  // namespace

}  // namespace ej

using namespace ej;

extern "C" {

ej_status ej_probe_valu(ej_ctx *ctx, uint32_t mix, uint32_t iters, uint32_t blocks_per_cu,
                        double *lane_ops, float *ms) {
    if (!lane_ops || !ms || iters == 0 || blocks_per_cu == 0 || blocks_per_cu > 64 || mix > 5)
        return EJ_EINVAL;
    return run_guarded(ctx, [&] {
        const uint32_t blocks = (uint32_t)ctx->num_cu * blocks_per_cu;
        uint32_t *out = ws<uint32_t>(ctx, "probe_out", (uint64_t)blocks * PROBE_BLOCK);
        hipEvent_t e0 = ctx->timers.ev[6], e1 = ctx->timers.ev[7];
        using Kern = void (*)(uint32_t, uint32_t, uint32_t *);
        const Kern kerns[] = {k_probe_valu<0>, k_probe_valu<1>, k_probe_valu<2>,
                              k_probe_valu<3>, k_probe_valu<4>, k_probe_valu<5>};
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
