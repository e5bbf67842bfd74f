// Context, workspace and error plumbing of the C ABI.
#include <string.h>

#include <mutex>
#include <new>

#include "ej_internal.h"

namespace ej {

// Scratch memory of ej_verify_static, for callers that cannot allocate: one
// array per device, held from the library's first use on that device until
// the process ends.  Host code never passes `scratch` itself to a kernel or a
// copy (its host-side name is a stand-in, not a device address); it uses the
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Called by ej_create with the context's device current.  A failed lookup
// is kept as the device's error and reported by ej_verify_static; the other
// entry points do not need the array.
hipError_t g_scratch_err[MAX_DEVICES] = {};

void static_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        (void)hipGetLastError();
        return;
    }
    g_scratch_ptr[device] = p;
}
}  // namespace

void *static_scratch(ej_ctx *ctx) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
        fail(EJ_EUNSUPPORTED, "no static scratch for device " + std::to_string(ctx->device));
    if (!g_scratch_ptr[ctx->device])
        fail(EJ_EHIP, std::string("hipGetSymbolAddress of the static scratch array failed: ") +
                          hipGetErrorString(g_scratch_err[ctx->device]));
    return g_scratch_ptr[ctx->device];
}

void fail(ej_status code, const std::string &msg) { throw Error{code, msg}; }

static void *arena_get(ej_ctx *ctx, const std::string &name, size_t bytes) {
    Arena &a = ctx->arena;
    auto it = a.named.find(name);
    if (it != a.named.end() && it->second.second >= bytes) return a.base + it->second.first;
    const size_t off = (a.used + 255) & ~(size_t)255;
    if (off > a.cap || bytes > a.cap - off)
        fail(EJ_ENOMEM, "the call needs more than the " + std::to_string(a.cap >> 20) +
                            " MiB of static scratch (buffer '" + name + "' of " +
                            std::to_string(bytes) + " bytes at offset " + std::to_string(off) +
                            "); use the allocating entry point for inputs this large");
    a.used = off + bytes;
    a.named[name] = {off, bytes};
    return a.base + off;
}

void *ws_get(ej_ctx *ctx, const std::string &name, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (ctx->arena.base) return arena_get(ctx, name, bytes);
    DevBuf &b = ctx->ws[name];
    if (b.bytes < bytes) {
        // a captured graph holds the addresses of the buffers it uses: no
        // buffer may move while a capture is open
        if (ctx->capturing)
            fail(EJ_EHIP, "workspace buffer '" + name + "' would grow inside a graph capture");
        ctx->ws_gen++;
        if (b.p) {
            EJ_HIP(hipStreamSynchronize(ctx->stream));
            EJ_HIP(hipFree(b.p));
            b.p = nullptr;
            b.bytes = 0;
        }
        size_t want = bytes + bytes / 8 + 256;  // grow with headroom
        hipError_t e = hipMalloc(&b.p, want);
        if (e != hipSuccess) {
            b.p = nullptr;
            fail(EJ_ENOMEM, "device allocation of " + std::to_string(want) + " bytes for '" +
                                name + "' failed: " + hipGetErrorString(e));
        }
        b.bytes = want;
    }
    return b.p;
}

size_t ws_capacity(ej_ctx *ctx, const std::string &name) {
    auto it = ctx->ws.find(name);
    return it == ctx->ws.end() ? 0 : it->second.bytes;
}

void sync(ej_ctx *ctx) { EJ_HIP(hipStreamSynchronize(ctx->stream)); }

void run_captured(ej_ctx *ctx, const std::string &key, const std::function<void()> &enqueue) {
    // inside an open capture (a whole join being captured) the launches
    // become part of that graph
    if (!ctx->graph_on || ctx->capturing) {
        enqueue();
        return;
    }
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= 32) {  // launch shapes changed often: start over
            for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
            ctx->graphs.clear();
        }
        hipGraph_t g = nullptr;
        EJ_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        ctx->capturing = true;
        try {
            enqueue();
        } catch (...) {
            ctx->capturing = false;
            (void)hipStreamEndCapture(ctx->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        ctx->capturing = false;
        EJ_HIP(hipStreamEndCapture(ctx->stream, &g));
        hipGraphExec_t ge = nullptr;
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) fail(EJ_EHIP, std::string("graph instantiation: ") + hipGetErrorString(e));
        it = ctx->graphs.emplace(key, ge).first;
    }
    EJ_HIP(hipGraphLaunch(it->second, ctx->stream));
}

void read_back(ej_ctx *ctx, const void *dsrc, size_t bytes, void *hdst) {
    if (bytes > 4096) fail(EJ_EINVAL, "read_back larger than the pinned staging buffer");
    EJ_HIP(hipMemcpyAsync(ctx->pinned, dsrc, bytes, hipMemcpyDeviceToHost, ctx->stream));
    EJ_HIP(hipStreamSynchronize(ctx->stream));
    memcpy(hdst, ctx->pinned, bytes);
}

}  // namespace ej

using namespace ej;

extern "C" {

int ej_version(void) { return 1 * 10000 + 0 * 100 + 0; }

ej_status ej_create(ej_ctx **out, int device, void *hip_stream) {
    if (!out) return EJ_EINVAL;
    *out = nullptr;
    ej_ctx *ctx = new (std::nothrow) ej_ctx();
    if (!ctx) return EJ_ENOMEM;
    try {
        int ndev = 0;
        EJ_HIP(hipGetDeviceCount(&ndev));
        if (device < 0 || device >= ndev) fail(EJ_EINVAL, "no such device");
        ctx->device = device;
        EJ_HIP(hipSetDevice(device));
        if (hip_stream) {
            ctx->stream = (hipStream_t)hip_stream;
            ctx->own_stream = false;
        } else {
            EJ_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
            ctx->own_stream = true;
        }
        EJ_HIP(hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, device));
        int lds = 65536;
        EJ_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
        ctx->lds_max = lds;
        EJ_HIP(hipHostMalloc((void **)&ctx->pinned, 4096, hipHostMallocDefault));
        static_scratch_init(device);
        for (int i = 0; i < 8; i++) EJ_HIP(hipEventCreate(&ctx->timers.ev[i]));
        for (int i = 0; i < 4; i++) EJ_HIP(hipEventCreate(&ctx->timers.kv[i]));
    } catch (const Error &e) {
        ej_status c = e.code;
        ej_destroy(ctx);
        return c;
    }
    *out = ctx;
    return EJ_OK;
}

void ej_destroy(ej_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->ws)
        if (kv.second.p) (void)hipFree(kv.second.p);
    ctx->ws.clear();
    for (int i = 0; i < 8; i++)
        if (ctx->timers.ev[i]) (void)hipEventDestroy(ctx->timers.ev[i]);
    for (int i = 0; i < 4; i++)
        if (ctx->timers.kv[i]) (void)hipEventDestroy(ctx->timers.kv[i]);
    for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->pinned_out) (void)hipHostFree(ctx->pinned_out);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *ej_last_error(const ej_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

uint64_t ej_workspace_bytes(const ej_ctx *ctx) {
    if (!ctx) return 0;
    uint64_t s = 0;
    for (auto &kv : ctx->ws) s += kv.second.bytes;
    return s;
}

static uint32_t *tune_slot(ej::Tuning &t, const char *name, uint32_t *lo, uint32_t *hi) {
    struct Item {
        const char *name;
        uint32_t Tuning::*field;
        uint32_t lo, hi;
    };
    static const Item items[] = {
        {"verify_lds_budget", &Tuning::verify_lds_budget, 4096, 1u << 20},
        {"verify_pass1_cols", &Tuning::verify_pass1_cols, 0, 1u << 30},
        {"verify_blocks_per_cu", &Tuning::verify_blocks_per_cu, 1, 1024},
        {"verify_ring", &Tuning::verify_ring, 0, 2},
        {"verify_mode", &Tuning::verify_mode, 0, 3},
        {"verify_order", &Tuning::verify_order, 0, 1},
        {"verify_split", &Tuning::verify_split, 0, 16},
        {"embed_lds_budget", &Tuning::embed_lds_budget, 0, 1u << 20},
        {"radix_bits", &Tuning::radix_bits, 4, 11},
        {"bucket_key_bits", &Tuning::bucket_key_bits, 0, 32},
        {"dedup_sort", &Tuning::dedup_sort, 0, 1},
        {"raw_limit", &Tuning::raw_limit, 0, 0xFFFFFFFEu},
        {"verify_wpl", &Tuning::verify_wpl, 1, 4},
        {"verify_len_order", &Tuning::verify_len_order, 0, 1},
    };
    if (!name) return nullptr;
    for (const Item &it : items)
        if (strcmp(it.name, name) == 0) {
            *lo = it.lo;
            *hi = it.hi;
            return &(t.*(it.field));
        }
    return nullptr;
}

ej_status ej_tune_set(ej_ctx *ctx, const char *name, uint32_t value) {
    if (!ctx) return EJ_EINVAL;
    uint32_t lo = 0, hi = 0;
    uint32_t *slot = tune_slot(ctx->tune, name, &lo, &hi);
    if (!slot || value < lo || value > hi) {
        ctx->err = std::string("unknown knob or value out of range: ") + (name ? name : "(null)");
        return EJ_EINVAL;
    }
    if (strcmp(name, "verify_pass1_cols") == 0 && (value % 32) != 0) {
        ctx->err = "verify_pass1_cols must be a multiple of 32";
        return EJ_EINVAL;
    }
    if (strcmp(name, "verify_split") == 0 && (value & (value - 1)) != 0) {
        ctx->err = "verify_split must be 0 or a power of two up to 16";
        return EJ_EINVAL;
    }
    *slot = value;
    return EJ_OK;
}

ej_status ej_tune_get(const ej_ctx *ctx, const char *name, uint32_t *value) {
    if (!ctx || !value) return EJ_EINVAL;
    uint32_t lo = 0, hi = 0;
    uint32_t *slot = tune_slot(const_cast<ej_ctx *>(ctx)->tune, name, &lo, &hi);
    if (!slot) return EJ_EINVAL;
    *value = *slot;
    return EJ_OK;
}

ej_status ej_set_explicit_randomness(ej_ctx *ctx, uint32_t r, uint32_t z, uint32_t m, uint32_t L,
                                     uint32_t sigma, const uint8_t *Rbits, const uint32_t *pos,
                                     const uint64_t *v) {
    if (!ctx) return EJ_EINVAL;
    try {
        Explicit &ex = ctx->ex;
        if (!Rbits) {
            ex = Explicit();
            return EJ_OK;
        }
        if (!pos || r == 0 || z == 0 || m == 0 || L == 0 || sigma == 0)
            fail(EJ_EINVAL, "explicit randomness needs Rbits, pos and non-zero sizes");
        uint64_t nbits = (uint64_t)L * sigma;
        ex.r = r;
        ex.z = z;
        ex.m = m;
        ex.L = L;
        ex.sigma = sigma;
        ex.nw = (uint32_t)((nbits + 31) / 32) + 2;
        ex.Rwords.assign((size_t)r * ex.nw, 0u);
        for (uint32_t l = 0; l < r; l++)
            for (uint64_t b = 0; b < nbits; b++)
                if (Rbits[l * nbits + b]) ex.Rwords[(size_t)l * ex.nw + b / 32] |= 1u << (b % 32);
        ex.pos.assign(pos, pos + (size_t)r * z * m);
        for (uint32_t x : ex.pos)
            if (x >= L) fail(EJ_EINVAL, "explicit coordinate outside [0, L)");
        if (v) {
            ex.v.assign(v, v + (size_t)r * z * m);
            for (uint64_t x : ex.v)
                if (x >= P61) fail(EJ_EINVAL, "explicit v outside [0, 2^61-1)");
        } else {
            ex.v.clear();
        }
        ex.active = true;
        return EJ_OK;
    } catch (const Error &e) {
        ctx->err = e.msg;
        return e.code;
    }
}

}  // extern "C"
