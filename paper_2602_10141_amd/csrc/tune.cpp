// Autotuner for the work partition: per (field, n), the per-lane chunk
// length 2^c of the Gray walk.  Candidates around the default are timed on
// the context's device with HIP events over a batch of matrices drawn from a
// fixed xorshift stream, and the fastest is stored in the context's table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace permk;
using namespace permi;

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return permi::fail(PERM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static uint64_t xorshift(uint64_t &s)
{
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
}

// Fastest of `reps` timed executions of a plan (after one warm-up).
static int time_plan(perm_ctx *ctx, Plan &pl, const void *src, void *out, size_t slots, int reps,
                     float *ms)
{
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    int rc = execute(ctx, pl, src, out, slots, ctx->stream);   // warm-up
    *ms = 0.0f;
    for (int r = 0; r < reps && rc == PERM_OK; ++r) {
        (void)hipEventRecord(a, ctx->stream);
        rc = execute(ctx, pl, src, out, slots, ctx->stream);
        (void)hipEventRecord(b, ctx->stream);
        float t = 0.0f;
        if (rc == PERM_OK && hipEventSynchronize(b) == hipSuccess &&
            hipEventElapsedTime(&t, a, b) == hipSuccess && (r == 0 || t < *ms))
            *ms = t;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

extern "C" int perm_autotune(perm_ctx *ctx, int field, int n_lo, int n_hi, int batch)
{
    if (!ctx || n_lo < 1 || n_hi < n_lo || n_hi > PERM_NMAX ||
        (field != PERM_C128 && field != PERM_F64 && field != PERM_MODP))
        return fail(PERM_EINVAL, "bad autotune arguments");
    const int count = std::max(1, batch);
    const int variant = field == PERM_C128 ? V_C128 : (field == PERM_F64 ? V_F64 : V_MODP);
    const uint32_t p = 2147483647u;   // 2^31 - 1, prime
    int rc = begin_call(ctx, ctx->stream);
    if (rc != PERM_OK) return rc;
    for (int n = n_lo; n <= n_hi; ++n) {
        const size_t per = (size_t)n * n * src_entry_bytes(variant);
        std::vector<unsigned char> host(per * count);
        uint64_t s = 0x9E3779B97F4A7C15ull ^ (uint64_t)(n * 1315423911u + field);
        if (variant == V_MODP) {
            uint32_t *h = (uint32_t *)host.data();
            for (size_t i = 0; i < host.size() / 4; ++i) h[i] = (uint32_t)(xorshift(s) % p);
        } else {
            double *h = (double *)host.data();
            for (size_t i = 0; i < host.size() / 8; ++i)
                h[i] = (double)(int64_t)(xorshift(s) >> 11) / 4503599627370496.0 - 1.0;
        }
        if ((rc = ensure(ctx, ctx->src, host.size())) != PERM_OK) return rc;
        HIPCHK(hipMemcpy(ctx->src.p, host.data(), host.size(), hipMemcpyHostToDevice));
        if ((rc = ensure(ctx, ctx->outs, (size_t)count * 16)) != PERM_OK) return rc;
        std::vector<MatIn> in(count);
        for (int i = 0; i < count; ++i) {
            in[i].variant = variant;
            in[i].n = n;
            in[i].p = variant == V_MODP ? p : 0;
            in[i].src_off = per * i;
            in[i].out_slot = (uint32_t)i;
            in[i].full = true;
        }
        const int cmax = std::min(n - 1 - 6, variant == V_MODP ? 20 : 24);
        const int cdef = default_log2_chunk(variant, n);
        const auto saved = ctx->tune;
        int best_c = 0;
        float best = 0.0f;
        // small jobs (a single permanent, say) try every chunk length and
        // repeat the timing; large ones a window around the default, once
        const double work = (double)count * std::ldexp(1.0, n - 1);
        const bool small = work < std::ldexp(1.0, 28);
        const int reps = small ? 5 : 1;
        const int c_lo = small ? 3 : std::max(3, cdef - 4);
        const int c_hi = small ? cmax : std::min(cmax, cdef + 4);
        for (int c = c_lo; c <= c_hi; ++c) {
            ctx->tune[{field, n}] = perm_tune{c, 0};
            Plan &pl = ctx->scratch_plan;
            if ((rc = plan(ctx, in, pl)) != PERM_OK) { ctx->tune = saved; return rc; }
            float ms = 0.0f;
            if ((rc = time_plan(ctx, pl, ctx->src.p, ctx->outs.p, (size_t)count, reps, &ms)) != PERM_OK) {
                ctx->tune = saved;
                return rc;
            }
            if (best_c == 0 || ms < best) { best = ms; best_c = c; }
        }
        ctx->tune = saved;
        if (best_c > 0) ctx->tune[{field, n}] = perm_tune{best_c, 0};
    }
    return end_call(ctx, ctx->stream);
}
