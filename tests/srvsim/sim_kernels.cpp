// CPU stand-ins for the stage, walk and finalize kernels, for testing the
// request loop.  Instead of a permanent they move tags: staging stores a hash
// of the request's matrix, each walk item writes (hash, x0) into its partial
// slot, and the finalize checks that every slot of the request carries the
// request's hash and the expected start index, so a skipped, misplaced or
// stale item is counted.  The walk follows the persistent kernels' work
// counter protocol exactly: waves take items from a 64-bit counter offset by
// `base` until the index passes `count`, one extra fetch per wave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <thread>

#include "internal.h"
#include "kernels.h"

using namespace permk;

std::atomic<long> sim_desync{0}, sim_bad_parts{0}, sim_items{0};

uint64_t sim_hash(const unsigned char *p, size_t b)
{
    uint64_t h = 1469598103934665603ull;       // FNV-1a
    for (size_t i = 0; i < b; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

namespace {
double ns_per_item()
{
    static const double v = getenv("SIM_NS_PER_ITEM") ? atof(getenv("SIM_NS_PER_ITEM")) : 0.0;
    return v;
}
}  // namespace

namespace permk {

int launch_stage(const MatDesc *d_mats, int nmats, const void *src, void *stage, void *stream)
{
    sim_enqueue((hipStream_t)stream, [=] {
        for (int q = 0; q < nmats; ++q) {
            const MatDesc &d = d_mats[q];
            const size_t b = (size_t)d.n * d.n * src_entry_bytes(d.variant);
            *(uint64_t *)((char *)stage + d.stage_off) =
                sim_hash((const unsigned char *)src + d.src_off, b);
        }
    });
    return 0;
}

int launch_walk(int, int, bool, bool, int, const WaveItem *d_items, uint32_t count,
                uint32_t grab, const MatDesc *d_mats, const void *stage, double *partials,
                unsigned long long *ctr, CtrState *state, int grid_blocks, void *stream,
                const void *fin_src, void *fin_out, int fin_nmats)
{
    // Fault injection: SIM_FAIL_WALK=k makes the k-th walk launch fail
    // (nothing of it is enqueued), as a failed kernel launch would.
    static std::atomic<long> launches{0};
    static const long fail_at = getenv("SIM_FAIL_WALK") ? atol(getenv("SIM_FAIL_WALK")) : 0;
    if (fail_at > 0 && ++launches == fail_at) return 1;
    if (fin_nmats) return 1;      // the request loop always stages and finalizes separately
    (void)fin_src;
    (void)fin_out;
    if (grab < 1 || !state) return 1;
    if (grid_blocks < 1) grid_blocks = 1;
    const uint64_t per_run = (uint64_t)(BLOCK / WAVE) * grab;
    const uint64_t runs = ((uint64_t)count + per_run - 1) / per_run;
    const uint32_t groups = ctr_groups(grid_blocks);
    CtrState before = *state;
    const bool dynamic = runs > (uint64_t)grid_blocks;
    if (dynamic)
        for (uint32_t x = 0; x < groups; ++x)
            state->base[x] += runs > x ? (runs - x + groups - 1) / groups : 0;
    sim_enqueue((hipStream_t)stream, [=] {
        auto walk_run = [&](uint64_t r) {
            const uint64_t end = std::min<uint64_t>(count, (r + 1) * per_run);
            for (uint64_t idx = r * per_run; idx < end; ++idx) {
                const WaveItem &w = d_items[idx];
                const MatDesc &d = d_mats[w.mat];
                // the descriptor slot still belongs to this item's request:
                // a slot handed to a new request while the item was in
                // flight shows up as a partial range that does not hold it
                if (w.slot < d.first_part || w.slot >= d.first_part + d.num_parts) sim_bad_parts++;
                uint64_t *slot = (uint64_t *)((char *)partials + 16 * (size_t)w.slot);
                slot[0] = *(const uint64_t *)((const char *)stage + d.stage_off);
                slot[1] = w.x0;
                sim_items++;
            }
        };
        // block b walks run b, then (more runs than blocks) claims more
        for (uint64_t b = 0; b < (uint64_t)grid_blocks && b < runs; ++b) walk_run(b);
        for (uint32_t x = 0; dynamic && x < groups; ++x) {
            unsigned long long *c = ctr + CTR_STRIDE * x;
            const uint64_t base = before.base[x];
            uint64_t v = *c;
            if (v != base) sim_desync++;
            const uint64_t nb = ((uint64_t)grid_blocks - x + groups - 1) / groups;
            long blocks = (long)nb;
            while (blocks > 0) {
                const uint64_t r = x + (uint64_t)groups * (nb + (uint32_t)(v - base));
                ++v;
                if (r >= runs) {
                    --blocks;
                    continue;
                }
                walk_run(r);
            }
            *c = v;
        }
        if (ns_per_item() > 0)
            std::this_thread::sleep_for(std::chrono::nanoseconds((long)(ns_per_item() * count)));
    });
    return 0;
}

int walk_occupancy(int, int n, bool, bool, int, int *blocks_per_cu)
{
    *blocks_per_cu = n > 30 ? 3 : 4;
    return 0;
}

int launch_finalize(const MatDesc *d_mats, int nmats, const double *partials, void *out,
                    void *stream)
{
    sim_enqueue((hipStream_t)stream, [=] {
        for (int q = 0; q < nmats; ++q) {
            const MatDesc &d = d_mats[q];
            const uint64_t h = *(const uint64_t *)((const char *)partials + d.stage_off);
            uint64_t bad = 0;
            if (d.n > 0) {
                const uint64_t T = 1ull << (d.n - 1);
                const uint64_t step = d.num_parts > 1 ? T / d.num_parts : 0;
                for (uint32_t i = 0; i < d.num_parts; ++i) {
                    const uint64_t *slot =
                        (const uint64_t *)((const char *)partials + 16 * (size_t)(d.first_part + i));
                    if (slot[0] != h || slot[1] != i * step) ++bad;
                }
            }
            sim_bad_parts += (long)bad;
            uint64_t *o = (uint64_t *)((char *)out + 16 * (size_t)d.out_slot);
            o[0] = h;
            o[1] = bad;
        }
    });
    return 0;
}

}  // namespace permk

namespace permi {

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    fprintf(stderr, "error %d: ", code);
    vfprintf(stderr, fmt, ap);
    fprintf(stderr, "\n");
    va_end(ap);
    return code;
}

// the library's default partition rule
int log2_chunk_for(const perm_ctx *, int variant, int n)
{
    if (n < 8) return 3;
    if (variant == V_MODP || variant == V_MONT) {
        const int c = n <= 26 ? n / 2 - 5 : std::min(n / 2 - 4, 13);
        return std::min(std::max(std::max(c, n - 27), 3), 20);
    }
    if (n < 14) return std::max(3, n - 7);
    if (n < 16) return n - 9;
    if (n <= 17) return n - 8;
    return n <= 22 ? std::min(n - 9, 11) : 10;
}

}  // namespace permi
