// Host checks of the planner (csrc/perm.cpp): for seeded random mixes of
// fields, orders and Gray ranges, every matrix's wave items tile its range
// exactly once with aligned power-of-two chunks and one partial slot each,
// launch groups are homogeneous (or fused) and sorted largest first, staged
// matrices do not overlap, and a repeated call reuses its plan only while
// the tuning table leaves its chunk lengths unchanged.  Exit code 0 = pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <unistd.h>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace permk;
using namespace permi;

static int failures = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            if (failures++ < 10) {                         \
                fprintf(stderr, "check failed: %s: ", #cond); \
                fprintf(stderr, __VA_ARGS__);              \
                fprintf(stderr, "\n");                     \
            }                                              \
        }                                                  \
    } while (0)

static void check_plan(const perm_ctx *ctx, const std::vector<MatIn> &in, const Plan &pl)
{
    CHECK(pl.mats.size() == in.size(), "mats %zu", pl.mats.size());
    // stage regions: 256-aligned, disjoint, in input order
    size_t next_stage = 0;
    for (size_t m = 0; m < in.size(); ++m) {
        const MatDesc &d = pl.mats[m];
        CHECK(d.n == in[m].n && d.variant == in[m].variant && d.out_slot == in[m].out_slot, "desc %zu", m);
        CHECK(d.stage_off % 256 == 0 && d.stage_off >= next_stage, "stage %zu", m);
        if (in[m].n > 0) next_stage = d.stage_off + stage_bytes(d.variant, d.n);
        // F_p finalize factor: f 2^(n-1) = R^(n-1) (Montgomery) or 1 (Barrett)
        // mod p for a whole permanent, f = R^(n-1) or 1 for an unscaled sum
        if ((d.variant == V_MODP || d.variant == V_MONT) && d.n > 0) {
            const uint64_t p = d.p, e = (uint64_t)d.n - 1;
            uint64_t want = 1, two = 1;
            for (uint64_t i = 0; i < e; ++i) {
                if (d.variant == V_MONT) want = want * ((1ull << 32) % p) % p;
                two = two * 2 % p;
            }
            const uint64_t got = in[m].no_scale ? d.fin_scale : (uint64_t)d.fin_scale * two % p;
            CHECK(got == want, "desc %zu: F_p finalize factor", m);
        }
    }
    // items per matrix tile the range once, slots once each
    std::vector<std::vector<const WaveItem *>> per(in.size());
    for (const WaveItem &w : pl.items) {
        CHECK(w.mat < in.size(), "item names matrix %u", w.mat);
        if (w.mat < in.size()) per[w.mat].push_back(&w);
    }
    size_t parts = 0;
    for (size_t m = 0; m < in.size(); ++m) {
        const MatIn &a = in[m];
        const MatDesc &d = pl.mats[m];
        if (a.n == 0) {
            CHECK(per[m].empty(), "n = 0 matrix %zu has items", m);
            continue;
        }
        const uint64_t T = 1ull << (a.n - 1);
        const uint64_t x0 = a.full ? 0 : a.x0, x1 = a.full ? T : a.x1;
        auto v = per[m];
        std::sort(v.begin(), v.end(), [](const WaveItem *p, const WaveItem *q) { return p->x0 < q->x0; });
        uint64_t at = x0;
        std::vector<bool> slot_seen(d.num_parts, false);
        for (const WaveItem *w : v) {
            CHECK(w->x0 == at, "matrix %zu: gap or overlap at %llu", m, (unsigned long long)at);
            CHECK(w->nlanes >= 1 && w->nlanes <= 64, "lanes");
            CHECK((w->x0 & ((1ull << w->log2L) - 1)) == 0, "unaligned chunk");
            CHECK(w->nlanes == 64 || w->log2L == 0, "partial wave with long chunks");
            if ((a.variant == V_MODP || a.variant == V_MONT)) CHECK(w->log2L <= 20, "F_p chunk");
            const uint32_t s = w->slot - d.first_part;
            CHECK(w->slot >= d.first_part && s < d.num_parts && !slot_seen[s], "slot");
            if (s < d.num_parts) slot_seen[s] = true;
            at += (uint64_t)w->nlanes << w->log2L;
        }
        CHECK(at == x1, "matrix %zu: tiles end at %llu, range ends at %llu", m, (unsigned long long)at,
              (unsigned long long)x1);
        CHECK(v.size() == d.num_parts, "parts");
        parts += d.num_parts;
    }
    CHECK(parts == pl.nparts, "nparts");
    // groups: contiguous, homogeneous unless fused, largest first
    size_t covered = 0;
    for (const Group &g : pl.groups) {
        CHECK(g.first_item == covered, "group order");
        covered += g.count;
        uint64_t prev = ~0ull;
        for (uint32_t q = 0; q < g.count; ++q) {
            const WaveItem &w = pl.items[g.first_item + q];
            const MatIn &a = in[w.mat];
            if (!g.fused) CHECK(a.variant == g.variant && a.n == g.n, "mixed group");
            else CHECK(a.variant != V_MONT && a.n <= g.nmax_fused, "fused bucket");
            const uint64_t work = ((uint64_t)w.nlanes << w.log2L) * step_cost(a.variant, a.n);
            CHECK(work <= prev, "group not sorted largest first");
            prev = work;
        }
    }
    CHECK(covered == pl.items.size(), "groups cover items");
    (void)ctx;
}

// The tuning file is keyed by device architecture and HIP runtime version:
// a saved table loads back; a table for another architecture or runtime,
// one without the key lines, or one with an F_p chunk above 2^20 or a
// malformed line is refused and leaves the context's table unchanged.
static void check_tune_files(perm_ctx *ctx)
{
    char path[] = "/tmp/plan_driver_tuneXXXXXX";
    const int fd = mkstemp(path);
    CHECK(fd >= 0, "mkstemp");
    if (fd < 0) return;
    close(fd);
    perm_tune t{11, 2};
    CHECK(perm_tune_set(ctx, PERM_C128, 21, &t) == PERM_OK, "set");
    CHECK(perm_tune_save(ctx, path) == PERM_OK, "save");
    ctx->tune.clear();
    CHECK(perm_tune_load(ctx, path) == PERM_OK, "load of a saved table");
    perm_tune got{};
    perm_tune_get(ctx, PERM_C128, 21, &got);
    CHECK(got.log2_chunk == 11 && got.grid_per_cu == 2, "round trip");
    std::string text;
    {
        FILE *f = fopen(path, "r");
        char buf[512];
        while (f && fgets(buf, sizeof buf, f)) text += buf;
        if (f) fclose(f);
    }
    auto write = [&](const std::string &body) {
        FILE *f = fopen(path, "w");
        fputs(body.c_str(), f);
        fclose(f);
    };
    auto replace = [&](const std::string &from, const std::string &to) {
        std::string b = text;
        const size_t at = b.find(from);
        CHECK(at != std::string::npos, "%s not in the saved table", from.c_str());
        if (at != std::string::npos) b.replace(at, from.size(), to);
        return b;
    };
    const std::string arch_line = "# arch " + ctx->arch + "\n";
    const std::vector<std::string> refused = {
        replace(arch_line, "# arch gfx942\n"),                 // another architecture
        replace("# hip 70200000\n", "# hip 60400000\n"),      // another runtime
        replace(arch_line, ""),                                 // no key
        text + "2 40 21 0\n",                                   // F_p chunk above 2^20
        text + "1 20 11\n",                                     // malformed
    };
    for (size_t i = 0; i < refused.size(); ++i) {
        write(refused[i]);
        CHECK(perm_tune_load(ctx, path) == PERM_EINVAL, "tuning file %zu was accepted", i);
        perm_tune_get(ctx, PERM_C128, 21, &got);
        CHECK(got.log2_chunk == 11, "a refused file changed the table");
    }
    unlink(path);
}

// The latency partition: a lone matrix whose batch partition leaves
// resident waves idle is split finer (never below 2^3 indices per lane, and
// never for orders below 10, where one item holds the whole range); the
// batch partition stays for calls that fill the device, for matrices not
// marked latency-eligible, and for (field, n) with a tuning-table entry.
// Either way the range is tiled exactly once.
static void check_latency_partition(perm_ctx *ctx)
{
    ctx->tune.clear();
    ctx->num_cus = 256;
    // waves per SIMD in a round: two for c128 and F_p, four for f64, capped
    // by the stub occupancy of 3 blocks per CU
    auto slots_of = [](int variant) { return (variant == V_F64 ? 3ull : 2ull) * 256 * 4; };
    Plan pl;
    for (int variant : {(int)V_C128, (int)V_F64, (int)V_MODP})
        for (int n = 8; n <= 32; ++n) {
            const uint64_t slots = slots_of(variant);
            std::vector<MatIn> in(1);
            in[0].variant = variant;
            in[0].n = n;
            in[0].p = variant == V_MODP ? 2147483647u : 0;
            in[0].latency = true;
            plan(ctx, in, pl);
            check_plan(ctx, in, pl);
            const uint32_t lat_items = (uint32_t)pl.items.size();
            const uint32_t lat_c = pl.items[0].log2L;
            in[0].latency = false;
            plan(ctx, in, pl);
            check_plan(ctx, in, pl);
            const uint32_t items = (uint32_t)pl.items.size();
            const uint32_t c0 = pl.items[0].log2L;
            if (n < 10 || items >= slots) {
                CHECK(lat_items == items, "v%d n=%d: latency partition where the batch one fills", variant, n);
            } else {
                CHECK(lat_c <= c0 && (lat_c >= 3 || lat_c == c0), "v%d n=%d: chunk 2^%u", variant, n, lat_c);
                CHECK(lat_items >= items, "v%d n=%d: fewer items", variant, n);
                // a lone matrix that one wave per SIMD holds at 2^3
                // indices per lane takes that length
                if ((1ull << (n - 1)) >> 9 <= 256ull * 4)
                    CHECK(lat_c == 3, "v%d n=%d: chunk 2^%u, not 2^3", variant, n, lat_c);
            }
            // a table entry decides
            perm_tune t{c0 > 4 ? (int)c0 - 1 : (int)c0, 0};
            perm_tune_set(ctx, variant == V_MODP ? PERM_MODP : variant, n, &t);
            in[0].latency = true;
            plan(ctx, in, pl);
            CHECK(pl.items[0].log2L == (uint32_t)t.log2_chunk, "v%d n=%d: table entry ignored", variant, n);
            ctx->tune.clear();
        }
    // one c128 matrix of order 24 fills two waves per SIMD
    std::vector<MatIn> in(1);
    in[0].variant = V_C128;
    in[0].n = 24;
    in[0].latency = true;
    plan(ctx, in, pl);
    CHECK(pl.items.size() >= slots_of(V_C128), "U(24) alone: %zu items", pl.items.size());
}

int main()
{
    perm_ctx *ctx = nullptr;
    if (perm_ctx_create(0, 0, &ctx) != PERM_OK) return 2;
    std::mt19937_64 g(2602);
    for (int trial = 0; trial < 300; ++trial) {
        const int count = 1 + (int)(g() % (trial % 3 == 0 ? 200 : 12));
        const bool one_shape = trial % 4 == 0;
        std::vector<MatIn> in(count);
        const int v0 = (int)(g() % 3), n0 = (int)(g() % 30);
        for (int m = 0; m < count; ++m) {
            MatIn &a = in[m];
            a.variant = one_shape ? v0 : (int)(g() % 4);
            a.n = one_shape ? n0 : (int)(g() % 35);
            a.p = (a.variant >= V_MODP) ? 2147483647u : 0;
            a.src_off = (uint64_t)m * 16 * 48 * 48;
            a.out_slot = (uint32_t)m;
            a.kahan = true;
            a.full = (g() % 3) != 0 || a.n == 0;
            if (!a.full) {
                const uint64_t T = 1ull << (a.n - 1);
                uint64_t u = g() % (T + 1), w = g() % (T + 1);
                a.x0 = std::min(u, w);
                a.x1 = std::max(u, w);
                a.no_scale = true;
            }
        }
        Plan &pl = ctx->scratch_plan;
        if (plan(ctx, in, pl) != PERM_OK) { fprintf(stderr, "plan failed\n"); return 1; }
        check_plan(ctx, in, pl);
    }
    // cache: identical small inputs reuse the plan; a table change does not
    std::vector<MatIn> in(3);
    for (int m = 0; m < 3; ++m) {
        in[m].variant = V_MODP; in[m].n = 28; in[m].p = 1073742209u;
        in[m].src_off = (uint64_t)m * 28 * 28 * 4; in[m].out_slot = (uint32_t)m;
    }
    Plan &pl = ctx->scratch_plan;
    plan(ctx, in, pl);
    const uint64_t id = ctx->plan_id;
    const size_t items = pl.items.size();
    plan(ctx, in, pl);
    CHECK(ctx->plan_id == id, "identical call rebuilt the plan");
    perm_tune t{12, 0};
    perm_tune_set(ctx, PERM_MODP, 28, &t);
    plan(ctx, in, pl);
    CHECK(ctx->plan_id != id, "table change did not rebuild");
    CHECK(pl.items.size() * 4 == items, "chunk 2^12 should give a quarter of the items of 2^10");
    check_plan(ctx, in, pl);
    in[1].src_off += 4;
    plan(ctx, in, pl);
    CHECK(ctx->plan_id != id, "changed input reused the plan");
    check_tune_files(ctx);
    check_latency_partition(ctx);
    perm_ctx_destroy(ctx);
    printf("planner checks: %d failures\n", failures);
    fflush(stdout);
    _Exit(failures ? 1 : 0);
}
