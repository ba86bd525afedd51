// libperm host library: the C ABI of include/perm.h.
//
// Every call follows the same pipeline (the hot path of the paper's Sec. 2):
//   plan     host: split each matrix's Gray index range [0, 2^(n-1)) into
//                  wavefront items of 64 lanes x 2^c indices, largest first;
//   stage    device: matrices -> +-2A columns in field-native form;
//   walk     device: persistent Gray-code Glynn walk, one partial per item;
//   finalize device: fixed-order reduction per matrix, 2^-(n-1) scaling;
//   lift     host (CRT only): Garner reconstruction of the signed integer.
// The host never evaluates any part of a permanent itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/perm.h"
#include "internal.h"
#include "kernels.h"
#include "noalloc.h"
#include "numth.h"

using namespace permk;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

int permi::fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

extern "C" const char *perm_strerror(int status)
{
    switch (status) {
    case PERM_OK: return "ok";
    case PERM_EINVAL: return "invalid argument";
    case PERM_ERANGE: return "out of range";
    case PERM_ENOMEM: return "out of memory or over the HBM budget";
    case PERM_EDEVICE: return "device error";
    case PERM_EAGAIN: return "queue full, try again";
    case PERM_ENOTFOUND: return "unknown ticket";
    case PERM_ECANCELED: return "cancelled";
    }
    return "unknown status";
}

extern "C" const char *perm_last_error(void) { return g_last_error.c_str(); }

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return permi::fail(PERM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace permi {

// ------------------------------------------------------------ device memory
int ensure(perm_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes <= b.cap) return PERM_OK;
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    want = (want + 4095) & ~(size_t)4095;
    if (ctx->used - b.cap + want > ctx->budget) {
        want = (bytes + 4095) & ~(size_t)4095;
        if (ctx->used - b.cap + want > ctx->budget)
            return fail(PERM_ENOMEM, "need %zu bytes of device scratch, budget %zu (in use %zu)",
                        bytes, ctx->budget, ctx->used);
    }
    if (b.p) {
        // queued work may still read the old buffer
        if (ctx->has_last) HIPCHK(hipEventSynchronize(ctx->last_ev));
        HIPCHK(hipFree(b.p));
        ctx->used -= b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PERM_ENOMEM, "hipMalloc(%zu) failed", want);
    }
    b.p = p;
    b.cap = want;
    ctx->used += want;
    return PERM_OK;
}

static int ensure_pinned(perm_ctx *ctx, size_t bytes)
{
    if (ctx->pinned_busy) {
        HIPCHK(hipEventSynchronize(ctx->pinned_ev));
        ctx->pinned_busy = false;
    }
    if (bytes <= ctx->pinned_cap) return PERM_OK;
    if (ctx->pinned) HIPCHK(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_cap = 0;
    const size_t want = std::max(bytes, (size_t)1 << 20);
    void *p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PERM_ENOMEM, "hipHostMalloc(%zu) failed", want);
    }
    ctx->pinned = p;
    ctx->pinned_cap = want;
    return PERM_OK;
}

// Pinned result slots (at least `bytes`) for calls that return their
// results to the host.  Such calls wait for their kernels before returning,
// so the slots are free at the next call.
static int ensure_host_out(perm_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->host_out_cap) return PERM_OK;
    if (ctx->host_out) HIPCHK(hipHostFree(ctx->host_out));
    ctx->host_out = ctx->host_out_dev = nullptr;
    ctx->host_out_cap = 0;
    const size_t want = std::max(bytes, (size_t)4096);
    void *p = nullptr, *d = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PERM_ENOMEM, "hipHostMalloc(%zu) failed", want);
    }
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(p);
        return fail(PERM_EDEVICE, "hipHostGetDevicePointer failed");
    }
    ctx->host_out = p;
    ctx->host_out_dev = d;
    ctx->host_out_cap = want;
    return PERM_OK;
}

// ------------------------------------------------------------------ tuning
int default_log2_chunk(int variant, int n)
{
    // 64 * 2^c indices per wave item; the partition (and so the summation
    // order of float results) depends on (field, n) only, never on what else
    // is in a batch.  Fitted to a sweep on gfx950 over batches that fill the
    // device (three primes for F_p, 2,000 to 50,000 matrices for floats):
    //  * floats: one item per matrix up to n = 13 (c = n - 7: shorter walks
    //    make the per-lane seed dominate), four items at n = 14, 15 (a
    //    single permanent's latency; one item is up to 13% faster in
    //    batches), two at n = 16, 17, four for n = 18..20 (a block's four
    //    waves then walk one matrix), c = 11 at n = 21, 22 and 10 beyond
    //    (enough items for one large matrix to fill the device);
    //  * F_p: c = n/2 - 5 up to n = 26 and n/2 - 4 (at most 13) from n = 28,
    //    so that the per-lane seed (n^2 work) stays near 1% of the walk with
    //    a few items per resident wave and the host plan stays small, then
    //    n - 27 (2^20 items per matrix at most); at most 20, so that a
    //    lane's sum of 2^c residues stays below 2^52.
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

int log2_chunk_for(const perm_ctx *ctx, int variant, int n)
{
    const int field = variant == V_MONT ? PERM_MODP : variant;
    auto it = ctx->tune.find({field, n});
    if (it != ctx->tune.end() && it->second.log2_chunk > 0) return it->second.log2_chunk;
    return default_log2_chunk(variant, n);
}

// ----------------------------------------------------------------- planner
// Split [x0, x1) into aligned power-of-two blocks and each block into wave
// items of 64 lanes x 2^c indices (smaller blocks: fewer indices per lane or
// fewer lanes).
static void split_range(uint64_t x0, uint64_t x1, int c, uint32_t mat, uint32_t first_slot,
                        std::vector<WaveItem> &items, uint32_t &nparts)
{
    nparts = 0;
    while (x0 < x1) {
        // the largest aligned power-of-two block at x0 that fits in [x0, x1)
        const int fit = 63 - __builtin_clzll(x1 - x0);
        const int e = x0 ? std::min(__builtin_ctzll(x0), fit) : fit;
        const uint64_t B = 1ull << e;
        const uint64_t wave = 64ull << c;
        auto push = [&](uint64_t xs, uint32_t log2L, uint32_t lanes) {
            WaveItem it{};
            it.x0 = xs;
            it.mat = mat;
            it.slot = first_slot + nparts++;
            it.log2L = log2L;
            it.nlanes = lanes;
            items.push_back(it);
        };
        if (B >= wave) {
            for (uint64_t s = 0; s < B; s += wave) push(x0 + s, (uint32_t)c, 64);
        } else if (B >= 64) {
            push(x0, (uint32_t)(e - 6), 64);
        } else {
            push(x0, 0, (uint32_t)B);
        }
        x0 += B;
    }
}

static bool same_input(const MatIn &a, const MatIn &b)
{
    return a.variant == b.variant && a.n == b.n && a.p == b.p && a.src_off == b.src_off &&
           a.out_slot == b.out_slot && a.kahan == b.kahan && a.full == b.full && a.x0 == b.x0 &&
           a.x1 == b.x1 && a.no_scale == b.no_scale && a.out_bytes == b.out_bytes &&
           a.latency == b.latency;
}

static int occupancy(perm_ctx *ctx, const Group &g);

static int occupancy_of(perm_ctx *ctx, int variant, int n, bool kahan)
{
    Group g{};
    g.variant = variant;
    g.n = n;
    g.kahan = kahan;
    g.fused = false;
    return occupancy(ctx, g);
}

// The latency partition.  The default chunk length of (variant, n) is set
// for batches that fill the device; a call with only `nmats` whole matrices
// of that kind may leave most resident waves idle (one c128 matrix of order
// 24 is 128 items on 3,072 resident waves, one of order 14 a single block
// of four waves walking 2^5 indices a lane).  Its time is about
//   ceil(items / slots) x 2^c x step cost + ceil(items / SIMDs) x item cost
// in instruction slots of one SIMD: the walks of a round of `slots` waves
// share the SIMDs' issue, while each wave a SIMD holds adds its seed and
// item overhead (the seeds' loads of the matrix contend for the CU's caches
// and the extra blocks stage the matrix again).  The chunk length minimising
// it (down to 2^3, the shortest the unrolled walk takes) is used, the
// default when that fills the device already.  Only F_p results (exact) and
// single float calls without PERM_SHARED_PARTITION take it: the summation
// order of a float result follows the partition.
int latency_log2_chunk(const perm_ctx *ctx, int variant, int n, uint64_t nmats, int blocks_per_cu)
{
    const int c0 = log2_chunk_for(ctx, variant, n);
    if (n < 10) return c0;        // one item of at most 2^3 indices a lane holds it all
    const int field = variant == V_MONT ? PERM_MODP : variant;
    auto it = ctx->tune.find({field, n});
    if (it != ctx->tune.end() && it->second.log2_chunk > 0) return c0;   // the table decides
    // A round is two waves per SIMD for c128 and F_p: with four independent
    // chains of complex or modular products per lane two waves already issue
    // close to every cycle.  The f64 walk, a third of their instructions per
    // step, needs four (one matrix of order 26: 2^7-index lanes at four waves
    // walked 17% faster than the 2^8 that two waves per SIMD suggest).
    const int per_simd = variant == V_F64 ? 4 : 2;
    const uint64_t slots =
        (uint64_t)std::min(std::max(blocks_per_cu, 1), per_simd) * ctx->num_cus * (BLOCK / WAVE);
    const uint64_t T = 1ull << (n - 1);
    auto items = [&](int c) { return nmats * (T >= (64ull << c) ? T >> (6 + c) : 1ull); };
    if (items(c0) >= slots) return c0;
    // item cost: the seed's instructions -- the wave's common part (about n
    // a lane) and the seven columns whose signs differ across its lanes,
    // each an update of the n row sums (two words each for c128; the
    // Montgomery walk updates for all n - 1 columns) -- and a fixed part for
    // latency and overhead (claim, loads of the descriptors and the matrix,
    // LDS exchange, wave sum), fitted to single calls of orders 10..27 timed
    // at every chunk length: 2^3 fastest up to order 20, then one wave per
    // SIMD (2^4 at 21, 2^5 at 22) rather than two of half the length; the
    // Barrett F_p walk kept one wave per SIMD up to order 24 (2^7; two waves
    // of 2^6 were 2-7% slower from order 22) and two from 25, which takes a
    // fixed part of about 16,000 slots, the float walks about 1,860
    const int upd = variant == V_MONT ? n - 1 : std::min(n - 1, 7);
    const double fixed = variant == V_MODP ? 16000.0 : 1860.0;
    const double item = (double)upd * n * (variant == V_C128 ? 2.0 : 1.0) + n + fixed;
    const double step = (double)step_cost(variant, n);
    const double simds = (double)ctx->num_cus * (BLOCK / WAVE);
    int best = c0;
    double best_t = 1e300;
    for (int c = c0; c >= 3; --c) {
        const double rounds = std::ceil((double)items(c) / (double)slots);
        const double waves = std::ceil((double)items(c) / simds);
        const double t = rounds * std::ldexp(1.0, c) * step + waves * item;
        if (t < 0.98 * best_t) {          // a shorter chunk only when clearly faster
            best_t = t;
            best = c;
        }
    }
    return best;
}

// A call that is one short walk launch of at most this many blocks
// finalizes in its last block instead of in a launch of its own (with more,
// the blocks' device-scope releases cost more than that launch: one U(19)
// in 64 blocks took 0.9 us longer per call).
constexpr int kFinInWalkMaxGrid = 32;

// Plans of at most this many matrices are cached (repeated small calls such
// as a CRT over a few primes); larger ones cost more to compare than to build.
constexpr size_t kPlanCacheMax = 64;

int plan(perm_ctx *ctx, const std::vector<MatIn> &in, Plan &pl)
{
    const bool cacheable = &pl == &ctx->scratch_plan && in.size() <= kPlanCacheMax;
    if (cacheable && ctx->plan_cached && in.size() == ctx->plan_in.size()) {
        bool hit = true;
        for (size_t m = 0; m < in.size() && hit; ++m) hit = same_input(in[m], ctx->plan_in[m]);
        for (size_t q = 0; q < ctx->plan_chunks.size() && hit; ++q) {
            const auto &e = ctx->plan_chunks[q];
            hit = log2_chunk_for(ctx, e.first.first, e.first.second) == e.second;
        }
        for (size_t q = 0; q < ctx->plan_latency.size() && hit; ++q) {
            const auto &e = ctx->plan_latency[q];
            uint64_t cnt = 0;
            for (const MatIn &a : in)
                cnt += a.latency && a.full && a.variant == e.first.first && a.n == e.first.second;
            hit = latency_log2_chunk(ctx, e.first.first, e.first.second, cnt,
                                     occupancy_of(ctx, e.first.first, e.first.second, in[0].kahan)) ==
                  e.second;
        }
        if (hit) return PERM_OK;                 // pl still holds that plan
    }
    ctx->plan_cached = false;
    ctx->plan_id++;
    pl.mats.clear();
    pl.items.clear();
    pl.groups.clear();
    pl.stage_bytes = 0;
    pl.nparts = 0;
    pl.mats.resize(in.size());
    // Group matrices by launch kernel: one specialized (variant, n) kernel,
    // the fused kernel of the smallest order bucket, or several specialized
    // launches when neither fits.
    bool same = true, fusable = true;
    int nmax = 0;
    for (size_t m = 0; m < in.size(); ++m) {
        const MatIn &a = in[m];
        if (a.variant < 0 || a.variant >= V_COUNT || a.n < 0 || a.n > NMAX)
            return fail(PERM_EINVAL, "plan: matrix %zu has variant %d, n = %d", m, a.variant, a.n);
        if (a.variant != in[0].variant || a.n != in[0].n) same = false;
        if (a.variant == V_MONT || a.kahan != in[0].kahan) fusable = false;
        nmax = std::max(nmax, a.n);
    }
    if (nmax > FUSED_BUCKETS[1]) fusable = false;

    std::vector<std::vector<uint32_t>> groups;   // matrix ids per launch
    std::vector<Group> gdesc;
    if (same && !in.empty() && in[0].n > 0) {
        // one specialized launch over every matrix
        std::vector<uint32_t> ids(in.size());
        for (size_t m = 0; m < in.size(); ++m) ids[m] = (uint32_t)m;
        groups.push_back(std::move(ids));
        Group g{};
        g.variant = in[0].variant;
        g.n = in[0].n;
        g.kahan = in[0].kahan;
        g.fused = false;
        gdesc.push_back(g);
    } else if (same || !fusable) {
        std::map<std::pair<int, int>, size_t> gi;
        for (size_t m = 0; m < in.size(); ++m) {
            if (in[m].n == 0) continue;                     // no walk needed
            auto key = std::make_pair(in[m].variant, in[m].n);
            auto it = gi.find(key);
            if (it == gi.end()) {
                gi[key] = groups.size();
                groups.push_back({(uint32_t)m});
                Group g{};
                g.variant = in[m].variant;
                g.n = in[m].n;
                g.kahan = in[m].kahan;
                g.fused = false;
                gdesc.push_back(g);
            } else {
                groups[it->second].push_back((uint32_t)m);
            }
        }
    } else {
        Group g{};
        g.fused = true;
        g.nmax_fused = nmax <= FUSED_BUCKETS[0] ? FUSED_BUCKETS[0] : FUSED_BUCKETS[1];
        g.kahan = in[0].kahan;
        g.variant = -1;
        g.n = nmax;
        std::vector<uint32_t> ids;
        for (size_t m = 0; m < in.size(); ++m)
            if (in[m].n > 0) ids.push_back((uint32_t)m);
        if (!ids.empty()) {
            groups.push_back(ids);
            gdesc.push_back(g);
        }
    }

    // descriptors (all matrices, including n = 0 ones, in input order)
    for (size_t m = 0; m < in.size(); ++m) {
        const MatIn &a = in[m];
        MatDesc &d = pl.mats[m];
        std::memset(&d, 0, sizeof d);
        d.src_off = a.src_off;
        d.stage_off = pl.stage_bytes;
        d.n = a.n;
        d.variant = a.variant;
        d.p = a.p;
        d.flags = (a.kahan ? MD_KAHAN : 0) | (a.no_scale ? MD_NO_SCALE : 0) |
                  (a.out_bytes == 8 ? MD_OUT_8 : 0) | (a.out_bytes == 4 ? MD_OUT_4 : 0);
        d.pinv = a.p ? 1.0 / (double)a.p : 0.0;
        d.mont_pp = (a.variant == V_MONT) ? permh::mont_pprime(a.p) : 0;
        if (a.variant == V_MODP || a.variant == V_MONT)
            d.fin_scale = permh::fp_finalize_factor(a.p, a.n, a.variant == V_MONT, !a.no_scale);
        d.out_slot = a.out_slot;
        if (a.n > 0) pl.stage_bytes += (stage_bytes(a.variant, a.n) + 255) & ~(size_t)255;
    }
    // chunk length per (variant, n), looked up once per call; matrices that
    // may take the latency partition get theirs from the count of whole
    // matrices of their kind in the call
    int chunk[V_COUNT][NMAX + 1];
    for (auto &row : chunk)
        for (int &c : row) c = -1;
    int lchunk[V_COUNT][NMAX + 1];
    {
        uint64_t cnt[V_COUNT][NMAX + 1] = {};
        bool any = false;
        for (const MatIn &a : in)
            if (a.latency && a.full && a.n > 0) { cnt[a.variant][a.n]++; any = true; }
        for (int v = 0; v < V_COUNT; ++v)
            for (int n = 0; n <= NMAX; ++n)
                lchunk[v][n] = (any && cnt[v][n])
                                   ? latency_log2_chunk(ctx, v, n, cnt[v][n],
                                                        occupancy_of(ctx, v, n, in[0].kahan))
                                   : -1;
    }
    auto chunk_of = [&](const MatIn &a) {
        if (a.latency && a.full && lchunk[a.variant][a.n] >= 0) return lchunk[a.variant][a.n];
        int &c = chunk[a.variant][a.n];
        if (c < 0) c = log2_chunk_for(ctx, a.variant, a.n);
        return c;
    };
    // items per group, each group sorted largest first (stable): key =
    // indices per item x cost of a step, so that the waves of a block, which
    // take neighbouring items, finish together in a fused launch of mixed
    // orders.  A whole range splits into items that are all alike, so when
    // every matrix of the group is whole the matrices are ordered instead of
    // the items (the same order, at a fraction of the cost); a matrix's
    // partial slots stay contiguous and in index order either way.
    for (size_t g = 0; g < groups.size(); ++g) {
        Group gd = gdesc[g];
        gd.first_item = (uint32_t)pl.items.size();
        std::vector<WaveItem> &gi = pl.items;            // the group's items are appended
        const size_t g0 = gi.size();
        std::vector<uint32_t> &mats = groups[g];
        bool all_full = true;
        for (uint32_t m : mats) all_full = all_full && in[m].full;
        if (all_full && mats.size() > 1) {
            std::vector<std::pair<uint64_t, uint32_t>> key(mats.size());
            for (size_t q = 0; q < mats.size(); ++q) {
                const MatIn &a = in[mats[q]];
                const int c = chunk_of(a);
                const uint64_t T = 1ull << (a.n - 1);
                key[q] = {std::min<uint64_t>(T, 64ull << c) * step_cost(a.variant, a.n), mats[q]};
            }
            bool sorted = true;
            for (size_t q = 1; q < key.size() && sorted; ++q) sorted = key[q].first <= key[q - 1].first;
            if (!sorted) {
                std::stable_sort(key.begin(), key.end(),
                                 [](const std::pair<uint64_t, uint32_t> &a,
                                    const std::pair<uint64_t, uint32_t> &b) { return a.first > b.first; });
                for (size_t q = 0; q < mats.size(); ++q) mats[q] = key[q].second;
            }
        }
        for (uint32_t m : mats) {
            const MatIn &a = in[m];
            MatDesc &d = pl.mats[m];
            const int c = chunk_of(a);
            const uint64_t T = 1ull << (a.n - 1);
            const uint64_t x0 = a.full ? 0 : a.x0;
            const uint64_t x1 = a.full ? T : a.x1;
            uint32_t np = 0;
            d.first_part = (uint32_t)pl.nparts;
            split_range(x0, x1, c, m, (uint32_t)pl.nparts, gi, np);
            d.num_parts = np;
            pl.nparts += np;
        }
        const size_t cnt = gi.size() - g0;
        auto work = [&](const WaveItem &w) {
            return ((uint64_t)w.nlanes << w.log2L) * step_cost(in[w.mat].variant, in[w.mat].n);
        };
        bool uniform = true;
        if (!all_full)
            for (size_t q = 1; q < cnt && uniform; ++q) uniform = work(gi[g0 + q]) == work(gi[g0]);
        if (!uniform) {
            std::vector<std::pair<uint64_t, uint32_t>> key(cnt);
            for (size_t q = 0; q < cnt; ++q) key[q] = {work(gi[g0 + q]), (uint32_t)q};
            std::stable_sort(key.begin(), key.end(),
                             [](const std::pair<uint64_t, uint32_t> &a,
                                const std::pair<uint64_t, uint32_t> &b) { return a.first > b.first; });
            std::vector<WaveItem> sorted(cnt);
            for (size_t q = 0; q < cnt; ++q) sorted[q] = gi[g0 + key[q].second];
            std::copy(sorted.begin(), sorted.end(), gi.begin() + g0);
        }
        gd.count = (uint32_t)cnt;
        pl.groups.push_back(gd);
    }
    if (cacheable) {
        ctx->plan_in = in;
        ctx->plan_chunks.clear();
        for (int v = 0; v < V_COUNT; ++v)
            for (int n = 0; n <= NMAX; ++n)
                if (chunk[v][n] >= 0) ctx->plan_chunks.push_back({{v, n}, chunk[v][n]});
        ctx->plan_latency.clear();
        for (int v = 0; v < V_COUNT; ++v)
            for (int n = 0; n <= NMAX; ++n)
                if (lchunk[v][n] >= 0) ctx->plan_latency.push_back({{v, n}, lchunk[v][n]});
        ctx->plan_cached = true;
    }
    return PERM_OK;
}

// Blocks per CU for a group's kernel (cached).
static int occupancy(perm_ctx *ctx, const Group &g)
{
    const int key = g.fused ? (1000 + g.nmax_fused * 2 + (g.kahan ? 1 : 0))
                            : (g.variant * 200 + g.n * 2 + (g.kahan ? 1 : 0));
    auto it = ctx->occ.find(key);
    if (it != ctx->occ.end()) return it->second;
    int nb = 1;
    if (walk_occupancy(g.variant, g.n, g.kahan, g.fused, g.nmax_fused, &nb) != 0 || nb < 1) nb = 1;
    ctx->occ[key] = nb;
    return nb;
}

// Order this call after the context's previous call when the stream changes.
int begin_call(perm_ctx *ctx, hipStream_t s)
{
    HIPCHK(hipSetDevice(ctx->device));
    if (ctx->has_last && s != ctx->last_stream) HIPCHK(hipStreamWaitEvent(s, ctx->last_ev, 0));
    return PERM_OK;
}

int end_call(perm_ctx *ctx, hipStream_t s)
{
    HIPCHK(hipEventRecord(ctx->last_ev, s));
    ctx->last_stream = s;
    ctx->has_last = true;
    return PERM_OK;
}

// Check on the host that every descriptor a kernel will dereference stays
// inside its buffer, so that a planning mistake is an error, not a GPU fault.
int validate_plan(const perm_ctx *ctx, const Plan &pl, size_t out_slots)
{
    const size_t nm = pl.mats.size();
    for (size_t m = 0; m < nm; ++m) {
        const MatDesc &d = pl.mats[m];
        if (d.n < 0 || d.n > NMAX || d.variant < 0 || d.variant >= V_COUNT)
            return fail(PERM_EINVAL, "plan: bad matrix %zu", m);
        if (d.n > 0 && d.stage_off + stage_bytes(d.variant, d.n) > ctx->stage.cap)
            return fail(PERM_EINVAL, "plan: staged matrix %zu outside the stage buffer", m);
        if ((size_t)d.first_part + d.num_parts > pl.nparts || pl.nparts * 16 > ctx->partials.cap)
            return fail(PERM_EINVAL, "plan: partial slots of matrix %zu out of range", m);
        if (d.out_slot >= out_slots) return fail(PERM_EINVAL, "plan: output slot of matrix %zu", m);
        if ((d.variant == V_MODP || d.variant == V_MONT) && !(d.p & 1u))
            return fail(PERM_EINVAL, "plan: even modulus");
    }
    for (const Group &g : pl.groups)
        if ((size_t)g.first_item + g.count > pl.items.size())
            return fail(PERM_EINVAL, "plan: launch group out of range");
    for (size_t i = 0; i < pl.items.size(); ++i) {
        const WaveItem &it = pl.items[i];
        if (it.mat >= nm) return fail(PERM_EINVAL, "plan: item %zu names matrix %u", i, it.mat);
        const MatDesc &d = pl.mats[it.mat];
        if (d.n < 1 || it.slot < d.first_part || it.slot >= d.first_part + d.num_parts)
            return fail(PERM_EINVAL, "plan: item %zu slot out of its matrix's range", i);
        if (it.nlanes < 1 || it.nlanes > 64 || it.log2L > 24 || (it.x0 & ((1ull << it.log2L) - 1)))
            return fail(PERM_EINVAL, "plan: item %zu has a bad shape", i);
        const uint64_t end = it.x0 + ((uint64_t)it.nlanes << it.log2L);
        if (end > (1ull << (d.n - 1)))
            return fail(PERM_EINVAL, "plan: item %zu runs past 2^(n-1)", i);
        if ((d.variant == V_MODP) && it.log2L > 20)
            return fail(PERM_EINVAL, "plan: F_p chunk longer than 2^20");
    }
    return PERM_OK;
}

// Upload the plan, stage, walk, finalize.  `src` holds the matrices (device),
// `out` receives 16-byte result slots (device).
int execute(perm_ctx *ctx, Plan &pl, const void *src, void *out, size_t out_slots, hipStream_t s)
{
    const size_t mb = pl.mats.size() * sizeof(MatDesc);
    const size_t ib = pl.items.size() * sizeof(WaveItem);
    int rc;
    if ((rc = ensure(ctx, ctx->plan_buf, mb + ib + 64)) != PERM_OK) return rc;
    if ((rc = ensure(ctx, ctx->stage, std::max<size_t>(pl.stage_bytes, 256))) != PERM_OK) return rc;
    if ((rc = ensure(ctx, ctx->partials, std::max<size_t>(pl.nparts, 1) * 16)) != PERM_OK) return rc;
    if ((rc = validate_plan(ctx, pl, out_slots)) != PERM_OK) return rc;
    // upload unless plan_buf already holds this plan (a repeated call)
    if (&pl != &ctx->scratch_plan || ctx->uploaded_plan_id != ctx->plan_id ||
        ctx->uploaded_ptr != ctx->plan_buf.p) {
        if ((rc = ensure_pinned(ctx, mb + ib)) != PERM_OK) return rc;
        std::memcpy(ctx->pinned, pl.mats.data(), mb);
        if (ib) std::memcpy((char *)ctx->pinned + mb, pl.items.data(), ib);
        HIPCHK(hipMemcpyAsync(ctx->plan_buf.p, ctx->pinned, mb + ib, hipMemcpyHostToDevice, s));
        HIPCHK(hipEventRecord(ctx->pinned_ev, s));
        ctx->pinned_busy = true;
        ctx->uploaded_plan_id = &pl == &ctx->scratch_plan ? ctx->plan_id : ~0ull;
        ctx->uploaded_ptr = ctx->plan_buf.p;
    }
    const MatDesc *d_mats = (const MatDesc *)ctx->plan_buf.p;
    const WaveItem *d_items = (const WaveItem *)((char *)ctx->plan_buf.p + mb);

    // launch shape per group: several items per claim only when there are
    // many more items than resident waves (a short launch keeps one item
    // per wave); grid = resident blocks, or fewer for a short launch
    std::vector<LaunchShape> &shape = ctx->scratch_shape;
    shape.assign(pl.groups.size(), LaunchShape{0, 0});
    int walks = 0, last = -1;
    for (size_t q = 0; q < pl.groups.size(); ++q) {
        const Group &g = pl.groups[q];
        if (!g.count) continue;
        const int occ = occupancy(ctx, g);
        const int per_cu = ctx->grid_per_cu > 0 ? std::min(ctx->grid_per_cu, occ) : occ;
        uint32_t max_l2 = 0;
        for (uint32_t i = 0; i < g.count; ++i) max_l2 = std::max(max_l2, pl.items[g.first_item + i].log2L);
        const uint32_t resident = (uint32_t)(per_cu * ctx->num_cus * (BLOCK / WAVE));
        const uint32_t grab = std::max(1u, std::min(grab_for(max_l2), g.count / (2 * resident)));
        const uint32_t runs = (g.count + grab * (BLOCK / WAVE) - 1) / (grab * (BLOCK / WAVE));
        shape[q] = LaunchShape{grab, (int)std::max(1u, std::min(runs, (uint32_t)(per_cu * ctx->num_cus)))};
        ++walks;
        last = (int)q;
    }
    // A call that is one walk of one block stages and finalizes in that
    // block.  A short walk (at most 2^26 terms, about 0.2 ms) over a few
    // small matrices -- a single permanent of order up to 27 -- stages them
    // in every block instead of in a launch of its own: such calls are
    // bound by the host's launches, which cost more than the blocks' copies
    // of at most 16 entries per thread cost the device (one U(16)..U(20) or
    // O(20) per call 11-14% faster).  With at most kFinInWalkMaxGrid blocks
    // the last block to finish also finalizes (one launch per call).
    size_t entries = 0;
    uint64_t terms = 0;
    for (const MatDesc &d : pl.mats) {
        entries += (size_t)d.n * d.n;
        terms += d.n > 0 ? 1ull << (d.n - 1) : 0;
    }
    const bool block_stage = walks == 1 && (shape[last].grid == 1 ||
                                            (pl.mats.size() <= 4 && entries <= 16 * BLOCK &&
                                             terms <= (1ull << 26)));
    const bool fin_in_walk = block_stage && shape[last].grid <= kFinInWalkMaxGrid;
    if (!block_stage)
        HIPCHK((hipError_t)launch_stage(d_mats, (int)pl.mats.size(), src, ctx->stage.p, s));
    for (size_t q = 0; q < pl.groups.size(); ++q) {
        const Group &g = pl.groups[q];
        if (!g.count) continue;
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        bool prof = false;
        {
            std::lock_guard<std::mutex> lk(ctx->prof_mu);
            if (ctx->prof_on && !ctx->prof_pool.empty()) {
                ev = ctx->prof_pool.back();
                ctx->prof_pool.pop_back();
                prof = true;
            }
        }
        if (ctx->prof_on && !prof) {          // pool used up: one more pair
            HIPCHK(hipEventCreate(&ev.first));
            if (hipEventCreate(&ev.second) != hipSuccess) {
                (void)hipEventDestroy(ev.first);
                return fail(PERM_EDEVICE, "hipEventCreate failed");
            }
            prof = true;
        }
        if (prof) HIPCHK(hipEventRecord(ev.first, s));
        HIPCHK((hipError_t)launch_walk(g.variant, g.n, g.kahan, g.fused, g.nmax_fused,
                                       d_items + g.first_item, g.count, shape[q].grab, d_mats,
                                       ctx->stage.p, (double *)ctx->partials.p,
                                       (unsigned long long *)ctx->ctr.p, &ctx->ctr_state,
                                       shape[q].grid, s, block_stage ? src : nullptr,
                                       fin_in_walk ? out : nullptr,
                                       block_stage ? (int)pl.mats.size() : 0));
        if (prof) {
            HIPCHK(hipEventRecord(ev.second, s));
            std::lock_guard<std::mutex> lk(ctx->prof_mu);
            ctx->prof_pending.push_back(ev);
        }
    }
    if (!fin_in_walk)
        HIPCHK((hipError_t)launch_finalize(d_mats, (int)pl.mats.size(),
                                           (const double *)ctx->partials.p, out, s));
    return PERM_OK;
}

}  // namespace permi

using namespace permi;

// ----------------------------------------------------------------- context
extern "C" int perm_ctx_create(int device, size_t hbm_budget, perm_ctx **out)
{
    if (!out) return fail(PERM_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return fail(PERM_EDEVICE, "no HIP device available");
    }
    if (device < 0 || device >= ndev) return fail(PERM_EDEVICE, "device %d out of range", device);
    HIPCHK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    perm_ctx *c = new (std::nothrow) perm_ctx();
    if (!c) return fail(PERM_ENOMEM, "host allocation failed");
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    c->budget = hbm_budget ? hbm_budget : prop.totalGlobalMem / 4;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->last_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->pinned_ev, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return fail(PERM_EDEVICE, "stream/event creation failed");
    }
    int rc = ensure(c, c->ctr, CTR_BYTES);
    if (rc != PERM_OK) { perm_ctx_destroy(c); return rc; }
    // kernels run on non-blocking streams, which do not order after the null
    // stream: the counter is zero before the first launch by waiting here
    if (hipMemset(c->ctr.p, 0, CTR_BYTES) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
        perm_ctx_destroy(c);
        return fail(PERM_EDEVICE, "counter init failed");
    }
    c->ctr_state = CtrState{};
    // the static scratch of perm_c128_noalloc: its device address on this
    // device (the device is current here)
    const int se = noalloc_scratch_init(device, &c->noalloc_ptr);
    if (se != (int)hipSuccess) {
        perm_ctx_destroy(c);
        return fail(PERM_EDEVICE, "static scratch lookup failed on device %d: %s", device,
                    hipGetErrorString((hipError_t)se));
    }
    *out = c;
    return PERM_OK;
}

extern "C" void perm_ctx_destroy(perm_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->has_last) (void)hipEventSynchronize(c->last_ev);
    for (DevBuf *b : {&c->src, &c->stage, &c->partials, &c->outs, &c->plan_buf, &c->ctr})
        if (b->p) (void)hipFree(b->p);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->host_out) (void)hipHostFree(c->host_out);
    for (auto *v : {&c->prof_pending, &c->prof_pool})
        for (auto &e : *v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    if (c->last_ev) (void)hipEventDestroy(c->last_ev);
    if (c->pinned_ev) (void)hipEventDestroy(c->pinned_ev);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// ---------------------------------------------------------- argument checks
static bool modulus_ok(uint32_t p) { return p >= 3 && (p & 1u) && p < (1u << 31); }

int permi::variant_of(int field, unsigned flags)
{
    switch (field) {
    case PERM_C128: return V_C128;
    case PERM_F64: return V_F64;
    case PERM_MODP: return (flags & PERM_MONTGOMERY) ? V_MONT : V_MODP;
    }
    return -1;
}

// Bring the matrices to the device: returns the device pointer to use as the
// staging source.
int permi::source_on_device(perm_ctx *ctx, const void *data, size_t bytes, unsigned flags,
                            hipStream_t s, const void **dev)
{
    if (flags & PERM_DEVICE_PTRS) {
        *dev = data;
        return PERM_OK;
    }
    int rc = ensure(ctx, ctx->src, std::max<size_t>(bytes, 256));
    if (rc != PERM_OK) return rc;
    if (bytes) HIPCHK(hipMemcpyAsync(ctx->src.p, data, bytes, hipMemcpyHostToDevice, s));
    *dev = ctx->src.p;
    return PERM_OK;
}

// One matrix, one result slot of `out_bytes` copied to `out`.
static int single(perm_ctx *ctx, int variant, const void *A, int n, uint32_t p, void *out,
                  size_t out_bytes, unsigned flags, void *stream)
{
    if (!ctx) return fail(PERM_EINVAL, "ctx is NULL");
    if (n < 0 || n > PERM_NMAX) return fail(PERM_EINVAL, "n = %d outside [0, %d]", n, PERM_NMAX);
    if (!out || (n > 0 && !A)) return fail(PERM_EINVAL, "NULL matrix or output pointer");
    hipStream_t s = (hipStream_t)stream;
    int rc = begin_call(ctx, s);
    if (rc != PERM_OK) return rc;
    const void *src = nullptr;
    const size_t bytes = (size_t)n * n * src_entry_bytes(variant);
    if ((rc = source_on_device(ctx, A, bytes, flags, s, &src)) != PERM_OK) return rc;
    std::vector<MatIn> in(1);
    in[0].variant = variant;
    in[0].n = n;
    in[0].p = p;
    in[0].kahan = !(flags & PERM_NO_KAHAN);
    in[0].full = true;
    in[0].latency = variant == V_MODP || variant == V_MONT || !(flags & PERM_SHARED_PARTITION);
    // A device output with the alignment of its element type receives the
    // result straight from the finalize step (only out_bytes written), with
    // no copy launch; otherwise the 16-byte slot goes through ctx->outs.
    const bool direct = (flags & PERM_DEVICE_PTRS) &&
                        (uintptr_t)out % (out_bytes >= 8 ? 8 : 4) == 0;
    in[0].out_bytes = direct ? (int)out_bytes : 16;
    Plan &pl = ctx->scratch_plan;
    if ((rc = plan(ctx, in, pl)) != PERM_OK) return rc;
    if (direct) {
        if ((rc = execute(ctx, pl, src, out, 1, s)) != PERM_OK) return rc;
        return end_call(ctx, s);
    }
    if (!(flags & PERM_DEVICE_PTRS)) {
        // a host output: the finalize step writes the slot in pinned host
        // memory (free here: the previous such call waited for its kernels)
        if ((rc = ensure_host_out(ctx, 16)) != PERM_OK) return rc;
        if ((rc = execute(ctx, pl, src, ctx->host_out_dev, 1, s)) != PERM_OK) return rc;
        if ((rc = end_call(ctx, s)) != PERM_OK) return rc;
        HIPCHK(hipStreamSynchronize(s));
        std::memcpy(out, ctx->host_out, out_bytes);
        return PERM_OK;
    }
    if ((rc = ensure(ctx, ctx->outs, 256)) != PERM_OK) return rc;
    if ((rc = execute(ctx, pl, src, ctx->outs.p, 1, s)) != PERM_OK) return rc;
    HIPCHK(hipMemcpyAsync(out, ctx->outs.p, out_bytes, hipMemcpyDeviceToDevice, s));
    return end_call(ctx, s);
}

extern "C" int perm_c128(perm_ctx *ctx, const double *A, int n, double *out, unsigned flags,
                         void *stream)
{
    return single(ctx, V_C128, A, n, 0, out, 16, flags, stream);
}

extern "C" int perm_f64(perm_ctx *ctx, const double *A, int n, double *out, unsigned flags,
                        void *stream)
{
    return single(ctx, V_F64, A, n, 0, out, 8, flags, stream);
}

extern "C" int perm_modp(perm_ctx *ctx, const uint32_t *A, int n, uint32_t p, uint32_t *out,
                         unsigned flags, void *stream)
{
    if (!modulus_ok(p)) return fail(PERM_EINVAL, "modulus %u must be odd with 3 <= p < 2^31", p);
    return single(ctx, variant_of(PERM_MODP, flags), A, n, p, out, 4, flags, stream);
}

// ------------------------------------------------------ no-allocation c128
// perm_c128 for callers that cannot allocate: device pointers only, every
// byte of device scratch in the static array of noalloc.hip, the partition
// written there by a kernel.  The partition and launch shape are those
// plan() and execute() give one whole c128 matrix, so the result has
// perm_c128's bits.  No host heap allocation either.
extern "C" int perm_c128_noalloc(perm_ctx *ctx, const double *A, int n, double *out,
                                 unsigned flags, void *stream)
{
    if (!ctx) return fail(PERM_EINVAL, "ctx is NULL");
    if (!(flags & PERM_DEVICE_PTRS))
        return fail(PERM_EINVAL, "perm_c128_noalloc takes device pointers only (PERM_DEVICE_PTRS)");
    if (flags & ~(PERM_DEVICE_PTRS | PERM_NO_KAHAN | PERM_SHARED_PARTITION))
        return fail(PERM_EINVAL, "perm_c128_noalloc: unsupported flags 0x%x", flags);
    if (n < 0 || n > NOALLOC_NMAX)
        return fail(PERM_EINVAL, "n = %d outside [0, %d], the orders of the no-allocation call", n,
                    NOALLOC_NMAX);
    if (!out || (n > 0 && !A)) return fail(PERM_EINVAL, "NULL matrix or output pointer");
    if ((uintptr_t)out % 8 || (uintptr_t)A % 8)
        return fail(PERM_EINVAL, "matrix and output must be 8-byte aligned");
    if (!ctx->noalloc_ptr) return fail(PERM_EDEVICE, "no static scratch on device %d", ctx->device);
    const bool kahan = !(flags & PERM_NO_KAHAN);
    // split_range over the whole of [0, 2^(n-1)): equal items of 64 lanes x
    // 2^c indices, or one item of fewer indices for a short range
    uint64_t count = 0;
    uint32_t log2L = 0, nlanes = 0;
    // occupancy from the context's cache when it has it (no insertion: the
    // call allocates nothing, host memory included)
    int occ = 0;
    if (n > 0) {
        const int key = V_C128 * 200 + n * 2 + (kahan ? 1 : 0);
        auto it = ctx->occ.find(key);
        if (it != ctx->occ.end()) occ = it->second;
        else if (walk_occupancy(V_C128, n, kahan, false, 0, &occ) != 0 || occ < 1) occ = 1;
    }
    if (n > 0) {
        // the chunk length perm_c128 uses for the same flags
        const int c = (flags & PERM_SHARED_PARTITION) ? log2_chunk_for(ctx, V_C128, n)
                                                      : latency_log2_chunk(ctx, V_C128, n, 1, occ);
        const uint64_t T = 1ull << (n - 1);
        const uint64_t W = 64ull << c;
        if (T >= W) {
            count = T / W;
            log2L = (uint32_t)c;
            nlanes = 64;
        } else if (T >= 64) {
            count = 1;
            log2L = (uint32_t)(n - 7);
            nlanes = 64;
        } else {
            count = 1;
            nlanes = (uint32_t)T;
        }
    }
    NoallocLayout L{};
    if (count > (1u << 20) || noalloc_layout(n, (uint32_t)count, &L) != 0)
        return fail(PERM_ENOMEM,
                    "order %d in %llu wave items needs more than the %zu bytes of static scratch",
                    n, (unsigned long long)count, NOALLOC_SCRATCH_BYTES);
    hipStream_t s = (hipStream_t)stream;
    int rc = begin_call(ctx, s);
    if (rc != PERM_OK) return rc;
    char *base = (char *)ctx->noalloc_ptr;
    HIPCHK((hipError_t)launch_noalloc_plan(base, &L, (uint32_t)count, n, log2L, nlanes,
                                           kahan ? MD_KAHAN : 0u, out, s));
    if (n > 0) {
        // launch shape as execute() picks it for this one group
        const int per_cu = ctx->grid_per_cu > 0 ? std::min(ctx->grid_per_cu, occ) : occ;
        const uint32_t cnt = (uint32_t)count;
        const uint32_t resident = (uint32_t)(per_cu * ctx->num_cus * (BLOCK / WAVE));
        const uint32_t grab = std::max(1u, std::min(grab_for(log2L), cnt / (2 * resident)));
        const uint32_t runs = (cnt + grab * (BLOCK / WAVE) - 1) / (grab * (BLOCK / WAVE));
        const int grid = (int)std::max(1u, std::min(runs, (uint32_t)(per_cu * ctx->num_cus)));
        const bool fin_in_walk = grid <= kFinInWalkMaxGrid;
        const MatDesc *d_mats = (const MatDesc *)(base + L.mat);
        void *stage = base + L.stage;
        double *partials = (double *)(base + L.partials);
        // every block stages the matrix (at most 32 x 32 entries)
        CtrState st{};                      // the plan kernel zeroed the counters
        HIPCHK((hipError_t)launch_walk(V_C128, n, kahan, false, 0,
                                       (const WaveItem *)(base + L.items), cnt, grab, d_mats, stage,
                                       partials, (unsigned long long *)(base + L.ctr), &st, grid, s,
                                       A, fin_in_walk ? out : nullptr, 1));
        if (!fin_in_walk) HIPCHK((hipError_t)launch_finalize(d_mats, 1, partials, out, s));
    }
    return end_call(ctx, s);
}

// ------------------------------------------------------------------- batch
static int check_item(const perm_item &it, uint64_t data_addr)
{
    if (it.n < 0 || it.n > PERM_NMAX) return fail(PERM_EINVAL, "n = %d outside [0, %d]", it.n, PERM_NMAX);
    if (it.field != PERM_C128 && it.field != PERM_F64 && it.field != PERM_MODP)
        return fail(PERM_EINVAL, "unknown field %d", it.field);
    if (it.field == PERM_MODP && !modulus_ok(it.p))
        return fail(PERM_EINVAL, "modulus %u must be odd with 3 <= p < 2^31", it.p);
    if (it.reserved != 0) return fail(PERM_EINVAL, "reserved field must be 0");
    const uint64_t align = it.field == PERM_MODP ? 4 : 8;
    if ((data_addr + it.offset) % align)
        return fail(PERM_EINVAL, "matrix at offset %llu is not %llu-byte aligned",
                    (unsigned long long)it.offset, (unsigned long long)align);
    return PERM_OK;
}

extern "C" int perm_batch(perm_ctx *ctx, const perm_item *items, int count, const void *data,
                          void *out, int *bad_index, unsigned flags, void *stream)
{
    if (bad_index) *bad_index = -1;
    if (!ctx) return fail(PERM_EINVAL, "ctx is NULL");
    if (count < 0 || (count > 0 && (!items || !out))) return fail(PERM_EINVAL, "bad count or NULL pointer");
    if (count == 0) return PERM_OK;
    uint64_t span = 0;
    bool any_data = false;
    for (int i = 0; i < count; ++i) {
        int rc = check_item(items[i], (uint64_t)(uintptr_t)data);
        if (rc != PERM_OK) {
            if (bad_index) *bad_index = i;
            return rc;
        }
        const uint64_t bytes = (uint64_t)items[i].n * items[i].n *
                               src_entry_bytes(variant_of(items[i].field, flags));
        if (bytes) any_data = true;
        span = std::max(span, items[i].offset + bytes);
    }
    if (any_data && !data) return fail(PERM_EINVAL, "data is NULL");
    hipStream_t s = (hipStream_t)stream;
    int rc = begin_call(ctx, s);
    if (rc != PERM_OK) return rc;
    const void *src = nullptr;
    if ((rc = source_on_device(ctx, data, span, flags, s, &src)) != PERM_OK) return rc;
    std::vector<MatIn> &in = ctx->scratch_in;
    in.assign(count, MatIn{});
    for (int i = 0; i < count; ++i) {
        in[i].variant = variant_of(items[i].field, flags);
        in[i].n = items[i].n;
        in[i].p = items[i].field == PERM_MODP ? items[i].p : 0;
        in[i].src_off = items[i].offset;
        in[i].out_slot = (uint32_t)i;
        in[i].kahan = !(flags & PERM_NO_KAHAN);
        in[i].full = true;
        in[i].latency = items[i].field == PERM_MODP;   // exact whatever the partition
    }
    Plan &pl = ctx->scratch_plan;
    if ((rc = plan(ctx, in, pl)) != PERM_OK) return rc;
    void *dout = out;
    if (!(flags & PERM_DEVICE_PTRS)) {
        if ((rc = ensure(ctx, ctx->outs, (size_t)count * 16)) != PERM_OK) return rc;
        dout = ctx->outs.p;
    }
    if ((rc = execute(ctx, pl, src, dout, (size_t)count, s)) != PERM_OK) return rc;
    if (flags & PERM_DEVICE_PTRS) return end_call(ctx, s);
    HIPCHK(hipMemcpyAsync(out, dout, (size_t)count * 16, hipMemcpyDeviceToHost, s));
    if ((rc = end_call(ctx, s)) != PERM_OK) return rc;
    HIPCHK(hipStreamSynchronize(s));
    return PERM_OK;
}

// ------------------------------------------------------------------- range
extern "C" int perm_range(perm_ctx *ctx, const perm_item *item, const void *data, uint64_t x0,
                          uint64_t x1, void *out16, unsigned flags, void *stream)
{
    if (!ctx || !item || !out16) return fail(PERM_EINVAL, "NULL argument");
    int rc = check_item(*item, (uint64_t)(uintptr_t)data);
    if (rc != PERM_OK) return rc;
    if (item->n < 1) return fail(PERM_EINVAL, "range needs n >= 1");
    const uint64_t T = 1ull << (item->n - 1);
    if (x0 > x1 || x1 > T) return fail(PERM_EINVAL, "range [%llu, %llu) outside [0, 2^%d)",
                                       (unsigned long long)x0, (unsigned long long)x1, item->n - 1);
    if (!data) return fail(PERM_EINVAL, "data is NULL");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = begin_call(ctx, s)) != PERM_OK) return rc;
    const int variant = variant_of(item->field, flags);
    const uint64_t bytes = (uint64_t)item->n * item->n * src_entry_bytes(variant);
    const void *src = nullptr;
    if (flags & PERM_DEVICE_PTRS) src = (const char *)data + item->offset;
    else if ((rc = source_on_device(ctx, (const char *)data + item->offset, bytes, flags, s, &src)) != PERM_OK)
        return rc;
    std::vector<MatIn> in(1);
    in[0].variant = variant;
    in[0].n = item->n;
    in[0].p = item->field == PERM_MODP ? item->p : 0;
    in[0].kahan = !(flags & PERM_NO_KAHAN);
    in[0].full = false;
    in[0].x0 = x0;
    in[0].x1 = x1;
    in[0].no_scale = true;
    Plan &pl = ctx->scratch_plan;
    if ((rc = plan(ctx, in, pl)) != PERM_OK) return rc;
    if ((rc = ensure(ctx, ctx->outs, 256)) != PERM_OK) return rc;
    if (x0 == x1) {
        // empty range: the sum is zero; finalize writes zero for num_parts = 0
        // only when n = 0, so fill the slot on the device
        HIPCHK(hipMemsetAsync(ctx->outs.p, 0, 16, s));
    } else if ((rc = execute(ctx, pl, src, ctx->outs.p, 1, s)) != PERM_OK) {
        return rc;
    }
    HIPCHK(hipMemcpyAsync(out16, ctx->outs.p, 16, hipMemcpyDeviceToHost, s));
    if ((rc = end_call(ctx, s)) != PERM_OK) return rc;
    HIPCHK(hipStreamSynchronize(s));
    return PERM_OK;
}

// --------------------------------------------------------------------- CRT
int permi::write_limbs(const permh::BigU &mag, int sgn, uint64_t *limbs, int max_limbs,
                       int *nlimbs, int *sign)
{
    if ((int)mag.limb.size() > max_limbs)
        return fail(PERM_ERANGE, "result needs %zu limbs, max_limbs = %d", mag.limb.size(), max_limbs);
    for (size_t i = 0; i < mag.limb.size(); ++i) limbs[i] = mag.limb[i];
    *nlimbs = (int)mag.limb.size();
    *sign = sgn;
    return PERM_OK;
}

int permi::check_primes(const uint32_t *primes, int k, double log2_bound)
{
    if (!primes || k < 1) return fail(PERM_EINVAL, "need k >= 1 primes");
    for (int i = 0; i < k; ++i) {
        if (!modulus_ok(primes[i]) || !permh::is_prime_u32(primes[i]))
            return fail(PERM_EINVAL, "modulus %u is not an odd prime below 2^31", primes[i]);
        for (int j = 0; j < i; ++j)
            if (primes[j] == primes[i]) return fail(PERM_EINVAL, "duplicate prime %u", primes[i]);
    }
    if (!(log2_bound >= 0.0) || !std::isfinite(log2_bound))
        return fail(PERM_EINVAL, "log2_bound must be finite and >= 0");
    // M > 2^(bound + 1), with a safety margin for the float sum of logs
    if (permh::log2_product(primes, k) <= log2_bound + 1.0 + 1e-9)
        return fail(PERM_ERANGE, "product of the primes (2^%.3f) does not exceed 2^(%.3f + 1)",
                    permh::log2_product(primes, k), log2_bound);
    return PERM_OK;
}

extern "C" int perm_crt_lift(const uint32_t *residues, const uint32_t *primes, int k,
                             double log2_bound, uint64_t *limbs, int max_limbs, int *nlimbs,
                             int *sign)
{
    if (!residues || !limbs || !nlimbs || !sign) return fail(PERM_EINVAL, "NULL argument");
    int rc = check_primes(primes, k, log2_bound);
    if (rc != PERM_OK) return rc;
    permh::BigU mag;
    int sg = 0;
    if (!permh::garner_lift(residues, primes, k, mag, sg)) return fail(PERM_EINVAL, "lift failed");
    return write_limbs(mag, sg, limbs, max_limbs, nlimbs, sign);
}

// log2 of a nonzero multi-limb magnitude (to about 1e-15 relative).
static double log2_big(const permh::BigU &m)
{
    const size_t L = m.limb.size();
    double top = (double)m.limb[L - 1];
    if (L >= 2) top += std::ldexp((double)m.limb[L - 2], -64);
    return std::log2(top) + 64.0 * (double)(L - 1);
}

extern "C" int perm_crt_check(const uint32_t *residues, const uint32_t *primes, int k,
                              double log2_bound, uint64_t *limbs, int max_limbs, int *nlimbs,
                              int *sign, int *bad)
{
    if (!residues || !limbs || !nlimbs || !sign || !bad) return fail(PERM_EINVAL, "NULL argument");
    int rc = check_primes(primes, k, log2_bound);
    if (rc != PERM_OK) return rc;
    if (k < 2) return fail(PERM_ERANGE, "a redundancy check needs at least two primes");
    std::vector<uint32_t> r(residues, residues + k), p(primes, primes + k);
    // every leave-one-out subset must still determine the integer
    for (int j = 0; j < k; ++j) {
        const double l = permh::log2_product(primes, k) - std::log2((double)primes[j]);
        if (l <= log2_bound + 1.0 + 1e-9)
            return fail(PERM_ERANGE, "without prime %u the product 2^%.3f does not exceed "
                        "2^(%.3f + 1): no redundant prime", primes[j], l, log2_bound);
    }
    permh::BigU all_m, m;
    int all_s = 0, sg = 0;
    if (!permh::garner_lift(r.data(), p.data(), k, all_m, all_s)) return fail(PERM_EINVAL, "lift failed");
    std::vector<permh::BigU> lm(k);
    std::vector<int> ls(k);
    bool agree = true;
    for (int j = 0; j < k; ++j) {
        std::vector<uint32_t> rj, pj;
        for (int i = 0; i < k; ++i)
            if (i != j) { rj.push_back(r[i]); pj.push_back(p[i]); }
        if (!permh::garner_lift(rj.data(), pj.data(), k - 1, lm[j], ls[j]))
            return fail(PERM_EINVAL, "lift failed");
        agree = agree && ls[j] == all_s && permh::BigU::cmp(lm[j], all_m) == 0;
    }
    if (agree) {
        *bad = -1;
        return write_limbs(all_m, all_s, limbs, max_limbs, nlimbs, sign);
    }
    // one corrupted residue: only the lift that leaves it out is within the bound
    int cand = -1, ncand = 0;
    for (int j = 0; j < k; ++j)
        if (ls[j] == 0 || log2_big(lm[j]) <= log2_bound) { cand = j; ++ncand; }
    if (ncand != 1)
        return fail(PERM_ERANGE, "residues inconsistent: %d leave-one-out lifts fall within the "
                    "bound, so no single residue can be named", ncand);
    *bad = cand;
    return write_limbs(lm[cand], ls[cand], limbs, max_limbs, nlimbs, sign);
}

extern "C" int perm_crt_int(perm_ctx *ctx, const uint32_t *mats, const uint32_t *primes, int k,
                            int n, double log2_bound, uint64_t *limbs, int max_limbs, int *nlimbs,
                            int *sign, uint32_t *residues_out, unsigned flags, void *stream)
{
    if (!ctx || !limbs || !nlimbs || !sign) return fail(PERM_EINVAL, "NULL argument");
    if (n < 0 || n > PERM_NMAX) return fail(PERM_EINVAL, "n = %d outside [0, %d]", n, PERM_NMAX);
    if (n > 0 && !mats) return fail(PERM_EINVAL, "mats is NULL");
    int rc = check_primes(primes, k, log2_bound);
    if (rc != PERM_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = begin_call(ctx, s)) != PERM_OK) return rc;
    const int variant = variant_of(PERM_MODP, flags);
    const size_t per = (size_t)n * n * 4;
    const void *src = nullptr;
    if ((rc = source_on_device(ctx, mats, per * k, flags, s, &src)) != PERM_OK) return rc;
    std::vector<MatIn> &in = ctx->scratch_in;
    in.assign(k, MatIn{});
    for (int i = 0; i < k; ++i) {
        in[i].variant = variant;
        in[i].n = n;
        in[i].p = primes[i];
        in[i].src_off = per * i;
        in[i].out_slot = (uint32_t)i;
        in[i].full = true;
        in[i].latency = true;              // exact: any partition gives the same residues
    }
    Plan &pl = ctx->scratch_plan;
    if ((rc = plan(ctx, in, pl)) != PERM_OK) return rc;
    // the residues' slots in pinned host memory, written by the finalize step
    if ((rc = ensure_host_out(ctx, (size_t)k * 16)) != PERM_OK) return rc;
    if ((rc = execute(ctx, pl, src, ctx->host_out_dev, (size_t)k, s)) != PERM_OK) return rc;
    if ((rc = end_call(ctx, s)) != PERM_OK) return rc;
    HIPCHK(hipStreamSynchronize(s));
    const uint32_t *slots = (const uint32_t *)ctx->host_out;
    std::vector<uint32_t> res(k);
    for (int i = 0; i < k; ++i) res[i] = slots[4 * (size_t)i];
    permh::BigU mag;
    int sg = 0;
    if (!permh::garner_lift(res.data(), primes, k, mag, sg)) return fail(PERM_EINVAL, "lift failed");
    if ((rc = write_limbs(mag, sg, limbs, max_limbs, nlimbs, sign)) != PERM_OK) return rc;
    if (residues_out) std::memcpy(residues_out, res.data(), (size_t)k * 4);
    return PERM_OK;
}

// --------------------------------------------------------------- profiling
extern "C" int perm_prof_enable(perm_ctx *ctx, int on)
{
    if (!ctx) return fail(PERM_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    if (on) {
        // event pairs for the next max(256, on) launches, created here
        // rather than inside timed calls
        HIPCHK(hipSetDevice(ctx->device));
        const size_t want = std::max(256, std::min(on, 1 << 16));
        while (ctx->prof_pool.size() + ctx->prof_pending.size() < want) {
            std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
            HIPCHK(hipEventCreate(&ev.first));
            if (hipEventCreate(&ev.second) != hipSuccess) {
                hipEventDestroy(ev.first);
                return fail(PERM_EDEVICE, "hipEventCreate failed");
            }
            ctx->prof_pool.push_back(ev);
        }
    }
    ctx->prof_on = on != 0;
    return PERM_OK;
}

extern "C" int perm_prof_read(perm_ctx *ctx, double *walk_ms, uint64_t *launches)
{
    if (!ctx || !walk_ms || !launches) return fail(PERM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    HIPCHK(hipSetDevice(ctx->device));
    double tot = 0.0;
    for (auto &e : ctx->prof_pending) {
        HIPCHK(hipEventSynchronize(e.second));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
        tot += ms;
    }
    *walk_ms = tot;
    *launches = ctx->prof_pending.size();
    ctx->prof_pool.insert(ctx->prof_pool.end(), ctx->prof_pending.begin(), ctx->prof_pending.end());
    ctx->prof_pending.clear();
    return PERM_OK;
}

// ------------------------------------------------------------------ helpers
extern "C" int perm_schur_primes(int n, int extra, uint32_t *primes, int max_primes, int *k)
{
    if (n < 1 || extra < 0 || !primes || !k) return fail(PERM_EINVAL, "bad argument");
    for (int cnt = 1; cnt <= 64; ++cnt) {
        std::vector<uint32_t> ps = permh::primes_1_mod_n(n, cnt);
        if ((int)ps.size() < cnt) return fail(PERM_ERANGE, "not enough 31-bit primes = 1 mod %d", n);
        if (permh::schur_bound_ok(n, ps)) {
            ps = permh::primes_1_mod_n(n, cnt + extra);
            if ((int)ps.size() < cnt + extra) return fail(PERM_ERANGE, "not enough primes");
            if ((int)ps.size() > max_primes) return fail(PERM_ERANGE, "max_primes too small");
            std::copy(ps.begin(), ps.end(), primes);
            *k = (int)ps.size();
            return PERM_OK;
        }
    }
    return fail(PERM_ERANGE, "bound not reached with 64 primes");
}

extern "C" int perm_pick_primes(int n, int extra, uint32_t *primes, int max_primes, int *k)
{
    return perm_schur_primes(n, extra, primes, max_primes, k);
}

extern "C" int perm_schur_residues(int n, uint32_t p, uint32_t *out)
{
    if (n < 1 || !out) return fail(PERM_EINVAL, "bad argument");
    if (!permh::is_prime_u32(p) || (p - 1) % (uint32_t)n)
        return fail(PERM_EINVAL, "p = %u is not a prime = 1 (mod %d)", p, n);
    const uint32_t g = permh::root_of_unity(n, p);
    if (!g) return fail(PERM_EINVAL, "no primitive root of unity");
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
            out[(size_t)j * n + k] = (uint32_t)permh::powmod(g, (uint64_t)j * k, p);
    return PERM_OK;
}

// ------------------------------------------------------------------ tuning
static bool tune_key_ok(int field, int n)
{
    return (field == PERM_C128 || field == PERM_F64 || field == PERM_MODP) && n >= 1 && n <= PERM_NMAX;
}

extern "C" int perm_tune_get(perm_ctx *ctx, int field, int n, perm_tune *out)
{
    if (!ctx || !out || !tune_key_ok(field, n)) return fail(PERM_EINVAL, "bad argument");
    auto it = ctx->tune.find({field, n});
    perm_tune t{};
    if (it != ctx->tune.end()) t = it->second;
    if (t.log2_chunk <= 0) t.log2_chunk = default_log2_chunk(field, n);
    *out = t;
    return PERM_OK;
}

extern "C" int perm_tune_set(perm_ctx *ctx, int field, int n, const perm_tune *t)
{
    if (!ctx || !t || !tune_key_ok(field, n)) return fail(PERM_EINVAL, "bad argument");
    if (t->log2_chunk < 0 || t->log2_chunk > 24 || t->grid_per_cu < 0)
        return fail(PERM_EINVAL, "log2_chunk must be in [0, 24], grid_per_cu >= 0");
    if (field == PERM_MODP && t->log2_chunk > 20)
        return fail(PERM_EINVAL, "F_p chunks are limited to 2^20 indices per lane");
    ctx->tune[{field, n}] = *t;
    return PERM_OK;
}

// The key of a tuning table: the device's architecture name and the HIP
// runtime version (timings, and so the best partition, change with both).
static int tune_key(perm_ctx *ctx, std::string &arch, int &hip_version)
{
    arch = ctx->arch;
    hip_version = 0;
    HIPCHK(hipRuntimeGetVersion(&hip_version));
    return PERM_OK;
}

extern "C" int perm_tune_save(perm_ctx *ctx, const char *path)
{
    if (!ctx || !path) return fail(PERM_EINVAL, "bad argument");
    std::string arch;
    int hv = 0;
    int rc = tune_key(ctx, arch, hv);
    if (rc != PERM_OK) return rc;
    FILE *f = fopen(path, "w");
    if (!f) return fail(PERM_EINVAL, "cannot open %s", path);
    fprintf(f, "# libperm tuning table: field n log2_chunk grid_per_cu\n# arch %s\n# hip %d\n",
            arch.c_str(), hv);
    for (auto &kv : ctx->tune)
        fprintf(f, "%d %d %d %d\n", kv.first.first, kv.first.second, kv.second.log2_chunk,
                kv.second.grid_per_cu);
    const bool ok = !ferror(f);
    if (fclose(f) != 0 || !ok) return fail(PERM_EINVAL, "writing %s failed", path);
    return PERM_OK;
}

extern "C" int perm_tune_load(perm_ctx *ctx, const char *path)
{
    if (!ctx || !path) return fail(PERM_EINVAL, "bad argument");
    std::string arch;
    int hv = 0;
    int rc = tune_key(ctx, arch, hv);
    if (rc != PERM_OK) return rc;
    FILE *f = fopen(path, "r");
    if (!f) return fail(PERM_EINVAL, "cannot open %s", path);
    char line[512];
    std::map<std::pair<int, int>, perm_tune> tab;
    bool have_arch = false, have_hip = false;
    auto bad = [&](const char *why) {
        fclose(f);
        return fail(PERM_EINVAL, "%s: %s", path, why);
    };
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '\n') continue;
        if (line[0] == '#') {
            char key[16] = {0}, val[400] = {0};
            if (sscanf(line, "# %15s %399s", key, val) == 2) {
                if (!strcmp(key, "arch")) {
                    if (arch != val) return bad("tuned for another device architecture");
                    have_arch = true;
                } else if (!strcmp(key, "hip")) {
                    if (atoi(val) != hv) return bad("tuned under another HIP runtime version");
                    have_hip = true;
                }
            }
            continue;
        }
        int field, n, c, g;
        if (sscanf(line, "%d %d %d %d", &field, &n, &c, &g) != 4 || !tune_key_ok(field, n) || c < 0 ||
            c > 24 || g < 0) {
            fclose(f);
            return fail(PERM_EINVAL, "malformed line in %s: %s", path, line);
        }
        if (field == PERM_MODP && c > 20) {
            fclose(f);
            return fail(PERM_EINVAL, "%s: F_p chunks are limited to 2^20 indices per lane: %s", path,
                        line);
        }
        tab[{field, n}] = perm_tune{c, g};
    }
    fclose(f);
    if (!have_arch || !have_hip)
        return fail(PERM_EINVAL, "%s: no '# arch' and '# hip' key lines", path);
    ctx->tune = tab;
    return PERM_OK;
}
