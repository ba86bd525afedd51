// Request loop with continuous batching for permanents.
//
// A request is one matrix.  On admission (HBM bytes and in-flight slots
// permitting) its matrix is copied into the server's device arena, staged,
// and its Gray index range is split into wavefront items exactly as
// perm_batch would split it (same chunk length, same partial slots), so its
// result is bit-identical to perm_batch's.  The worker thread then runs
// slices: each slice takes items from all admitted requests, shortest
// remaining work first with a guaranteed share for the oldest request, up to
// a work budget calibrated to `slice_us` of device time, launches the walk,
// and finalizes the requests whose last items it carried.  Slices alternate
// between two streams, so the next slice's waves start on compute units as
// soon as the current slice's waves drain, and requests submitted while a
// slice runs join the next one.  Ordering across the two streams: a slice
// waits (on the device) for the staging of requests admitted by the previous
// slice, and a finalize waits for the previous slice to complete.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "numth.h"

using namespace permk;
using namespace permi;

namespace {

double now_us()
{
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing.
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> bytes
    size_t size = 0, used = 0;
    void init(size_t s) { size = s; free_.clear(); free_[0] = s; used = 0; }
    bool alloc(size_t bytes, size_t &off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used += bytes;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum ReqState { R_PENDING, R_ADMITTED, R_DONE };

struct Req {
    uint64_t ticket = 0;
    int variant = 0, n = 0;
    uint32_t p = 0;
    std::vector<unsigned char> matrix;
    ReqState state = R_PENDING;
    int status = PERM_OK;
    bool cancel = false;
    double t_submit = 0, t_done = 0;
    double t_admit = 0, t_start = 0;     // admitted; first slice with its items launched
    // device placement (admitted)
    size_t off = 0, bytes = 0;
    int slot = -1;                       // row of the device MatDesc table
    MatDesc md{};
    // wave items, generated on demand in slot order: item i covers
    // [i * nlanes * 2^log2L, (i+1) * nlanes * 2^log2L) -- the split perm_batch
    // makes of a full index range
    int chunk = 0;                       // log2 chunk length fixed at submit
    uint32_t log2L = 0, nlanes = 0;
    size_t nitems = 0;
    size_t next = 0;                     // first item not yet scheduled
    int inflight_slices = 0;
    double work = 0;                     // remaining lane-steps x n (scheduling key)
    unsigned char result[16] = {0};
};

struct Slice {
    hipEvent_t done = nullptr;           // end of all of the slice's work
    hipEvent_t staged = nullptr;         // after its staging kernel (if any)
    bool has_staged = false;
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    std::vector<uint64_t> finishing;     // tickets finalized by this slice
    std::vector<uint64_t> touched;       // tickets with items in this slice
    double work = 0;
    size_t nitems = 0;
    double launch_us = 0;                // host time of the launch
    bool busy = false;
};

constexpr size_t kSliceItems = 1 << 17;   // wave items per slice, at most
// F_p results are exact whatever the partition, so served F_p requests use
// items of at most 64 x 2^8 indices (about 0.35 ms of a wave's time at
// n = 34 with three waves per SIMD): a slice is never stuck behind long
// items.  (Float requests keep the partition of perm_batch on
// the same context, whose summation order they reproduce bit for bit; the
// context's tuning table sets it.)
constexpr int kServeModpChunk = 8;

WaveItem request_item(const Req &r, size_t i)
{
    WaveItem it{};
    it.x0 = (uint64_t)i * ((uint64_t)r.nlanes << r.log2L);
    it.mat = (uint32_t)r.slot;
    it.slot = r.md.first_part + (uint32_t)i;
    it.log2L = r.log2L;
    it.nlanes = r.nlanes;
    return it;
}

double item_work(const WaveItem &it, int n)
{
    return (double)it.nlanes * std::ldexp(1.0, (int)it.log2L) * n;
}

}  // namespace

struct perm_srv {
    perm_ctx *ctx = nullptr;
    perm_srv_cfg cfg{};
    void *arena_dev = nullptr;
    Arena arena;
    void *table_dev = nullptr;           // max_inflight MatDescs
    void *results_dev = nullptr;         // max_inflight * 16 bytes
    void *ctr_dev = nullptr;             // one block of work counters per stream
    CtrState ctr_state[2];
    hipStream_t streams[2] = {nullptr, nullptr};
    bool prev_done_valid = false;        // slices[cur ^ 1].done refers to the previous slice
    std::vector<int> free_slots;
    Slice slices[2];
    int cur = 0;
    double rate = 2.0e12;                // work units per second, calibrated (under mu)
    double last_complete_us = -1.0;      // host time the previous slice was seen done

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<uint64_t> admitted;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    std::vector<double> lat_us;
    perm_srv_stats st{};
    double busy_since = -1.0;
};

namespace {

#define SRV_HIP(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            permi::fail(PERM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));           \
            return PERM_EDEVICE;                                                                \
        }                                                                                       \
    } while (0)

int ensure_slice_pinned(Slice &s, size_t bytes)
{
    if (bytes <= s.pinned_cap) return PERM_OK;
    if (s.pinned) (void)hipHostFree(s.pinned);
    s.pinned = nullptr;
    s.pinned_cap = 0;
    const size_t want = std::max(bytes, (size_t)1 << 20);
    SRV_HIP(hipHostMalloc(&s.pinned, want, hipHostMallocDefault));
    s.pinned_cap = want;
    return PERM_OK;
}

// Admit pending requests while the budgets allow (called with mu held).
// Returns the tickets admitted now.
std::vector<uint64_t> admit_locked(perm_srv *S)
{
    std::vector<uint64_t> now;
    while (!S->pending.empty() && !S->free_slots.empty()) {
        const uint64_t t = S->pending.front();
        Req &r = S->reqs[t];
        if (r.cancel) {
            S->pending.pop_front();
            r.state = R_DONE;
            r.status = PERM_ECANCELED;
            r.t_done = now_us();
            S->st.canceled++;
            S->cv_done.notify_all();
            continue;
        }
        size_t off = 0;
        if (!S->arena.alloc(r.bytes, off)) break;          // wait for memory
        S->pending.pop_front();
        r.off = off;
        r.slot = S->free_slots.back();
        S->free_slots.pop_back();
        r.state = R_ADMITTED;
        r.t_admit = now_us();
        S->admitted.push_back(t);
        S->st.admitted++;
        now.push_back(t);
    }
    return now;
}

// Describe an admitted request: arena layout [src][staged][partials].
void layout(perm_srv *S, Req &r)
{
    const size_t src_b = align256((size_t)r.n * r.n * src_entry_bytes(r.variant));
    const size_t stg_b = align256(stage_bytes(r.variant, r.n));
    MatDesc &d = r.md;
    std::memset(&d, 0, sizeof d);
    d.src_off = r.off;
    d.stage_off = r.off + src_b;
    d.first_part = (uint32_t)((r.off + src_b + stg_b) / 16);
    d.n = r.n;
    d.variant = r.variant;
    d.p = r.p;
    d.flags = (S->cfg.flags & PERM_NO_KAHAN) ? 0 : MD_KAHAN;
    d.pinv = r.p ? 1.0 / (double)r.p : 0.0;
    d.mont_pp = r.variant == V_MONT ? permh::mont_pprime(r.p) : 0;
    if (r.variant == V_MODP || r.variant == V_MONT)
        d.fin_scale = permh::fp_finalize_factor(r.p, r.n, r.variant == V_MONT, true);
    d.out_slot = 0;
    // items: the same split perm_batch makes of the full range [0, 2^(n-1))
    r.nitems = 0;
    if (r.n > 0) {
        const int c = r.chunk;
        const uint64_t T = 1ull << (r.n - 1);
        if (T >= (64ull << c)) {
            r.log2L = (uint32_t)c;
            r.nlanes = 64;
            r.nitems = (size_t)(T / (64ull << c));
        } else if (T >= 64) {
            r.log2L = (uint32_t)(r.n - 1 - 6);
            r.nlanes = 64;
            r.nitems = 1;
        } else {
            r.log2L = 0;
            r.nlanes = (uint32_t)T;
            r.nitems = 1;
        }
        d.num_parts = (uint32_t)r.nitems;
    }
    r.next = 0;
    r.work = (double)r.nitems * r.nlanes * std::ldexp(1.0, (int)r.log2L) * r.n;
}

size_t request_bytes(int variant, int n, int chunk)
{
    const size_t src_b = align256((size_t)n * n * src_entry_bytes(variant));
    const size_t stg_b = align256(stage_bytes(variant, n));
    size_t parts = 1;
    if (n > 0) {
        const uint64_t T = 1ull << (n - 1);
        parts = (size_t)(T >= (64ull << chunk) ? T / (64ull << chunk) : 1);
    }
    return src_b + stg_b + align256(parts * 16);
}

// Walk launch for a set of items (grouped by kernel).
int launch_items(perm_srv *S, const std::vector<WaveItem> &items,
                 const std::vector<int> &item_variant, const std::vector<int> &item_n,
                 const WaveItem *d_items_base, hipStream_t s)
{
    // items are ordered: fused-eligible first (one launch), then per (variant, n)
    const bool kahan = !(S->cfg.flags & PERM_NO_KAHAN);
    size_t i = 0;
    while (i < items.size()) {
        const bool fz = item_variant[i] != V_MONT && item_n[i] <= FUSED_BUCKETS[1];
        size_t j = i + 1;
        if (fz) {
            while (j < items.size() && item_variant[j] != V_MONT && item_n[j] <= FUSED_BUCKETS[1]) ++j;
        } else {
            while (j < items.size() && item_variant[j] == item_variant[i] && item_n[j] == item_n[i]) ++j;
        }
        int nmax = 0;
        uint32_t max_l2 = 0;
        for (size_t q = i; q < j; ++q) {
            nmax = std::max(nmax, item_n[q]);
            max_l2 = std::max(max_l2, items[q].log2L);
        }
        uint32_t grab = grab_for(max_l2);
        int occ = 1;
        walk_occupancy(item_variant[i], item_n[i], kahan, fz,
                       nmax <= FUSED_BUCKETS[0] ? FUSED_BUCKETS[0] : FUSED_BUCKETS[1], &occ);
        occ = std::max(occ, 1);
        const uint32_t count = (uint32_t)(j - i);
        // several items per claim only when items far outnumber resident waves
        grab = std::max(1u, std::min(grab, count / (2u * (uint32_t)(occ * S->ctx->num_cus * 4))));
        const uint32_t runs = (count + grab - 1) / grab;
        const int grid = std::max(1, std::min((int)((runs + 3) / 4), occ * S->ctx->num_cus));
        unsigned long long *ctr = (unsigned long long *)((char *)S->ctr_dev + CTR_BYTES * S->cur);
        // walk-launch timing (perm_prof_enable on the context), while the
        // context's pool of event pairs lasts
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        bool prof = false;
        {
            std::lock_guard<std::mutex> lk(S->ctx->prof_mu);
            if (S->ctx->prof_on && !S->ctx->prof_pool.empty()) {
                ev = S->ctx->prof_pool.back();
                S->ctx->prof_pool.pop_back();
                prof = true;
            }
        }
        if (prof) SRV_HIP(hipEventRecord(ev.first, s));
        SRV_HIP((hipError_t)launch_walk(item_variant[i], item_n[i], kahan, fz,
                                        nmax <= FUSED_BUCKETS[0] ? FUSED_BUCKETS[0] : FUSED_BUCKETS[1],
                                        d_items_base + i, count, grab, (const MatDesc *)S->table_dev,
                                        S->arena_dev, (double *)S->arena_dev, ctr,
                                        &S->ctr_state[S->cur], grid, s));
        if (prof) {
            SRV_HIP(hipEventRecord(ev.second, s));
            std::lock_guard<std::mutex> lk(S->ctx->prof_mu);
            S->ctx->prof_pending.push_back(ev);
        }
        i = j;
    }
    return PERM_OK;
}

// Mark a request finished with `status` (with mu held); a request already
// finished (failed, cancelled) is never revived.
void finish_locked(perm_srv *S, Req &r, int status, double t)
{
    if (r.state == R_DONE) return;
    r.state = R_DONE;
    r.status = r.cancel ? PERM_ECANCELED : status;
    r.t_done = t;
    r.next = r.nitems;                   // nothing more of it is scheduled
    if (r.status == PERM_OK) {
        S->st.completed++;
        S->lat_us.push_back(t - r.t_submit);
    } else if (r.status == PERM_ECANCELED) {
        S->st.canceled++;
    } else {
        S->st.failed++;
    }
}

// Complete a slice whose device work has ended: publish the results of its
// finishing requests.  With status != PERM_OK (the slice's device work
// failed, or it failed to launch) every request with items in it fails: its
// partial sums are incomplete.  A request's device memory and slot are
// released once no slice in flight carries its items.
void complete_slice(perm_srv *S, Slice &sl, int status)
{
    std::lock_guard<std::mutex> lk(S->mu);
    const double t = now_us();
    const size_t res_off = sl.pinned_cap - 16 * (size_t)S->cfg.max_inflight;
    for (size_t q = 0; q < sl.finishing.size(); ++q) {
        auto it = S->reqs.find(sl.finishing[q]);
        if (it == S->reqs.end() || it->second.state == R_DONE) continue;
        Req &r = it->second;
        if (status == PERM_OK) std::memcpy(r.result, (char *)sl.pinned + res_off + 16 * q, 16);
        finish_locked(S, r, status, t);
    }
    if (status != PERM_OK)
        for (uint64_t tk : sl.touched) {
            auto it = S->reqs.find(tk);
            if (it != S->reqs.end()) finish_locked(S, it->second, status, t);
        }
    for (uint64_t tk : sl.touched) {
        auto it = S->reqs.find(tk);
        if (it != S->reqs.end()) it->second.inflight_slices--;
    }
    // release device memory of requests that are done or cancelled and idle
    for (size_t a = 0; a < S->admitted.size();) {
        Req &r = S->reqs[S->admitted[a]];
        const bool finished = r.state == R_DONE || (r.cancel && r.inflight_slices == 0);
        if (finished && r.inflight_slices == 0) {
            if (r.state != R_DONE) {
                r.state = R_DONE;
                r.status = PERM_ECANCELED;
                r.t_done = t;
                S->st.canceled++;
            }
            S->arena.release(r.off, r.bytes);
            S->free_slots.push_back(r.slot);
            S->admitted[a] = S->admitted.back();
            S->admitted.pop_back();
        } else {
            ++a;
        }
    }
    S->st.terms += sl.work;
    sl.finishing.clear();
    sl.touched.clear();
    sl.busy = false;
    S->cv_done.notify_all();
}

// Launch the next slice on stream `cur`; *launched tells whether any work
// went to the device.
int run_slice(perm_srv *S, bool *launched)
{
    *launched = false;
    Slice &sl = S->slices[S->cur];
    if (sl.busy) {
        if (hipEventSynchronize(sl.done) != hipSuccess) {
            complete_slice(S, sl, PERM_EDEVICE);
            return PERM_EDEVICE;
        }
        // Throughput from the spacing of consecutive completions, sampled only
        // when this slice was already queued as the previous one finished (so
        // the device had its work the whole interval) and it carried enough
        // items to fill the device.  (Measuring against the other stream's
        // event instead samples only when the two completions happen to be
        // close together and overestimates the rate.)
        const double now = now_us();
        const size_t fill = (size_t)S->ctx->num_cus * 12;
        if (S->last_complete_us > 0 && sl.launch_us < S->last_complete_us && sl.work > 0 &&
            sl.nitems >= fill / 2 && now - S->last_complete_us > 20.0) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->rate = 0.7 * S->rate + 0.3 * (sl.work / ((now - S->last_complete_us) * 1e-6));
        }
        S->last_complete_us = now;
        complete_slice(S, sl, PERM_OK);
    }
    std::vector<uint64_t> fresh;
    // Requests admitted now.  Their nodes stay put while the map rehashes
    // and none is erased while admitted; only this thread writes the fields
    // read below, so they are read through these pointers without the lock.
    // A lookup in S->reqs must hold the lock: submit and poll change the map.
    std::vector<const Req *> fresh_r;
    std::vector<WaveItem> items;
    std::vector<int> iv, in_;
    std::vector<MatDesc> fin;
    std::vector<uint64_t> fin_t, touched;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        fresh = admit_locked(S);
        for (uint64_t t : fresh) {
            Req &r = S->reqs.at(t);
            layout(S, r);
            r.inflight_slices++;          // held until this slice completes
            touched.push_back(t);
            fresh_r.push_back(&r);
        }
        // choose items: shortest remaining work first; the oldest request
        // gets at least 1/8 of the budget.  A slice also carries at least
        // `fill` items (while any remain), about one per wave the device
        // holds, so that no slice leaves compute units idle.
        const double budget = std::max(S->rate * S->cfg.slice_us * 1e-6, 1.0);
        const size_t fill = (size_t)S->ctx->num_cus * 12;
        std::vector<uint64_t> order;
        uint64_t oldest = 0;
        double oldest_t = 1e300;
        for (uint64_t t : S->admitted) {
            Req &r = S->reqs[t];
            if (r.cancel || r.state == R_DONE || r.next >= r.nitems) continue;
            order.push_back(t);
            if (r.t_submit < oldest_t) { oldest_t = r.t_submit; oldest = t; }
        }
        std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
            const Req &x = S->reqs[a], &y = S->reqs[b];
            return x.work != y.work ? x.work < y.work : a < b;
        });
        double used = 0.0;
        auto take = [&](Req &r, double cap, bool to_fill) {
            bool any = false;
            while (r.next < r.nitems && (used < cap || (to_fill && items.size() < fill)) &&
                   items.size() < kSliceItems) {
                const WaveItem w = request_item(r, r.next++);
                const double wk = item_work(w, r.n);
                items.push_back(w);
                iv.push_back(r.variant);
                in_.push_back(r.n);
                used += wk;
                r.work -= wk;
                any = true;
            }
            if (any) { r.inflight_slices++; touched.push_back(r.ticket); }
            if (r.next == r.nitems && any) { fin.push_back(r.md); fin_t.push_back(r.ticket); }
        };
        if (oldest) take(S->reqs[oldest], budget / 8, false);
        for (uint64_t t : order) {
            if (used >= budget && items.size() >= fill) break;
            if (t == oldest && S->reqs[t].next >= S->reqs[t].nitems) continue;
            take(S->reqs[t], budget, true);
        }
        // n = 0 requests (no items): finalize directly
        for (uint64_t t : fresh) {
            Req &r = S->reqs[t];
            if (r.nitems == 0 && !r.cancel) {
                fin.push_back(r.md);
                fin_t.push_back(t);
            }
        }
    }
    if (fresh.empty() && items.empty() && fin.empty()) return PERM_OK;
    // From here on the slice owns these requests' items: if anything below
    // fails, the worker fails exactly the requests listed here.
    sl.finishing = fin_t;
    sl.touched = touched;
    sl.work = 0;
    if (items.size() > kSliceItems) return permi::fail(PERM_EINVAL, "slice item overflow");
    // every item must stay inside its request's Gray range and partial slots
    for (size_t q = 0; q < items.size(); ++q) {
        const WaveItem &w = items[q];
        const uint64_t end = w.x0 + ((uint64_t)w.nlanes << w.log2L);
        if (in_[q] < 1 || end > (1ull << (in_[q] - 1)) || w.mat >= (uint32_t)S->cfg.max_inflight ||
            ((size_t)w.slot + 1) * 16 > S->cfg.hbm_budget)
            return permi::fail(PERM_EINVAL, "server slice item %zu out of range", q);
    }

    // group items: fused-eligible first, then by (variant, n)
    {
        std::vector<size_t> idx(items.size());
        for (size_t q = 0; q < idx.size(); ++q) idx[q] = q;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
            const bool fa = iv[a] != V_MONT && in_[a] <= FUSED_BUCKETS[1];
            const bool fb = iv[b] != V_MONT && in_[b] <= FUSED_BUCKETS[1];
            if (fa != fb) return fa;
            if (!fa && (iv[a] != iv[b] || in_[a] != in_[b]))
                return iv[a] != iv[b] ? iv[a] < iv[b] : in_[a] < in_[b];
            return item_work(items[a], in_[a]) > item_work(items[b], in_[b]);
        });
        std::vector<WaveItem> i2;
        std::vector<int> v2, n2;
        for (size_t q : idx) { i2.push_back(items[q]); v2.push_back(iv[q]); n2.push_back(in_[q]); }
        items.swap(i2);
        iv.swap(v2);
        in_.swap(n2);
    }
    // pinned layout: [new MatDescs][matrices][items][finalize MatDescs] ... [results]
    size_t mat_bytes = 0;
    for (const Req *r : fresh_r) mat_bytes += align256(r->matrix.size());
    const size_t nb = fresh.size() * sizeof(MatDesc);
    const size_t ib = items.size() * sizeof(WaveItem);
    const size_t fb = fin.size() * sizeof(MatDesc);
    const size_t res_b = 16 * (size_t)S->cfg.max_inflight;
    const size_t need = align256(nb) + mat_bytes + align256(ib) + align256(fb) + res_b;
    if (need > sl.pinned_cap) {
        // keep the results area at the end
        if (ensure_slice_pinned(sl, need) != PERM_OK) return PERM_ENOMEM;
    }
    char *hp = (char *)sl.pinned;
    const hipStream_t s = S->streams[S->cur];
    Slice &prev = S->slices[S->cur ^ 1];
    // device scratch after the two result areas: one region per slice with
    // [new MatDescs][items][finalize MatDescs]
    const size_t mi = (size_t)S->cfg.max_inflight;
    const size_t region = align256(sizeof(MatDesc) * mi) + align256(sizeof(WaveItem) * kSliceItems) +
                          align256(sizeof(MatDesc) * mi);
    char *d_new = (char *)S->results_dev + res_b * 2 + (size_t)S->cur * region;
    char *d_slice = d_new + align256(sizeof(MatDesc) * mi);
    char *d_fin = d_slice + align256(sizeof(WaveItem) * kSliceItems);
    // requests admitted by the previous slice (other stream) must be staged first
    if (S->prev_done_valid && prev.has_staged) SRV_HIP(hipStreamWaitEvent(s, prev.staged, 0));
    sl.has_staged = false;
    size_t hoff = 0;
    // 1. new requests: descriptors into the table, matrices into the arena, stage
    if (!fresh.empty()) {
        for (size_t q = 0; q < fresh_r.size(); ++q) std::memcpy(hp + q * sizeof(MatDesc), &fresh_r[q]->md, sizeof(MatDesc));
        hoff = align256(nb);
        for (size_t q = 0; q < fresh_r.size(); ++q) {
            const Req &r = *fresh_r[q];
            if (!r.matrix.empty()) {
                std::memcpy(hp + hoff, r.matrix.data(), r.matrix.size());
                SRV_HIP(hipMemcpyAsync((char *)S->arena_dev + r.md.src_off, hp + hoff,
                                       r.matrix.size(), hipMemcpyHostToDevice, s));
            }
            SRV_HIP(hipMemcpyAsync((char *)S->table_dev + sizeof(MatDesc) * r.slot,
                                   hp + q * sizeof(MatDesc), sizeof(MatDesc),
                                   hipMemcpyHostToDevice, s));
            hoff += align256(r.matrix.size());
        }
        SRV_HIP(hipMemcpyAsync(d_new, hp, nb, hipMemcpyHostToDevice, s));
        SRV_HIP((hipError_t)launch_stage((const MatDesc *)d_new, (int)fresh.size(), S->arena_dev,
                                         S->arena_dev, s));
        SRV_HIP(hipEventRecord(sl.staged, s));
        sl.has_staged = true;
    }
    // 2. the walk over this slice's items
    if (!items.empty()) {
        std::memcpy(hp + hoff, items.data(), ib);
        SRV_HIP(hipMemcpyAsync(d_slice, hp + hoff, ib, hipMemcpyHostToDevice, s));
        hoff += align256(ib);
        if (launch_items(S, items, iv, in_, (const WaveItem *)d_slice, s) != PERM_OK) return PERM_EDEVICE;
    }
    // 3. finalize the requests whose last items ran, into this slice's result area
    if (!fin.empty()) {
        for (size_t q = 0; q < fin.size(); ++q) fin[q].out_slot = (uint32_t)q;
        std::memcpy(hp + hoff, fin.data(), fb);
        SRV_HIP(hipMemcpyAsync(d_fin, hp + hoff, fb, hipMemcpyHostToDevice, s));
        hoff += align256(fb);
        char *d_res = (char *)S->results_dev + res_b * S->cur;
        // every earlier slice has finished once the previous one (other stream) has
        if (S->prev_done_valid) SRV_HIP(hipStreamWaitEvent(s, prev.done, 0));
        SRV_HIP((hipError_t)launch_finalize((const MatDesc *)d_fin, (int)fin.size(),
                                            (const double *)S->arena_dev, d_res, s));
        SRV_HIP(hipMemcpyAsync((char *)sl.pinned + sl.pinned_cap - res_b, d_res, 16 * fin.size(),
                               hipMemcpyDeviceToHost, s));
    }
    SRV_HIP(hipEventRecord(sl.done, s));
    for (size_t q = 0; q < items.size(); ++q) sl.work += item_work(items[q], in_[q]);
    sl.nitems = items.size();
    sl.launch_us = now_us();
    sl.busy = true;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->st.slices++;
        S->st.items += items.size();
        for (uint64_t t : fresh) S->reqs.at(t).matrix.clear();
        for (uint64_t t : sl.touched) {
            Req &r = S->reqs.at(t);
            if (r.t_start == 0) r.t_start = sl.launch_us;
        }
    }
    S->cur ^= 1;
    S->prev_done_valid = true;
    *launched = true;
    return PERM_OK;
}

bool has_work_locked(perm_srv *S)
{
    if (!S->pending.empty() && !S->free_slots.empty()) return true;
    for (uint64_t t : S->admitted) {
        const Req &r = S->reqs.at(t);
        if (!r.cancel && r.state != R_DONE && r.next < r.nitems) return true;
    }
    return false;
}

void worker_main(perm_srv *S)
{
    (void)hipSetDevice(S->ctx->device);
    for (;;) {
        bool any_busy = S->slices[0].busy || S->slices[1].busy;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (!any_busy) {
                S->cv_work.wait(lk, [&] { return S->stop || has_work_locked(S); });
                if (S->stop && !has_work_locked(S)) break;
            }
            if (S->busy_since < 0 && (has_work_locked(S) || any_busy)) S->busy_since = now_us();
        }
        bool work, launched = false;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            work = has_work_locked(S);
        }
        if (work) {
            if (run_slice(S, &launched) != PERM_OK) {
                // The slice on stream `cur` failed to launch (part of it may
                // have been issued) or an earlier slice's device work failed.
                // First drain both streams, so that no issued work still
                // reads or writes a request's arena range or descriptor slot
                // when it is released; then the other stream's slice
                // completes as its event says, and every request with items
                // in the failed slice fails.  Requests it did not touch keep
                // being served.
                for (hipStream_t st : S->streams) (void)hipStreamSynchronize(st);
                Slice &other = S->slices[S->cur ^ 1];
                if (other.busy)
                    complete_slice(S, other, hipEventQuery(other.done) == hipSuccess ? PERM_OK
                                                                                     : PERM_EDEVICE);
                complete_slice(S, S->slices[S->cur], PERM_EDEVICE);
                launched = true;
            }
        }
        if (!launched) {
            // Nothing left to launch, or admission waits for device memory
            // held by in-flight requests: drain the in-flight slices.
            for (int q = 0; q < 2; ++q) {
                Slice &sl = S->slices[S->cur];
                if (sl.busy) {
                    const int st = hipEventSynchronize(sl.done) == hipSuccess ? PERM_OK : PERM_EDEVICE;
                    complete_slice(S, sl, st);
                }
                S->cur ^= 1;
            }
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->busy_since >= 0 && !has_work_locked(S)) {
                S->st.busy_s += (now_us() - S->busy_since) * 1e-6;
                S->busy_since = -1;
            }
        }
    }
}

}  // namespace

extern "C" int perm_srv_create(perm_ctx *ctx, const perm_srv_cfg *cfg, perm_srv **out)
{
    if (!ctx || !out) return fail(PERM_EINVAL, "NULL argument");
    *out = nullptr;
    perm_srv *S = new (std::nothrow) perm_srv();
    if (!S) return fail(PERM_ENOMEM, "host allocation failed");
    S->ctx = ctx;
    if (cfg) S->cfg = *cfg;
    if (!S->cfg.hbm_budget) S->cfg.hbm_budget = (size_t)1 << 30;
    if (S->cfg.max_inflight <= 0) S->cfg.max_inflight = 4096;
    if (S->cfg.max_pending <= 0) S->cfg.max_pending = 65536;
    if (!(S->cfg.slice_us > 0)) S->cfg.slice_us = 500.0;
    S->cfg.hbm_budget = align256(S->cfg.hbm_budget);
    auto bail = [&](const char *what) {
        perm_srv_destroy(S);
        return fail(PERM_EDEVICE, "server setup failed: %s", what);
    };
    if (hipSetDevice(ctx->device) != hipSuccess) return bail("hipSetDevice");
    for (int q = 0; q < 2; ++q)
        if (hipStreamCreateWithFlags(&S->streams[q], hipStreamNonBlocking) != hipSuccess)
            return bail("stream");
    if (hipMalloc(&S->arena_dev, S->cfg.hbm_budget) != hipSuccess) {
        (void)hipGetLastError();
        perm_srv_destroy(S);
        return fail(PERM_ENOMEM, "hipMalloc(%zu) for the server arena failed", S->cfg.hbm_budget);
    }
    S->arena.init(S->cfg.hbm_budget);
    const size_t mi = (size_t)S->cfg.max_inflight;
    if (hipMalloc(&S->table_dev, sizeof(MatDesc) * mi) != hipSuccess) return bail("table");
    const size_t res_b = 16 * mi;
    const size_t scratch = res_b * 2 + 2 * (2 * align256(sizeof(MatDesc) * mi) +
                                            align256(sizeof(WaveItem) * kSliceItems));
    if (hipMalloc(&S->results_dev, scratch) != hipSuccess) return bail("results");
    if (hipMalloc(&S->ctr_dev, 2 * CTR_BYTES) != hipSuccess) return bail("counter");
    // zeroed before the worker's first launch on the non-blocking streams
    if (hipMemset(S->ctr_dev, 0, 2 * CTR_BYTES) != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess)
        return bail("counter init");
    for (Slice &sl : S->slices) {
        if (hipEventCreate(&sl.done) != hipSuccess ||
            hipEventCreateWithFlags(&sl.staged, hipEventDisableTiming) != hipSuccess)
            return bail("events");
        if (ensure_slice_pinned(sl, (size_t)4 << 20) != PERM_OK) return bail("pinned");
    }
    for (int q = (int)mi - 1; q >= 0; --q) S->free_slots.push_back(q);
    S->worker = std::thread(worker_main, S);
    *out = S;
    return PERM_OK;
}

extern "C" int perm_srv_submit(perm_srv *S, const perm_item *item, const void *matrix, uint64_t *ticket)
{
    if (!S || !item || !ticket) return fail(PERM_EINVAL, "NULL argument");
    if (item->n < 0 || item->n > PERM_NMAX) return fail(PERM_EINVAL, "n out of range");
    if (item->field != PERM_C128 && item->field != PERM_F64 && item->field != PERM_MODP)
        return fail(PERM_EINVAL, "unknown field");
    if (item->field == PERM_MODP && (item->p < 3 || !(item->p & 1) || item->p >= (1u << 31)))
        return fail(PERM_EINVAL, "modulus must be odd with 3 <= p < 2^31");
    if (item->n > 0 && !matrix) return fail(PERM_EINVAL, "matrix is NULL");
    const int variant = item->field == PERM_C128 ? V_C128
                        : item->field == PERM_F64 ? V_F64
                        : ((S->cfg.flags & PERM_MONTGOMERY) ? V_MONT : V_MODP);
    const size_t mbytes = (size_t)item->n * item->n * src_entry_bytes(variant);
    int chunk = item->n > 0 ? log2_chunk_for(S->ctx, variant, item->n) : 0;
    if (variant == V_MODP || variant == V_MONT) chunk = std::min(chunk, kServeModpChunk);
    const size_t need = request_bytes(variant, item->n, chunk);
    if (need > S->cfg.hbm_budget)
        return fail(PERM_ENOMEM, "request needs %zu device bytes, budget %zu", need, S->cfg.hbm_budget);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(PERM_EINVAL, "server is shutting down");
    if ((int)S->pending.size() >= S->cfg.max_pending) return fail(PERM_EAGAIN, "pending queue full");
    Req r;
    r.ticket = S->next_ticket++;
    r.variant = variant;
    r.n = item->n;
    r.p = item->field == PERM_MODP ? item->p : 0;
    r.matrix.assign((const unsigned char *)matrix, (const unsigned char *)matrix + mbytes);
    r.bytes = need;
    r.chunk = chunk;
    r.t_submit = now_us();
    *ticket = r.ticket;
    S->reqs.emplace(r.ticket, std::move(r));
    S->pending.push_back(*ticket);
    S->st.submitted++;
    S->cv_work.notify_one();
    return PERM_OK;
}

static int poll_impl(perm_srv *S, uint64_t ticket, void *out16, int *done, double *latency_us,
                     perm_srv_times *times)
{
    if (!S || !done) return fail(PERM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(PERM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Req &r = it->second;
    if (r.state != R_DONE) { *done = 0; return PERM_OK; }
    // keep the record while the server still references it
    bool referenced = false;
    for (uint64_t t : S->admitted) if (t == ticket) referenced = true;
    *done = 1;
    const int st = r.status;
    if (out16 && st == PERM_OK) std::memcpy(out16, r.result, 16);
    if (latency_us) *latency_us = r.t_done - r.t_submit;
    if (times) {
        // phases end where the next begins; a phase never reached ends at t_done
        const double a = r.t_admit > 0 ? r.t_admit : r.t_done;
        const double b = r.t_start > 0 ? r.t_start : r.t_done;
        times->queued_us = a - r.t_submit;
        times->admitted_us = b - a;
        times->running_us = r.t_done - b;
        times->latency_us = r.t_done - r.t_submit;
    }
    if (!referenced) S->reqs.erase(it);
    return st;
}

static int wait_impl(perm_srv *S, uint64_t ticket, double timeout_s, void *out16, int *done,
                     double *latency_us, perm_srv_times *times)
{
    if (!S || !done) return fail(PERM_EINVAL, "NULL argument");
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::microseconds((int64_t)(std::max(0.0, timeout_s) * 1e6));
        S->cv_done.wait_until(lk, deadline, [&] {
            auto it = S->reqs.find(ticket);
            return it == S->reqs.end() || it->second.state == R_DONE;
        });
    }
    return poll_impl(S, ticket, out16, done, latency_us, times);
}

extern "C" int perm_srv_poll(perm_srv *S, uint64_t ticket, void *out16, int *done,
                             double *latency_us)
{
    return poll_impl(S, ticket, out16, done, latency_us, nullptr);
}

extern "C" int perm_srv_wait(perm_srv *S, uint64_t ticket, double timeout_s, void *out16, int *done,
                             double *latency_us)
{
    return wait_impl(S, ticket, timeout_s, out16, done, latency_us, nullptr);
}

extern "C" int perm_srv_wait_times(perm_srv *S, uint64_t ticket, double timeout_s, void *out16,
                                   int *done, perm_srv_times *times)
{
    return wait_impl(S, ticket, timeout_s, out16, done, nullptr, times);
}

extern "C" int perm_srv_cancel(perm_srv *S, uint64_t ticket)
{
    if (!S) return fail(PERM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(PERM_ENOTFOUND, "unknown ticket");
    Req &r = it->second;
    if (r.state == R_DONE) return PERM_OK;
    r.cancel = true;
    if (r.state == R_ADMITTED && r.inflight_slices == 0) {
        // nothing of it is on the device: release it now
        S->arena.release(r.off, r.bytes);
        S->free_slots.push_back(r.slot);
        S->admitted.erase(std::remove(S->admitted.begin(), S->admitted.end(), ticket), S->admitted.end());
        r.state = R_DONE;
        r.status = PERM_ECANCELED;
        r.t_done = now_us();
        S->st.canceled++;
        S->cv_done.notify_all();
    } else if (r.state == R_PENDING) {
        S->pending.erase(std::remove(S->pending.begin(), S->pending.end(), ticket), S->pending.end());
        r.state = R_DONE;
        r.status = PERM_ECANCELED;
        r.t_done = now_us();
        S->st.canceled++;
        S->cv_done.notify_all();
    }
    S->cv_work.notify_one();
    return PERM_OK;
}

extern "C" int perm_srv_get_stats(perm_srv *S, perm_srv_stats *out)
{
    if (!S || !out) return fail(PERM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    perm_srv_stats st = S->st;
    std::vector<double> v = S->lat_us;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)std::min<double>(v.size() - 1, std::floor(q * (v.size() - 1) + 0.5));
            return v[i];
        };
        st.p50_us = pct(0.50);
        st.p99_us = pct(0.99);
        double s = 0;
        for (double x : v) s += x;
        st.mean_us = s / v.size();
        st.max_us = v.back();
    }
    if (S->busy_since >= 0) st.busy_s += (now_us() - S->busy_since) * 1e-6;
    st.rate = S->rate;
    *out = st;
    return PERM_OK;
}

extern "C" void perm_srv_destroy(perm_srv *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (uint64_t t : S->pending) {
            Req &r = S->reqs[t];
            r.state = R_DONE;
            r.status = PERM_ECANCELED;
        }
        S->pending.clear();
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->ctx->device);
    for (hipStream_t st : S->streams)
        if (st) (void)hipStreamSynchronize(st);
    for (Slice &sl : S->slices) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.staged) (void)hipEventDestroy(sl.staged);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
    }
    if (S->arena_dev) (void)hipFree(S->arena_dev);
    if (S->table_dev) (void)hipFree(S->table_dev);
    if (S->results_dev) (void)hipFree(S->results_dev);
    if (S->ctr_dev) (void)hipFree(S->ctr_dev);
    for (hipStream_t st : S->streams)
        if (st) (void)hipStreamDestroy(st);
    delete S;
}
