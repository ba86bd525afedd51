// Internal state of libperm shared by the host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/perm.h"
#include "kernels.h"
#include "numth.h"

namespace permi {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

// One matrix to evaluate (or one Gray index range of it).
struct MatIn {
    int variant = 0;
    int n = 0;
    uint32_t p = 0;
    uint64_t src_off = 0;
    uint32_t out_slot = 0;
    bool kahan = true;
    bool full = true;          // whole range [0, 2^(n-1))
    uint64_t x0 = 0, x1 = 0;   // else this range
    bool no_scale = false;     // leave the Glynn sum unscaled
    int out_bytes = 16;        // bytes of the result slot written (16, 8 or 4)
    bool latency = false;      // may use the latency partition (see plan())
};

// One walk launch.
struct Group {
    int variant;
    int n;
    bool kahan;
    bool fused;
    int nmax_fused;
    uint32_t first_item;
    uint32_t count;
};

// Launch shape of one walk group: items per claim and blocks.
struct LaunchShape {
    uint32_t grab;
    int grid;
};

struct Plan {
    std::vector<permk::MatDesc> mats;
    std::vector<permk::WaveItem> items;
    std::vector<Group> groups;
    size_t stage_bytes = 0;
    size_t nparts = 0;
};

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

}  // namespace permi

struct perm_ctx {
    int device = 0;
    int num_cus = 1;
    std::string arch;
    hipStream_t stream = nullptr;
    hipEvent_t last_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
    size_t budget = 0, used = 0;
    permi::DevBuf src, stage, partials, outs, plan_buf, ctr;
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t pinned_ev = nullptr;
    bool pinned_busy = false;
    // pinned result slots of calls whose results go to the host (single
    // calls with a host output, CRT residues), written by the finalize step
    // through their device address (no copy launch)
    void *host_out = nullptr;
    void *host_out_dev = nullptr;
    size_t host_out_cap = 0;
    permk::CtrState ctr_state;
    int grid_per_cu = 0;
    std::map<std::pair<int, int>, perm_tune> tune;
    std::map<int, int> occ;
    bool prof_on = false;
    // walk-launch timing events; a server's worker thread records into them
    // too, so they are guarded
    std::mutex prof_mu;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending, prof_pool;
    // host scratch reused across calls (keeps its capacity: large batches
    // would otherwise fault in fresh pages on every call)
    std::vector<permi::MatIn> scratch_in;
    permi::Plan scratch_plan;
    std::vector<permi::LaunchShape> scratch_shape;
    // The last small plan built in scratch_plan, with the chunk length it
    // used per (variant, n): a call with the same inputs and chunk lengths
    // reuses it, and its upload when plan_buf still holds it.
    std::vector<permi::MatIn> plan_in;
    std::vector<std::pair<std::pair<int, int>, int>> plan_chunks;
    std::vector<std::pair<std::pair<int, int>, int>> plan_latency;
    bool plan_cached = false;
    // device address of the static scratch of perm_c128_noalloc on this device
    void *noalloc_ptr = nullptr;
    uint64_t plan_id = 0, uploaded_plan_id = ~0ull;
    const void *uploaded_ptr = nullptr;
};

namespace permi {
int ensure(perm_ctx *ctx, DevBuf &b, size_t bytes);
int default_log2_chunk(int variant, int n);
int log2_chunk_for(const perm_ctx *ctx, int variant, int n);
int latency_log2_chunk(const perm_ctx *ctx, int variant, int n, uint64_t nmats, int blocks_per_cu);
int plan(perm_ctx *ctx, const std::vector<MatIn> &in, Plan &pl);
int begin_call(perm_ctx *ctx, hipStream_t s);
int end_call(perm_ctx *ctx, hipStream_t s);
int execute(perm_ctx *ctx, Plan &pl, const void *src, void *out, size_t out_slots, hipStream_t s);
int validate_plan(const perm_ctx *ctx, const Plan &pl, size_t out_slots);
int variant_of(int field, unsigned flags);
int source_on_device(perm_ctx *ctx, const void *data, size_t bytes, unsigned flags, hipStream_t s,
                     const void **dev);
int check_primes(const uint32_t *primes, int k, double log2_bound);
int write_limbs(const permh::BigU &mag, int sgn, uint64_t *limbs, int max_limbs, int *nlimbs,
                int *sign);
}  // namespace permi
