// Staging, finalize and launch code for the Gray walk kernels.
// The walk itself is described in walk_impl.h; its instantiations for every
// (variant, n) live in the walk_inst_*.hip translation units.
#include "walk_impl.h"

namespace permk {

// ----------------------------------------------------------------- staging
__global__ __launch_bounds__(256) void stage_kernel(const MatDesc *mats, const char *src, char *stage)
{
    stage_one(mats[blockIdx.x], src, stage);
}

// ---------------------------------------------------------------- finalize
__global__ __launch_bounds__(256) void finalize_kernel(const MatDesc *mats, const double *partials,
                                                       char *out)
{
    __shared__ double sa[256], sb[256];
    __shared__ unsigned long long su[256];
    finalize_one(mats[blockIdx.x], partials, out, sa, sb, su);
}

// ---------------------------------------------------------- host launchers
static WalkFn fused_fn(int nmax, bool kahan)
{
    if (nmax <= 16) return kahan ? walk_fn_fused16_k() : walk_fn_fused16_nok();
    if (nmax <= 26) return kahan ? walk_fn_fused26_k() : walk_fn_fused26_nok();
    return nullptr;
}

static WalkFn pick(int variant, int n, bool kahan, bool fused, int nmax_fused)
{
    if (fused) return fused_fn(nmax_fused, kahan);
    if (variant < 0 || variant >= V_COUNT || n < 1 || n > NMAX) return nullptr;
    switch (variant) {
    case V_C128: return n <= 24 ? walk_fn_c128_lo(n, kahan) : walk_fn_c128_hi(n, kahan);
    case V_F64: return walk_fn_f64(n, kahan);
    case V_MODP: return walk_fn_modp(n);
    case V_MONT: return walk_fn_mont(n);
    }
    return nullptr;
}

int launch_stage(const MatDesc *d_mats, int nmats, const void *src, void *stage, void *stream)
{
    if (nmats <= 0) return (int)hipSuccess;
    hipLaunchKernelGGL(stage_kernel, dim3(nmats), dim3(256), 0, (hipStream_t)stream, d_mats,
                       (const char *)src, (char *)stage);
    return (int)hipGetLastError();
}

int walk_occupancy(int variant, int n, bool kahan, bool fused, int nmax_fused, int *blocks_per_cu)
{
    WalkFn f = pick(variant, n, kahan, fused, nmax_fused);
    if (!f) return (int)hipErrorInvalidValue;
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)f, BLOCK, 0);
    *blocks_per_cu = nb;
    return (int)e;
}

int launch_walk(int variant, int n, bool kahan, bool fused, int nmax_fused, const WaveItem *d_items,
                uint32_t count, uint32_t grab, const MatDesc *d_mats, const void *stage,
                double *partials, unsigned long long *ctr, CtrState *state, int grid_blocks,
                void *stream, const void *fin_src, void *fin_out, int fin_nmats)
{
    WalkFn f = pick(variant, n, kahan, fused, nmax_fused);
    if (!f || grab < 1 || !state) return (int)hipErrorInvalidValue;
    if (grid_blocks < 1) grid_blocks = 1;
    if (fin_nmats < 0 || (fin_nmats > 0 && !fin_src) || (fin_out && !fin_nmats))
        return (int)hipErrorInvalidValue;
    const uint64_t per_run = (uint64_t)(BLOCK / WAVE) * grab;
    const uint64_t runs = ((uint64_t)count + per_run - 1) / per_run;
    CtrArgs ca{};
    ca.groups = ctr_groups(grid_blocks);
    ca.runs = (uint32_t)runs;
    ca.fin_out = (char *)fin_out;
    ca.fin_src = (const char *)fin_src;
    ca.fin_nmats = (uint32_t)fin_nmats;
    ca.done_base = state->done;
    for (int x = 0; x < CTR_GROUPS; ++x) ca.base[x] = state->base[x];
    const char *st = (const char *)stage;
    void *args[] = {(void *)&d_items, (void *)&count, (void *)&grab, (void *)&d_mats, (void *)&st,
                    (void *)&partials, (void *)&ctr, (void *)&ca};
    hipError_t e = hipLaunchKernel((const void *)f, dim3(grid_blocks), dim3(BLOCK), args, 0,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return (int)e;
    // Block b walks run b without a claim.  With more runs than blocks,
    // counter x then takes one claim per remaining run r = x (mod groups)
    // and one failing claim per block b = x (mod groups): runs_x in all.
    const uint64_t g = ca.groups;
    if (runs > (uint64_t)grid_blocks)
        for (uint64_t x = 0; x < g; ++x) state->base[x] += runs > x ? (runs - x + g - 1) / g : 0;
    if (fin_out && grid_blocks > 1) state->done += (uint64_t)grid_blocks;
    return (int)hipGetLastError();
}

int launch_finalize(const MatDesc *d_mats, int nmats, const double *partials, void *out, void *stream)
{
    if (nmats <= 0) return (int)hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(nmats), dim3(256), 0, (hipStream_t)stream, d_mats,
                       partials, (char *)out);
    return (int)hipGetLastError();
}

}  // namespace permk
