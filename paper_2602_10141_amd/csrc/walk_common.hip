// Staging, finalize and launch code for the Gray walk kernels.
// The walk itself is described in walk_impl.h; its instantiations for every
// (variant, n) live in the walk_inst_*.hip translation units.
#include "walk_impl.h"

namespace permk {

// ----------------------------------------------------------------- staging
// Staged layout, column-major (column k, row i at k*n + i):
//   c128, f64, F_p (Barrett): [+2A][-2A] as binary64 (complex: re, im pairs);
//                             F_p entries are first mapped to balanced
//                             residues in [-(p-1)/2, (p-1)/2];
//   F_p (Montgomery):         [2a mod p][(p - 2a) mod p][a][(p - a) mod p] as uint32.
// Entries of F_p matrices are reduced mod p first.
__global__ __launch_bounds__(256) void stage_kernel(const MatDesc *mats, const char *src, char *stage)
{
    const MatDesc md = mats[blockIdx.x];
    const int n = md.n;
    const int nn = n * n;
    const char *s = src + md.src_off;
    char *d = stage + md.stage_off;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
        const int i = e / n;          // source row
        const int k = e - i * n;      // source column
        const int t = k * n + i;      // staged: column k, row i
        switch (md.variant) {
        case V_C128: {
            const double *a = (const double *)s + 2 * (size_t)e;
            double *o = (double *)d;
            o[2 * t] = 2.0 * a[0];
            o[2 * t + 1] = 2.0 * a[1];
            o[2 * nn + 2 * t] = -2.0 * a[0];
            o[2 * nn + 2 * t + 1] = -2.0 * a[1];
            break;
        }
        case V_F64: {
            const double a = ((const double *)s)[e];
            ((double *)d)[t] = 2.0 * a;
            ((double *)d)[nn + t] = -2.0 * a;
            break;
        }
        case V_MODP: {
            const uint32_t p = md.p;
            const uint32_t a = ((const uint32_t *)s)[e] % p;
            const double b = a > p / 2 ? (double)a - (double)p : (double)a;
            ((double *)d)[t] = 2.0 * b;
            ((double *)d)[nn + t] = -2.0 * b;
            break;
        }
        case V_MONT: {
            const uint32_t p = md.p;
            const uint32_t a = ((const uint32_t *)s)[e] % p;
            const uint32_t two = (uint32_t)((2ull * a) % p);
            uint32_t *o = (uint32_t *)d;
            o[t] = two;
            o[nn + t] = two ? p - two : 0u;
            o[2 * nn + t] = a;
            o[3 * nn + t] = a ? p - a : 0u;
            break;
        }
        }
    }
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
                void *stream, void *fin_out, int fin_nmats)
{
    WalkFn f = pick(variant, n, kahan, fused, nmax_fused);
    if (!f || grab < 1 || !state) return (int)hipErrorInvalidValue;
    if (grid_blocks < 1) grid_blocks = 1;
    if (fin_nmats < 0 || (fin_nmats > 0 && (grid_blocks != 1 || !fin_out)))
        return (int)hipErrorInvalidValue;
    const uint64_t per_run = (uint64_t)(BLOCK / WAVE) * grab;
    const uint64_t runs = ((uint64_t)count + per_run - 1) / per_run;
    CtrArgs ca{};
    ca.groups = ctr_groups(grid_blocks);
    ca.runs = (uint32_t)runs;
    ca.fin_out = (char *)fin_out;
    ca.fin_nmats = (uint32_t)fin_nmats;
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
