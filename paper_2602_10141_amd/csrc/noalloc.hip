// One complex128 permanent with no allocation: the device memory the call
// needs beyond its input and output (work counters, the matrix descriptor,
// wave items, partial sums and staged columns) lives in a file-scope device
// array, and the work partition is written into it by a small kernel, so the
// call makes no hipMalloc, no hipFree and no host-to-device copy.  It runs the
// same stage / walk / finalize kernels as perm_c128 with the same partition,
// so the two give identical bits.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"
#include "walk_impl.h"

namespace permk {

// The call's scratch.  Host code never names it except in the symbol lookup
// below: on the host `scratch` is a stand-in, not a device address.
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` per device, looked up once per device with
// that device current.
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

int noalloc_scratch_init(int device, void **ptr)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES || !ptr) return (int)hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return (int)hipSuccess;
}

// Writes the descriptor of one c128 matrix of order n (staged at offset 0
// of `stage`, result in slot 0), the `count` wave items that split
// [0, 2^(n-1)) into aligned blocks of 2^log2L indices per lane (nlanes lanes
// each) and zeroes the work counters.  n = 0 writes perm = 1 to `out`
// instead.  Thread i of the grid writes item i.
__global__ __launch_bounds__(256) void noalloc_plan_kernel(MatDesc *md, WaveItem *items,
                                                           unsigned long long *ctr, uint32_t count,
                                                           int n, uint32_t log2L, uint32_t nlanes,
                                                           uint32_t flags, double *out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0) {
        for (uint32_t q = threadIdx.x; q < CTR_BYTES / 8; q += blockDim.x) ctr[q] = 0ull;
        if (threadIdx.x == 0) {
            MatDesc d{};
            d.src_off = 0;
            d.stage_off = 0;
            d.first_part = 0;
            d.num_parts = count;
            d.n = n;
            d.variant = V_C128;
            d.flags = flags;
            d.out_slot = 0;
            *md = d;
            if (n == 0) {
                out[0] = 1.0;
                out[1] = 0.0;
            }
        }
    }
    if (i < count) {
        WaveItem it{};
        it.x0 = (uint64_t)i << (log2L + 6);
        it.mat = 0;
        it.slot = i;
        it.log2L = log2L;
        it.nlanes = nlanes;
        items[i] = it;
    }
}

int noalloc_layout(int n, uint32_t count, NoallocLayout *L)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    L->ctr = off;
    off = up(off + CTR_BYTES);
    L->mat = off;
    off = up(off + sizeof(MatDesc));
    L->items = off;
    off = up(off + (size_t)count * sizeof(WaveItem));
    L->partials = off;
    off = up(off + (size_t)count * 16);
    L->stage = off;
    off = up(off + stage_bytes(V_C128, n));
    L->total = off;
    return off <= NOALLOC_SCRATCH_BYTES ? 0 : -1;
}

int launch_noalloc_plan(void *base, const NoallocLayout *L, uint32_t count, int n, uint32_t log2L,
                        uint32_t nlanes, uint32_t flags, double *out, void *stream)
{
    char *b = (char *)base;
    const uint32_t blocks = count ? (count + 255) / 256 : 1;
    hipLaunchKernelGGL(noalloc_plan_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (MatDesc *)(b + L->mat), (WaveItem *)(b + L->items),
                       (unsigned long long *)(b + L->ctr), count, n, log2L, nlanes, flags, out);
    return (int)hipGetLastError();
}

}  // namespace permk
