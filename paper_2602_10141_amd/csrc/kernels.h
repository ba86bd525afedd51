// Internal interface between the host library and the HIP kernels of libperm.
// Not part of the public C ABI (that is include/perm.h).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace permk {

// Arithmetic variants of the Gray walk.
enum Variant : int32_t {
    V_C128 = 0,   // complex128 row sums, Kahan-compensated signed sum
    V_F64  = 1,   // float64 row sums, Kahan-compensated signed sum
    V_MODP = 2,   // F_p: exact integer row sums in binary64, FP64 Barrett modmul
    V_MONT = 3,   // F_p: uint32 residues, 32-bit Montgomery modmul
    V_COUNT = 4
};

constexpr int NMAX = 48;        // largest matrix order any kernel handles
constexpr int WAVE = 64;        // wavefront width on gfx950
constexpr int BLOCK = 256;      // threads per block of the walk kernels (4 waves)

// MatDesc.flags
constexpr uint32_t MD_KAHAN    = 1u;   // compensated summation (floats)
constexpr uint32_t MD_NO_SCALE = 2u;   // finalize leaves the Glynn sum unscaled (range partials)
constexpr uint32_t MD_OUT_8    = 4u;   // finalize writes only the first 8 bytes of the slot (f64)
constexpr uint32_t MD_OUT_4    = 8u;   // ... only the first 4 bytes (F_p residue)

// One matrix of a launch.  64 bytes, read with scalar loads.
struct MatDesc {
    uint64_t src_off;     // byte offset of the caller's matrix in the source buffer
    uint64_t stage_off;   // byte offset of the staged columns in the stage buffer
    uint32_t first_part;  // partial-sum slots [first_part, first_part + num_parts)
    uint32_t num_parts;
    int32_t  n;
    int32_t  variant;
    uint32_t p;           // modulus (F_p variants), else 0
    uint32_t flags;
    double   pinv;        // 1/p rounded to binary64 (V_MODP)
    uint32_t mont_pp;     // -p^{-1} mod 2^32 (V_MONT)
    uint32_t out_slot;    // result slot (16 bytes each) in the output buffer
    uint32_t fin_scale;   // F_p: what finalize multiplies the residue sum by, mod p:
                          //   inv(2)^(n-1) (1 with MD_NO_SCALE), times R^(n-1) for V_MONT
    uint32_t pad;
};
static_assert(sizeof(MatDesc) == 64, "MatDesc layout");

// One wavefront's share of one matrix.  32 bytes, read with scalar loads.
// Lane l < nlanes walks the Gray indices [x0 + l*2^log2L, x0 + (l+1)*2^log2L);
// x0 is a multiple of 2^log2L.  The unscaled signed sum of the wave goes to
// partial slot `slot`.
struct WaveItem {
    uint64_t x0;
    uint32_t mat;
    uint32_t slot;
    uint32_t log2L;
    uint32_t nlanes;
    uint32_t pad[2];
};
static_assert(sizeof(WaveItem) == 32, "WaveItem layout");

// Bytes of staged columns per matrix for a variant.
inline size_t stage_bytes(int variant, int n)
{
    const size_t nn = (size_t)n * (size_t)n;
    switch (variant) {
    case V_C128: return 32 * nn;     // +2A and -2A, complex
    case V_F64:  return 16 * nn;     // +2A and -2A
    case V_MODP: return 16 * nn;     // +2A and -2A, balanced residues
    case V_MONT: return 16 * nn;     // four uint32 arrays
    }
    return 0;
}

// Approximate VALU instructions of one Gray step (flip, product, signed
// accumulate) per lane, used to order wave items by duration: a complex step
// is 2n adds and n - 1 four-instruction complex products, a real step n adds
// and n - 1 products, an F_p (Barrett) step n adds and n - 1 six-instruction
// products; Montgomery's 32-bit products issue at a quarter of that rate.
inline uint64_t step_cost(int variant, int n)
{
    switch (variant) {
    case V_C128: return 6 * (uint64_t)n;
    case V_F64:  return 2 * (uint64_t)n;
    case V_MODP: return 7 * (uint64_t)n;
    case V_MONT: return 10 * (uint64_t)n;
    }
    return (uint64_t)n;
}

// Bytes of one source matrix entry for a variant.
inline size_t src_entry_bytes(int variant)
{
    return variant == V_C128 ? 16 : (variant == V_F64 ? 8 : 4);
}

// ---------------------------------------------------------------- launchers
// All return a hipError_t as int and launch on `stream` (a hipStream_t).

// Staging: for each of `nmats` descriptors, read the source matrix at
// src + src_off and write its staged columns at stage + stage_off.
int launch_stage(const MatDesc *d_mats, int nmats, const void *src, void *stage, void *stream);

// Walk: `count` wave items, all of one (variant, n) when `fused` is false;
// with fused = true the matrices may mix variants and orders n <= nmax_fused.
// `ctr` points at CTR_BYTES of device counters (see below).
//
// Work counters of the persistent kernels: one per XCD (MI355X has 8), 256
// bytes apart.  Block b claims runs of items from counter b mod `groups`
// (groups = the largest power of two <= min(8, grid), so that the remainder
// is a scalar AND); workgroups are dispatched round-robin over the XCDs, so
// each counter serves the blocks of one XCD.  Block b walks run b without a
// claim; counter x then hands out the runs x + groups * (nb + k), k = 0, 1,
// ..., nb being the number of blocks of group x (striding keeps the
// largest-first order balanced across XCDs).  The host tracks each
// counter's value.
constexpr int CTR_GROUPS = 8;
constexpr int CTR_STRIDE = 32;                                  // in uint64
constexpr size_t CTR_BYTES = (size_t)CTR_GROUPS * CTR_STRIDE * 8;
// The blocks of a launch that finalizes in its last block count themselves
// done on the uint64 at this index (in counter group 0's 256 bytes, a cache
// line away from its claim counter).
constexpr int CTR_DONE = 16;
struct CtrState {
    uint64_t base[CTR_GROUPS] = {};
    uint64_t done = 0;
};
inline uint32_t ctr_groups(int grid_blocks)
{
    uint32_t g = 1;
    while (g < (uint32_t)CTR_GROUPS && (int)(2 * g) <= grid_blocks) g *= 2;
    return g;
}
struct CtrArgs {                 // kernel argument (by value)
    uint64_t base[CTR_GROUPS];
    uint32_t groups;
    uint32_t runs;               // runs of items, computed on the host
    char *fin_out;               // fin_nmats > 0: every block stages matrices
    const char *fin_src;         //   0 .. fin_nmats from fin_src before walking;
    uint32_t fin_nmats;          //   with fin_out the last block to finish
    uint32_t pad;                //   also finalizes them into fin_out
    uint64_t done_base;          // the done counter's value before the launch
};

// Items are walked in runs of (BLOCK / WAVE) * grab consecutive items
// (grab >= 1), the block's waves taking every (BLOCK / WAVE)-th item of a
// run: block b walks run b first, then claims runs with one atomic each
// (several items per run keep tiny items from making the claims the
// bottleneck).  `state` holds the counters' values before the launch and
// is advanced past it.  With fin_nmats > 0 (the call's matrices being all of
// d_mats[0 .. fin_nmats)) every block first does launch_stage's work from
// fin_src, and the caller does not launch it: the blocks write the same bytes
// and each reads only after its own stores and barrier.  With fin_out as
// well the block that finishes last (the only one, for grid_blocks == 1)
// also does launch_finalize's work into fin_out, and the caller does not
// launch that either; with several blocks they count themselves done on
// ctr[CTR_DONE], whose value the host tracks in state->done.
int launch_walk(int variant, int n, bool kahan, bool fused, int nmax_fused,
                const WaveItem *d_items, uint32_t count, uint32_t grab, const MatDesc *d_mats,
                const void *stage, double *partials, unsigned long long *ctr,
                CtrState *state, int grid_blocks, void *stream, const void *fin_src = nullptr,
                void *fin_out = nullptr, int fin_nmats = 0);

// Items per atomic claim for items of at most 2^max_log2L steps per lane:
// enough that one claim is at least 64 lane-steps of walk, at most 16.
inline uint32_t grab_for(uint32_t max_log2L)
{
    return max_log2L >= 6 ? 1u : (max_log2L <= 2 ? 16u : (64u >> max_log2L));
}

// Largest resident blocks per CU for the walk kernel of (variant, n).
int walk_occupancy(int variant, int n, bool kahan, bool fused, int nmax_fused, int *blocks_per_cu);

// Finalize: per matrix, reduce its partial slots in a fixed order, apply
// 2^{-(n-1)} (floats) or inv(2)^{n-1} (F_p), and write the 16-byte result slot.
int launch_finalize(const MatDesc *d_mats, int nmats, const double *partials, void *out,
                    void *stream);

// Fused-kernel order buckets (a ragged batch with max order n uses the first
// bucket >= n).
constexpr int FUSED_BUCKETS[] = {16, 26};

}  // namespace permk
