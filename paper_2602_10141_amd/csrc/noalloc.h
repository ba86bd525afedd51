// Interface between the host library and noalloc.hip (the static scratch of
// perm_c128_noalloc).  Not part of the public C ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace permk {

// Size of the per-device static scratch: counters, one descriptor, up to
// 32,768 wave items with their partial sums and the staged columns of one
// complex matrix of order 32, rounded up.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)2 << 20;
constexpr int NOALLOC_NMAX = 32;

// Byte offsets inside the scratch.
struct NoallocLayout {
    size_t ctr, mat, items, partials, stage, total;
};

// Device address of the scratch on `device`; call with that device current.
// Returns a hipError_t as int.
int noalloc_scratch_init(int device, void **ptr);

// Offsets for a c128 matrix of order n split into `count` wave items;
// returns 0 if they fit in NOALLOC_SCRATCH_BYTES, -1 otherwise.
int noalloc_layout(int n, uint32_t count, NoallocLayout *L);

// Launch the kernel that writes the descriptor and items into the scratch at
// `base` and zeroes its counters (n = 0: writes perm = 1 to out instead).
int launch_noalloc_plan(void *base, const NoallocLayout *L, uint32_t count, int n, uint32_t log2L,
                        uint32_t nlanes, uint32_t flags, double *out, void *stream);

}  // namespace permk
