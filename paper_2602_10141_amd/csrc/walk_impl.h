// Gray-code Glynn walk kernels for gfx950 (CDNA4, wave64).
//
// What is computed (paper Sec. 1 Note, Sec. 2.2-2.3; Glynn's formula): for an
// n x n matrix A,
//
//   perm(A) = 2^{-(n-1)} * sum_{x=0}^{2^{n-1}-1} (-1)^x prod_{i<n} r_i(x),
//   r_i(x)  = a_{i0} + sum_{k=1}^{n-1} d_k(x) a_{ik},
//   d_k(x)  = 1 - 2 * bit_{k-1}(gray(x)),   gray(x) = x XOR (x >> 1).
//
// Going from x-1 to x flips gray bit b = ctz(x), i.e. column k = b + 1: all n
// row sums move by -2 a_{ik} when that bit turns on and by +2 a_{ik} when it
// turns off.  The product of the d_k equals (-1)^x.
//
// Work split (the paper's contiguous Gray-code blocks, Sec. 2.2): a wave item
// is 64 lanes, lane l walking the 2^c consecutive indices starting at
// x_l = x0 + l * 2^c with x0 a multiple of 2^c.  Because every x_l is aligned,
// at step j (0 < j < 2^c) all lanes flip the same column ctz(j)+1 in the same
// direction, except at j = 2^{c-1}, where the direction depends on bit c of
// x_l.  So the flip column is wave-uniform: the staging kernel stores +2A and
// -2A column by column, the walk picks the column with scalar arithmetic,
// reads it with scalar loads (s_load into SGPRs) and adds it to the per-lane
// row sums held in VGPRs (v_add_f64 with an SGPR operand): a flip is n adds
// and no branch.
//
// Per step each lane does: n adds (flip), an n-way product (four interleaved
// chains, then a fixed combining tree), and one signed accumulate.  For the
// floating-point fields the four terms of a group of steps (signs + - + -)
// are first combined as (t0 - t1) + (t2 - t3), which costs three adds and
// one compensated add per four terms instead of four compensated adds; the
// extra rounding is below the n roundings each term already carries.
//
//   V_C128  complex row sums; complex products with FMA; Kahan-compensated
//           sums of the real and imaginary parts (paper Sec. 1 Note).
//   V_F64   the same over R.
//   V_MODP  F_p with p < 2^31 odd.  Entries are taken as balanced residues
//           |a| <= (p-1)/2, so every row sum is an exact integer of magnitude
//           below n*p/2 < 2^36 and is never reduced.  Products are reduced by
//           an exact Barrett step in binary64: h = a*b rounded, l = fma(a,b,-h)
//           (the exact rounding error), q = rint(h * (1/p)), d = fma(-q,p,h)
//           (exact), result d + l, exactly congruent to a*b and of magnitude
//           below p.  The signed sum of a lane is an exact integer below 2^52.
//   V_MONT  F_p with uint32 residues in [0,p) and 32-bit Montgomery products
//           (R = 2^32); the n-1 products leave a factor R^{-(n-1)} that the
//           finalize step removes.
//
// Reduction: lane sums -> xor-butterfly across the wave -> one partial per
// wave item -> per matrix, a fixed-order block reduction in finalize.  No
// atomics touch the values, so results are bit-reproducible for a fixed
// partition of [0, 2^{n-1}).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

#include "kernels.h"

namespace permk {

template <typename T>
using sptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ sptr<T> sp(const void *p)
{
    return (sptr<T>)(p);
}

// Copy a descriptor with scalar loads (the struct is uniform across the wave).
template <typename T>
__device__ __forceinline__ T sload(const T *p)
{
    static_assert(sizeof(T) % 8 == 0, "descriptor size");
    uint64_t w[sizeof(T) / 8];
    sptr<uint64_t> q = sp<uint64_t>(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 8); ++i) w[i] = q[i];
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

// Hide a uniform pointer's provenance so that column loads stay inside the
// loop iteration that uses them (hoisting whole columns out of the loop would
// overflow the SGPR file).
__device__ __forceinline__ const char *opaque(const char *p)
{
    asm volatile("" : "+s"(p));
    return p;
}

__device__ __forceinline__ void kahan_add(double &s, double &c, double v)
{
    const double y = v - c;
    const double t = s + y;
    c = (t - s) - y;
    s = t;
}

__device__ __forceinline__ void cmul(double &ar, double &ai, double br, double bi)
{
    const double r = __builtin_fma(ar, br, -(ai * bi));
    const double i = __builtin_fma(ar, bi, ai * br);
    ar = r;
    ai = i;
}

// Exact a*b mod p as a balanced value, for integers |a|,|b| < 2^36, p < 2^31.
__device__ __forceinline__ double mulmod_f64(double a, double b, double p, double pinv)
{
    const double h = a * b;
    const double l = __builtin_fma(a, b, -h);
    const double q = __builtin_rint(h * pinv);
    const double d = __builtin_fma(-q, p, h);
    return d + l;
}

__device__ __forceinline__ uint32_t montmul(uint32_t a, uint32_t b, uint32_t p, uint32_t pp)
{
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * pp;
    const uint64_t u = (t + (uint64_t)m * p) >> 32;      // < 2p
    const uint32_t r = (uint32_t)u;
    return min(r, r - p);
}

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t p)
{
    const uint32_t s = a + b;                            // a, b < p < 2^31
    return min(s, s - p);
}

// Number of interleaved product chains.
template <int N>
struct Chains {
    static constexpr int K = N < 4 ? N : 4;
};

// Column entries held in SGPRs between steps (at most 80 of the 102 SGPRs).
constexpr int PF_MAX = 40;

// Order LDS writes of some lanes before reads of other lanes of the same
// wave.  A wave's LDS operations complete in program order, so this only
// keeps the compiler from moving memory operations across it.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row sums as binary64 values, common to the c128, f64 and F_p (Barrett)
// variants.  E = doubles per entry (2 for complex, 1 for real).  The staged
// buffer holds [+2A columns][-2A columns], each column n*E doubles.  PFN
// column entries are prefetched per step (0: none).
template <int N, int E, int PFN>
struct RealRows {
    double r[N * E];
    const char *cols;

    __device__ __forceinline__ sptr<double> col(int k, bool neg) const
    {
        return sp<double>(cols) + (neg ? N * N * E : 0) + N * E * k;
    }
    // Row sums at the lane's start index x.  Lane l of an item starts at
    // x0 + l 2^L with x0 a multiple of nl 2^L, so the Gray codes of the nl
    // active lanes differ only in bits L-1 .. h, h the highest bit in which
    // x0 and x0 + (nl - 1) 2^L differ: columns klo = max(L, 1) .. khi = h + 1
    // (seven for a full item).  Every other column enters every lane's sums
    // with the sign lane 0 gives it.  The wave therefore forms that common
    // part once, lane j summing value j of the N*E with coalesced loads that
    // are all in flight together, and hands it to every lane through LDS;
    // each lane then adds the varying columns with its own signs, read
    // through the scalar cache as in the walk.  Against every lane summing
    // all n columns from the scalar cache (n - 1 dependent rounds of column
    // loads), this takes about n + 7 N*E vector instructions instead of
    // n N*E, and seven rounds.  Lanes past nl get no valid sums (their
    // results are discarded).  lds_block: the block's exchange area, `stride`
    // (at least SEED_LDS) doubles per wave.
    static constexpr int SEED_LDS = N * E;
    __device__ __forceinline__ void seed(uint64_t x, uint64_t x0, uint32_t L, uint32_t nl,
                                         double *lds_block, int stride)
    {
        constexpr int V = N * E;
        constexpr int P = (V + WAVE - 1) / WAVE;    // values per lane
        // The lane and wave numbers are formed afresh in every seed: values
        // derived from them and kept across the walk loop would cost registers
        // the loop needs (they were spilled there).
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & (WAVE - 1);
        double *lds = lds_block + __builtin_amdgcn_readfirstlane(tid / WAVE) * stride;
        const uint64_t g = x ^ (x >> 1);
        const uint64_t g0 = x0 ^ (x0 >> 1);
        int klo = N, khi = N - 1;                   // no varying column
        if (nl > 1) {
            const uint64_t xe = x0 + ((uint64_t)(nl - 1) << L);
            klo = L > 0 ? (int)L : 1;
            khi = min(64 - __builtin_clzll(x0 ^ xe), N - 1);
        }
        const double *c = (const double *)cols;     // the +2A columns, V doubles each
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int j0 = lane + q * WAVE;
            const int j = j0 < V ? j0 : V - 1;
            double u = c[j];
#pragma unroll
            for (int k = 1; k < N; ++k) {
                const double d = (k >= klo && k <= khi) ? 0.0
                               : ((g0 >> (k - 1)) & 1) ? -1.0 : 1.0;
                u = __builtin_fma(d, c[V * k + j], u);
            }
            if (j0 < V) lds[j0] = 0.5 * u;
        }
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < V; ++i) r[i] = lds[i];
        wave_lds_sync();                            // read before the next seed writes
#pragma unroll 1
        for (int k = klo; k <= khi; ++k) {
            const double d = ((g >> (k - 1)) & 1) ? -0.5 : 0.5;
            sptr<double> ck = col(k, false);
#pragma unroll
            for (int i = 0; i < V; ++i) r[i] = __builtin_fma(d, ck[i], r[i]);
        }
    }
    __device__ __forceinline__ void flip(sptr<double> c)
    {
#pragma unroll
        for (int i = 0; i < N * E; ++i) r[i] += c[i];
    }
    // Software pipelining of the column loads: the first PF entries of the
    // next step's column are loaded into SGPRs while this step's product is
    // formed, and flip_pf adds them (loading the rest, if any, directly).
    static constexpr int PF = PFN;
    double pf[PF > 0 ? PF : 1];
    __device__ __forceinline__ void prefetch(sptr<double> c)
    {
#pragma unroll
        for (int i = 0; i < PF; ++i) pf[i] = c[i];
    }
    __device__ __forceinline__ void flip_pf(sptr<double> c)
    {
#pragma unroll
        for (int i = 0; i < PF; ++i) r[i] += pf[i];
#pragma unroll
        for (int i = PF; i < N * E; ++i) r[i] += c[i];
    }
    __device__ __forceinline__ void flip_lane(int k, bool up)
    {
        const double s = up ? 1.0 : -1.0;
        sptr<double> c = col(k, false);
#pragma unroll
        for (int i = 0; i < N * E; ++i) r[i] = __builtin_fma(s, c[i], r[i]);
    }
};

// ------------------------------------------------------------------- C128
// Prefetched column entries per variant.  F_p and c128 up to n = 20 (the
// whole column) were faster in same-device comparisons.  For c128 from
// n = 21 only part of the column fits; the depth per order is the deepest of
// 16, 24, 32, 40 entries whose walk loop the compiler keeps free of spills
// (the allocation changes erratically with the depth: 40 entries spilled at
// n = 22..28 and at most orders from 32, 32 at n = 24, 25, 27, 28), with the
// fewest waits per group; 16 is spill-free at every order from 21.
// The f64 walk, whose VGPR budget at its occupancy leaves no room for the
// earlier loads, was not faster with it.
template <int N>
struct PfC128 {
    static constexpr int n = 2 * N <= PF_MAX ? 2 * N
                           : N == 21 ? 40
                           : (N <= 23 || N == 26) ? 32
                           : N <= 28 ? 16
                           : N == 29 ? 32
                           : N <= 31 ? PF_MAX
                           : 16;
};

template <int N, bool KAHAN>
struct OpsC128 : RealRows<N, 2, PfC128<N>::n> {
    using RealRows<N, 2, PfC128<N>::n>::r;
    double sr, si, cr, ci;
    double gr, gi, hr, hi;      // the running group of four terms

    __device__ __forceinline__ void setup(const MatDesc &, const char *c)
    {
        this->cols = c;
        sr = si = cr = ci = 0.0;
    }
    __device__ __forceinline__ void product(double &pr, double &pi) const
    {
        constexpr int K = Chains<N>::K;
        double ar[K], ai[K];
#pragma unroll
        for (int c = 0; c < K; ++c) { ar[c] = r[2 * c]; ai[c] = r[2 * c + 1]; }
#pragma unroll
        for (int i = K; i < N; ++i) cmul(ar[i % K], ai[i % K], r[2 * i], r[2 * i + 1]);
#pragma unroll
        for (int w = 1; w < K; w *= 2)
#pragma unroll
            for (int c = 0; c + w < K; c += 2 * w) cmul(ar[c], ai[c], ar[c + w], ai[c + w]);
        pr = ar[0];
        pi = ai[0];
    }
    __device__ __forceinline__ void acc(double pr, double pi)
    {
        if (KAHAN) { kahan_add(sr, cr, pr); kahan_add(si, ci, pi); }
        else { sr += pr; si += pi; }
    }
    template <bool NEG>
    __device__ __forceinline__ void term()
    {
        double pr, pi;
        product(pr, pi);
        if (NEG) acc(-pr, -pi); else acc(pr, pi);
    }
    __device__ __forceinline__ void term_lane(bool neg)
    {
        double pr, pi;
        product(pr, pi);
        const double s = neg ? -1.0 : 1.0;
        acc(s * pr, s * pi);
    }
    // Step Q (0..3) of a group of four consecutive Gray steps, signs + - + -:
    // the group sum (t0 - t1) + (t2 - t3) enters the compensated sum once.
    template <int Q>
    __device__ __forceinline__ void gterm()
    {
        double pr, pi;
        if (Q == 0) { product(gr, gi); return; }
        if (Q == 2) { product(hr, hi); return; }
        product(pr, pi);
        if (Q == 1) { gr -= pr; gi -= pi; return; }
        hr -= pr;
        hi -= pi;
        acc(gr + hr, gi + hi);
    }
    __device__ __forceinline__ void result(double &a, double &b) const
    {
        a = KAHAN ? sr - cr : sr;
        b = KAHAN ? si - ci : si;
    }
    __device__ __forceinline__ void store(double *part, double a, double b) const
    {
        part[0] = a;
        part[1] = b;
    }
};

// -------------------------------------------------------------------- F64
template <int N, bool KAHAN, int PFN = 0>
struct OpsF64 : RealRows<N, 1, PFN> {
    using RealRows<N, 1, PFN>::r;
    double s, c;
    double g, h;                // the running group of four terms

    __device__ __forceinline__ void setup(const MatDesc &, const char *cc)
    {
        this->cols = cc;
        s = c = 0.0;
    }
    __device__ __forceinline__ double product() const
    {
        constexpr int K = Chains<N>::K;
        double a[K];
#pragma unroll
        for (int q = 0; q < K; ++q) a[q] = r[q];
#pragma unroll
        for (int i = K; i < N; ++i) a[i % K] *= r[i];
#pragma unroll
        for (int w = 1; w < K; w *= 2)
#pragma unroll
            for (int q = 0; q + w < K; q += 2 * w) a[q] *= a[q + w];
        return a[0];
    }
    __device__ __forceinline__ void acc(double v)
    {
        if (KAHAN) kahan_add(s, c, v); else s += v;
    }
    template <bool NEG>
    __device__ __forceinline__ void term()
    {
        const double v = product();
        acc(NEG ? -v : v);
    }
    __device__ __forceinline__ void term_lane(bool neg)
    {
        const double v = product();
        acc(neg ? -v : v);
    }
    template <int Q>
    __device__ __forceinline__ void gterm()
    {
        if (Q == 0) { g = product(); return; }
        if (Q == 2) { h = product(); return; }
        const double v = product();
        if (Q == 1) { g -= v; return; }
        h -= v;
        acc(g + h);
    }
    __device__ __forceinline__ void result(double &a, double &b) const
    {
        a = KAHAN ? s - c : s;
        b = 0.0;
    }
    __device__ __forceinline__ void store(double *part, double a, double) const
    {
        part[0] = a;
        part[1] = 0.0;
    }
};

// ------------------------------------------------------ F_p, FP64 Barrett
__device__ __forceinline__ double reduce_to_range(double v, double p, double pinv)
{
    // v an integer with |v| < 2^52: return v mod p in [0, p)
    const double q = __builtin_rint(v * pinv);
    double r = __builtin_fma(-q, p, v);
    if (r < 0.0) r += p;
    if (r >= p) r -= p;
    return r;
}

// F_p prefetches the whole column up to 40 entries, 32 at the orders where
// 40 left the walk loop spilling registers (43, 46, 47).
template <int N>
struct PfModp {
    static constexpr int n = (N == 43 || N == 46 || N == 47) ? 32 : (N < PF_MAX ? N : PF_MAX);
};

template <int N>
struct OpsModp : RealRows<N, 1, PfModp<N>::n> {
    using RealRows<N, 1, PfModp<N>::n>::r;
    double s;
    double p, pinv;

    __device__ __forceinline__ void setup(const MatDesc &md, const char *cc)
    {
        this->cols = cc;
        s = 0.0;
        p = (double)md.p;
        pinv = md.pinv;
    }
    __device__ __forceinline__ double product() const
    {
        constexpr int K = Chains<N>::K;
        double a[K];
#pragma unroll
        for (int q = 0; q < K; ++q) a[q] = r[q];
#pragma unroll
        for (int i = K; i < N; ++i) a[i % K] = mulmod_f64(a[i % K], r[i], p, pinv);
#pragma unroll
        for (int w = 1; w < K; w *= 2)
#pragma unroll
            for (int q = 0; q + w < K; q += 2 * w) a[q] = mulmod_f64(a[q], a[q + w], p, pinv);
        return a[0];
    }
    template <bool NEG>
    __device__ __forceinline__ void term()
    {
        const double v = product();
        s = NEG ? s - v : s + v;
    }
    __device__ __forceinline__ void term_lane(bool neg)
    {
        const double v = product();
        s = neg ? s - v : s + v;
    }
    template <int Q>
    __device__ __forceinline__ void gterm() { term<(Q & 1) != 0>(); }
    __device__ __forceinline__ void result(double &a, double &b) const
    {
        // For N == 1 the "product" is the unreduced row sum itself.
        a = reduce_to_range(s, p, pinv);
        b = 0.0;
    }
    __device__ __forceinline__ void store(double *part, double a, double) const
    {
        part[0] = reduce_to_range(a, p, pinv);     // wave sum < 64 p
        part[1] = 0.0;
    }
};

// ------------------------------------------------- F_p, 32-bit Montgomery
template <int N>
struct OpsMont {
    uint32_t r[N];
    uint64_t spos, sneg;
    uint32_t p, pp;
    const char *cols;

    __device__ __forceinline__ void setup(const MatDesc &md, const char *cc)
    {
        cols = cc;
        spos = sneg = 0;
        p = md.p;
        pp = md.mont_pp;
    }
    // staged arrays: [2a mod p][(p - 2a) mod p][a][(p - a) mod p], column-major
    __device__ __forceinline__ sptr<uint32_t> col(int k, bool neg) const
    {
        return sp<uint32_t>(cols) + (neg ? N * N : 0) + N * k;
    }
    __device__ __forceinline__ sptr<uint32_t> aval(int k, bool neg) const
    {
        return sp<uint32_t>(cols) + (neg ? 3 * N * N : 2 * N * N) + N * k;
    }
    // Each lane sums its own start (the item's layout is not used).
    static constexpr int SEED_LDS = 0;
    __device__ __forceinline__ void seed(uint64_t x, uint64_t, uint32_t, uint32_t, double *, int)
    {
        const uint64_t g = x ^ (x >> 1);
        sptr<uint32_t> c0 = aval(0, false);
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = c0[i];
#pragma unroll 1
        for (int k = 1; k < N; ++k) {
            const bool neg = (g >> (k - 1)) & 1;
            sptr<uint32_t> ca = aval(k, false);
            sptr<uint32_t> cn = aval(k, true);
#pragma unroll
            for (int i = 0; i < N; ++i) r[i] = addmod(r[i], neg ? cn[i] : ca[i], p);
        }
    }
    __device__ __forceinline__ void flip(sptr<uint32_t> c)
    {
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = addmod(r[i], c[i], p);
    }
    static constexpr int PF = N;
    uint32_t pf[N];                 // the next step's column (see RealRows)
    __device__ __forceinline__ void prefetch(sptr<uint32_t> c)
    {
#pragma unroll
        for (int i = 0; i < N; ++i) pf[i] = c[i];
    }
    __device__ __forceinline__ void flip_pf(sptr<uint32_t>)
    {
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = addmod(r[i], pf[i], p);
    }
    __device__ __forceinline__ void flip_lane(int k, bool up)
    {
        sptr<uint32_t> cp = col(k, false);
        sptr<uint32_t> cm = col(k, true);
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = addmod(r[i], up ? cp[i] : cm[i], p);
    }
    __device__ __forceinline__ uint32_t product() const
    {
        constexpr int K = Chains<N>::K;
        uint32_t a[K];
#pragma unroll
        for (int q = 0; q < K; ++q) a[q] = r[q];
#pragma unroll
        for (int i = K; i < N; ++i) a[i % K] = montmul(a[i % K], r[i], p, pp);
#pragma unroll
        for (int w = 1; w < K; w *= 2)
#pragma unroll
            for (int q = 0; q + w < K; q += 2 * w) a[q] = montmul(a[q], a[q + w], p, pp);
        return a[0];
    }
    template <bool NEG>
    __device__ __forceinline__ void term()
    {
        const uint32_t v = product();
        if (NEG) sneg += v; else spos += v;
    }
    __device__ __forceinline__ void term_lane(bool neg)
    {
        const uint32_t v = product();
        spos += neg ? 0u : v;
        sneg += neg ? v : 0u;
    }
    template <int Q>
    __device__ __forceinline__ void gterm() { term<(Q & 1) != 0>(); }
    __device__ __forceinline__ void result(double &a, double &b) const
    {
        const uint64_t P = p;
        a = (double)((spos % P + P - sneg % P) % P);
        b = 0.0;
    }
    __device__ __forceinline__ void store(double *part, double a, double) const
    {
        part[0] = (double)((uint64_t)a % (uint64_t)p);
        part[1] = 0.0;
    }
};

template <int V, int N, bool K> struct OpsFor;
template <int N, bool K> struct OpsFor<V_C128, N, K> { using type = OpsC128<N, K>; };
// f64 prefetches the whole column at orders 16..28 (at four waves per SIMD,
// below), elsewhere none (see Occupancy).
template <int N>
struct PfF64 {
    static constexpr int n = (N >= 16 && N <= 28) ? N : 0;
};
template <int N, bool K> struct OpsFor<V_F64, N, K> { using type = OpsF64<N, K, PfF64<N>::n>; };
template <int N, bool K> struct OpsFor<V_MODP, N, K> { using type = OpsModp<N>; };
template <int N, bool K> struct OpsFor<V_MONT, N, K> { using type = OpsMont<N>; };

// ------------------------------------------------------------- the walk
// Steps j = 4m .. 4m+3 of a lane's chunk (m > 0, j != L/2).  Steps 4m+1 and
// 4m+3 flip column 1 (down, then up); step 4m+2 flips column 2, down for even
// m and up for odd m; step 4m flips column b+1 with b = ctz(4m), up exactly
// when bit b+1 of j is set.
// Keep each step's instructions between step boundaries: letting the
// scheduler pull future steps' scalar loads forward overflows the SGPR file.
// Instead each step loads the next step's column by hand (prefetch) right
// after its own adds, so the loads are in flight during its product.
__device__ __forceinline__ void step_boundary() { __builtin_amdgcn_sched_barrier(0); }

// The column flipped by the first step of group m (0 < m, 4m != L/2).  For
// 4m = L/2 and 4m = L it still names a column of the matrix (c + 1 <= n - 6,
// since a wave item never exceeds 2^(n-1) indices): the last group before
// either prefetches it unconditionally, without a branch that would let the
// compiler move the step's code past its boundaries, and does not use it.
template <class Ops>
__device__ __forceinline__ auto first_col(const Ops &S, uint32_t m)
{
    const uint32_t j = m << 2;
    const uint32_t b = __builtin_ctz(j);
    return S.col(b + 1, !((j >> (b + 1)) & 1));
}

// One Gray step: add the prefetched column `cur`, start loading `nxt`, then
// form the term.
template <int Q, class Ops, class C>
__device__ __forceinline__ void pstep(Ops &S, C cur, C nxt)
{
    S.flip_pf(cur);
    S.prefetch(nxt);
    if (Ops::PF > 0) step_boundary();   // the loads go out before the product
    S.template gterm<Q>();
    step_boundary();
}

// Steps 4m+1 .. 4m+3; the last one prefetches `nxt`, the column of the next
// group's first step.
template <class Ops, class C>
__device__ __forceinline__ void group_rest(Ops &S, uint32_t m, C nxt)
{
    pstep<1>(S, S.col(1, true), S.col(2, !(m & 1)));
    pstep<2>(S, S.col(2, !(m & 1)), S.col(1, false));
    pstep<3>(S, S.col(1, false), nxt);
}

// Group m (0 < m, 4m != L/2).
template <class Ops>
__device__ __forceinline__ void group(Ops &S, const char *cols, uint32_t m)
{
    S.cols = opaque(cols);
    pstep<0>(S, first_col(S, m), S.col(1, true));
    group_rest(S, m, first_col(S, m + 1));
}

// One lane of item `it`: seed at xl, then the 2^c - 1 Gray steps of its
// chunk (c = it.log2L).
template <class Ops>
__device__ __forceinline__ void walk_lane(Ops &S, const WaveItem &it, uint64_t xl,
                                          double *lds_block, int stride)
{
    const uint32_t c = it.log2L;
    const char *cols = S.cols;
    S.seed(xl, it.x0, c, it.nlanes, lds_block, stride);
    if (c >= 3) {
        const uint32_t G = 1u << (c - 2);      // groups of four steps
        const uint32_t H = G >> 1;             // the group holding j = L/2
        // group 0: step 0 is the seed's own term
        S.prefetch(S.col(1, true));
        S.template gterm<0>();
        step_boundary();
        group_rest(S, 0, first_col(S, 1));
#pragma unroll 1
        for (uint32_t m = 1; m < H; ++m) group(S, cols, m);
        // j = L/2: column c, direction from bit c of the lane's start index.
        S.cols = opaque(cols);
        S.flip_lane(c, (xl >> c) & 1);
        S.prefetch(S.col(1, true));
        S.template gterm<0>();
        step_boundary();
        group_rest(S, H, first_col(S, H + 1));
#pragma unroll 1
        for (uint32_t m = H + 1; m < G; ++m) group(S, cols, m);
    } else {
        // Chunks of 1, 2 or 4 indices (tiny matrices, range ends): take the
        // direction and sign of every step from the lane's own index.
        S.term_lane(xl & 1);
#pragma unroll 1
        for (uint32_t j = 1; j < (1u << c); ++j) {
            const uint32_t b = __builtin_ctz(j);
            const uint64_t x = xl + j;
            S.flip_lane(b + 1, (x >> (b + 1)) & 1);
            S.term_lane(x & 1);
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

template <class Ops>
__device__ __forceinline__ void run_item(const WaveItem &it, const MatDesc &md, const char *stage,
                                         double *partials, int lane, double *lds_block,
                                         int stride)
{
    Ops S;
    S.setup(md, stage + md.stage_off);
    // the lane's start index, its 64-bit lane offset formed afresh per item
    // (kept across the item loop, it was spilled there)
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const uint64_t xl = it.x0 + ((uint64_t)(uint32_t)ln << it.log2L);
    walk_lane(S, it, xl, lds_block, stride);
    double a, b;
    S.result(a, b);
    if ((uint32_t)lane >= it.nlanes) { a = 0.0; b = 0.0; }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) S.store(partials + 2 * (size_t)it.slot, a, b);
}

// Fetch the next wave item index, uniform across the wave.  Every lane
// executes the atomic (lane 0 adds 1, the others 0) so that no divergent
// branch precedes the readfirstlane: with the add under `if (lane == 0)` the
// compiler may thread that branch into the loop's other lane-0 branch and
// leave lanes 1..63 in a loop that re-reads a stale index.
__device__ __forceinline__ uint32_t next_item(unsigned long long *ctr, uint64_t base, int lane)
{
    const unsigned long long got = atomicAdd(ctr, lane == 0 ? 1ull : 0ull);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(got - base));
    return lo;
}

// Waves per SIMD asked of the compiler for each variant and order.  The
// budgets come from a sweep on gfx950: a larger budget lets the scheduler
// overlap consecutive steps with registers that cost occupancy, a smaller one
// makes it spill the row sums around the per-item seed.  c128 runs best at 3
// waves for n = 20..28; F_p (Barrett) runs at 3 waves from n = 21 up to 48
// (the walk loop stays free of spills; from n = 36 the per-item seed
// spills, once per item) and F_p (Montgomery) at 4 compiles without spills;
// both run as fast as any setting measured.  f64 at orders 16..28 runs at 4
// waves with the whole column prefetched (as in the fused kernel), which
// keeps its walk loop free of spills: against 5..8 waves without prefetch a
// batch of 50,000 O(20) walked 3% faster and single calls 9-17%; batches
// of orders 10..13 were 3-9% slower that way and keep the occupancy, as do
// orders from 29 (2% slower at 32).
template <int V, int N>
struct Occupancy {
    static constexpr int clamp(int w) { return w < 1 ? 1 : (w > 8 ? 8 : w); }
    static constexpr int waves =
        V == V_C128 ? clamp(512 / (4 * N + 56))
      : V == V_MODP ? (N > 20 ? 3 : N > 12 ? 4 : clamp(512 / (2 * N + 44)))
      : V == V_F64  ? (N >= 16 && N <= 28 ? 4 : clamp(512 / (2 * N + 32)))
                    : (N > 40 ? 3 : 4);
};

// ----------------------------------------------------------------- staging
// Staged layout, column-major (column k, row i at k*n + i):
//   c128, f64, F_p (Barrett): [+2A][-2A] as binary64 (complex: re, im pairs);
//                             F_p entries are first mapped to balanced
//                             residues in [-(p-1)/2, (p-1)/2];
//   F_p (Montgomery):         [2a mod p][(p - 2a) mod p][a][(p - a) mod p] as uint32.
// Entries of F_p matrices are reduced mod p first.
__device__ inline void stage_one(const MatDesc md, const char *src, char *stage)
{
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
// Per matrix, with the 256 threads of a block: reduce its partial slots in a
// fixed order (strided compensated sums, then a fixed tree), apply
// 2^{-(n-1)} (floats) or the host's factor md.fin_scale (F_p: inv(2)^{n-1},
// and for Montgomery R^{n-1} against the R^{-(n-1)} its products leave),
// write the 16-byte result slot (only its first 8 or 4 bytes with MD_OUT_8
// or MD_OUT_4: a caller's f64 or F_p output written in place).  Shared by
// finalize_kernel and by walk launches that finalize their own matrices, so
// the two give identical bits.  sa, sb, su: 256 entries each in LDS.

static_assert(BLOCK == 256, "finalize_one reduces with 256 threads");
__device__ inline void finalize_one(const MatDesc md, const double *partials, char *out,
                                    double *sa, double *sb, unsigned long long *su)
{
    const int t = threadIdx.x;
    const bool modp = md.variant == V_MODP || md.variant == V_MONT;
    char *o = out + 16 * (size_t)md.out_slot;

    if (md.num_parts == 0) {                // n = 0: the empty permanent is 1
        if (t == 0) {
            if (modp) {
                ((uint32_t *)o)[0] = 1u % md.p;
                if (!(md.flags & MD_OUT_4))
                    ((uint32_t *)o)[1] = ((uint32_t *)o)[2] = ((uint32_t *)o)[3] = 0u;
            } else {
                ((double *)o)[0] = 1.0;
                if (!(md.flags & MD_OUT_8)) ((double *)o)[1] = 0.0;
            }
        }
        return;
    }
    if (modp) {
        const uint64_t P = md.p;
        uint64_t acc = 0;
        for (uint32_t q = t; q < md.num_parts; q += 256) {
            acc += (uint64_t)partials[2 * ((size_t)md.first_part + q)];
            if (acc >= (1ull << 62)) acc %= P;
        }
        su[t] = acc % P;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (t < w) {                    // both below P < 2^31: one subtraction reduces
                const unsigned long long v = su[t] + su[t + w];
                su[t] = v >= P ? v - P : v;
            }
            __syncthreads();
        }
        if (t == 0) {
            const uint64_t v = (su[0] * (uint64_t)md.fin_scale) % P;
            ((uint32_t *)o)[0] = (uint32_t)v;
            if (!(md.flags & MD_OUT_4))
                ((uint32_t *)o)[1] = ((uint32_t *)o)[2] = ((uint32_t *)o)[3] = 0u;
        }
        return;
    }
    // Floats: per-thread compensated sums over a fixed stride, then a fixed tree.
    double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
    for (uint32_t q = t; q < md.num_parts; q += 256) {
        const double *pp = partials + 2 * ((size_t)md.first_part + q);
        kahan_add(s0, c0, pp[0]);
        kahan_add(s1, c1, pp[1]);
    }
    sa[t] = s0 - c0;
    sb[t] = s1 - c1;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) { sa[t] += sa[t + w]; sb[t] += sb[t + w]; }
        __syncthreads();
    }
    if (t == 0) {
        double a = sa[0], b = sb[0];
        if (!(md.flags & MD_NO_SCALE)) {
            a = __builtin_ldexp(a, -(md.n - 1));
            b = __builtin_ldexp(b, -(md.n - 1));
        }
        ((double *)o)[0] = a;
        if (!(md.flags & MD_OUT_8)) ((double *)o)[1] = md.variant == V_C128 ? b : 0.0;
    }
}


// Block-level claims.  Block b first walks run b (the grid never exceeds the
// number of runs), so a launch with no more runs than blocks, such as one
// small matrix, makes no atomic at all; in a larger launch wave 0 of the
// block then claims further runs of WPB * grab consecutive wave items from
// its counter and publishes each in LDS.  Wave w takes the items w, w + WPB,
// w + 2 WPB, ... of a run.  Consecutive items belong to the same matrix (the
// host orders them so), so the four waves of a block walk one matrix side by
// side and its columns are shared in the CU's scalar cache; with one claim
// per wave, the waves of a CU walked as many different matrices as there
// were waves and the scalar cache missed on about half of the column loads
// in batches.  Counter x (of `groups`, serving the blocks b = x mod groups)
// hands out the runs x + groups * (nb + k), k = 0, 1, ..., where nb is the
// number of blocks in group x (their first runs were static).  The LDS slot
// is double-buffered: the slot written for claim i + 2 is read for claim i
// before every wave passes the barrier of claim i + 1, so one barrier per
// claim suffices.
constexpr uint32_t WPB = BLOCK / WAVE;

struct BlockClaims {
    unsigned long long *c;
    uint64_t base;
    uint32_t x, groups, nb, runs, wave, parity;
    uint32_t *slot;                 // two uint32 in LDS

    __device__ __forceinline__ uint32_t next(int lane)
    {
        if (wave == 0) {
            const uint64_t r = x + (uint64_t)groups * (nb + next_item(c, base, lane));
            slot[parity] = r < runs ? (uint32_t)r : runs;
        }
        __syncthreads();
        const uint32_t r = __builtin_amdgcn_readfirstlane(slot[parity]);
        parity ^= 1u;
        return r;
    }
};

// Scalar operations only, so that the counter address and the loop bounds
// stay in SGPRs (a divide would run on the VALU and hold them in VGPRs,
// which the walk needs for its row sums); groups is a power of two.
__device__ __forceinline__ BlockClaims block_claims(unsigned long long *ctr, const CtrArgs &ca,
                                                    uint32_t *slot)
{
    const uint32_t x = blockIdx.x & (ca.groups - 1);
    const uint32_t nb = (gridDim.x - x + ca.groups - 1) >> __builtin_ctz(ca.groups);
    return BlockClaims{ctr + CTR_STRIDE * x, ca.base[x], x, ca.groups, nb, ca.runs,
                       (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), 0u, slot};
}

// Walk the runs of this block: the static first one, then claimed ones (one
// loop, so that the walk's code is instantiated once).
template <class F>
__device__ __forceinline__ void for_each_run(BlockClaims &bc, int lane, F &&walk_run)
{
    const bool claims = bc.runs > gridDim.x;
    for (uint32_t r = blockIdx.x; r < bc.runs; r = claims ? bc.next(lane) : bc.runs) walk_run(r);
}

// Wait until this wave's vector stores are written to L2.  The workgroup
// barrier does not (it waits for LDS and scalar operations only), which is
// enough for the vector loads of other waves of the CU, but not for scalar
// loads, which reach L2 through the scalar cache.
__device__ __forceinline__ void wait_stores()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// A launch over a few small matrices stages them in every block before
// walking, saving the stage launch; one that is the whole call (a single
// small matrix, or a few tiny ones) also finalizes them afterwards, in the
// block that finishes last, saving the finalize launch.  The blocks write
// the same bytes.  Every wave's stores reach L2 before the block's barrier,
// and its waves read the staged columns only after that barrier, from this
// XCD's L2, which then holds the block's own write or another block's
// identical one; the scalar and vector L1 caches start every dispatch
// empty, so a line they hold was fetched after some block of the XCD had
// written it.
__device__ __forceinline__ void stage_in_walk(const CtrArgs &ca, const MatDesc *mats,
                                              const char *stage)
{
    if (!ca.fin_nmats) return;
    for (uint32_t m = 0; m < ca.fin_nmats; ++m)
        stage_one(mats[m], ca.fin_src, const_cast<char *>(stage));
    wait_stores();
    __syncthreads();
}

// With several blocks, each counts itself done on ctr[CTR_DONE] once its
// waves' partials are in L2: wave 0 releases at device scope (writing the
// XCD's L2 back to memory) in the atomic, and the block that takes the last
// count acquires (dropping its stale L1 and L2 lines) before it reads the
// other blocks' partials.  One release per block: a device-scope fence in
// every wave, after each item, cost more than the finalize launch it saved.
__device__ __forceinline__ void finalize_in_walk(const CtrArgs &ca, const MatDesc *mats,
                                                 const double *partials,
                                                 unsigned long long *ctr)
{
    if (!ca.fin_nmats || !ca.fin_out) return;
    __shared__ double sa[256], sb[256];
    __shared__ unsigned long long su[256];
    if (gridDim.x > 1) {
        __shared__ uint32_t last;
        wait_stores();
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long before = __hip_atomic_fetch_add(
                ctr + CTR_DONE, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            last = before - ca.done_base == gridDim.x - 1u;
        }
        __syncthreads();
        if (!last) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    for (uint32_t m = 0; m < ca.fin_nmats; ++m) {
        __syncthreads();
        finalize_one(mats[m], partials, ca.fin_out, sa, sb, su);
    }
}

// Persistent kernel over the host's item list (largest items first).  W > 0
// overrides the waves-per-SIMD target (used when tuning the budgets).
template <int V, int N, bool KAHAN, int W = 0>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(W > 0 ? W : Occupancy<V, N>::waves, 8)))
void walk_kernel(const WaveItem *items, uint32_t count, uint32_t grab,
                                                     const MatDesc *mats, const char *stage,
                                                     double *partials, unsigned long long *ctr,
                                                     CtrArgs ca)
{
    using Ops = typename OpsFor<V, N, KAHAN>::type;
    constexpr int SL = Ops::SEED_LDS > 0 ? Ops::SEED_LDS : 1;
    __shared__ uint32_t slot[2];
    __shared__ double seed_lds[WPB * SL];
    const int lane = threadIdx.x & (WAVE - 1);
    stage_in_walk(ca, mats, stage);
    stage = opaque(stage);              // no column load moves above the staging
    BlockClaims bc = block_claims(ctr, ca, slot);
    const uint32_t per_run = WPB * grab;
    for_each_run(bc, lane, [&](uint32_t r) __attribute__((always_inline)) {
        r = __builtin_amdgcn_readfirstlane(r);
        const uint32_t end = (uint32_t)min((uint64_t)count, ((uint64_t)r + 1) * per_run);
        for (uint32_t idx = r * per_run + bc.wave; idx < end; idx += WPB) {
            const WaveItem it = sload(items + idx);
            const MatDesc md = sload(mats + it.mat);
            run_item<Ops>(it, md, stage, partials, lane, seed_lds, SL);
        }
    });
    finalize_in_walk(ca, mats, partials, ctr);
}

// Fused kernel: any mix of c128 / f64 / F_p (Barrett) matrices of order <= NF.
template <int N, bool KAHAN>
__device__ __forceinline__ void run_variant(int v, const WaveItem &it, const MatDesc &md,
                                            const char *stage, double *partials, int lane,
                                            double *lds_block, int stride)
{
    if (v == V_C128) run_item<OpsC128<N, KAHAN>>(it, md, stage, partials, lane, lds_block, stride);
    else if (v == V_F64)    // at the fused kernel's 3 waves f64 has registers for the prefetch
        run_item<OpsF64<N, KAHAN, (N < PF_MAX ? N : PF_MAX)>>(it, md, stage, partials, lane,
                                                              lds_block, stride);
    else run_item<OpsModp<N>>(it, md, stage, partials, lane, lds_block, stride);
}

template <bool KAHAN, int... Ns>
__device__ __forceinline__ void run_fused(std::integer_sequence<int, Ns...>, int n, int v,
                                          const WaveItem &it, const MatDesc &md, const char *stage,
                                          double *partials, int lane, double *lds_block,
                                          int stride)
{
    (void)((n == Ns + 1 ? (run_variant<Ns + 1, KAHAN>(v, it, md, stage, partials, lane, lds_block,
                                                      stride), true)
                        : false) || ...);
}

template <int NF, bool KAHAN>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(Occupancy<V_C128, NF>::waves, 8)))
void walk_fused(const WaveItem *items, uint32_t count, uint32_t grab,
                                                    const MatDesc *mats, const char *stage,
                                                    double *partials, unsigned long long *ctr,
                                                    CtrArgs ca)
{
    // the largest seed exchange of the orders and variants it runs (c128, NF)
    constexpr int SL = OpsC128<NF, KAHAN>::SEED_LDS;
    __shared__ uint32_t slot[2];
    __shared__ double seed_lds[WPB * SL];
    const int lane = threadIdx.x & (WAVE - 1);
    stage_in_walk(ca, mats, stage);
    stage = opaque(stage);              // no column load moves above the staging
    BlockClaims bc = block_claims(ctr, ca, slot);
    const uint32_t per_run = WPB * grab;
    for_each_run(bc, lane, [&](uint32_t r) __attribute__((always_inline)) {
        r = __builtin_amdgcn_readfirstlane(r);
        const uint32_t end = (uint32_t)min((uint64_t)count, ((uint64_t)r + 1) * per_run);
        for (uint32_t idx = r * per_run + bc.wave; idx < end; idx += WPB) {
            const WaveItem it = sload(items + idx);
            const MatDesc md = sload(mats + it.mat);
            run_fused<KAHAN>(std::make_integer_sequence<int, NF>{}, md.n, md.variant, it, md,
                             stage, partials, lane, seed_lds, SL);
        }
    });
    finalize_in_walk(ca, mats, partials, ctr);
}

// ------------------------------------------------ instantiation tables
using WalkFn = void (*)(const WaveItem *, uint32_t, uint32_t, const MatDesc *, const char *,
                        double *, unsigned long long *, CtrArgs);

template <int V, bool K, int LO, int... Ns>
inline WalkFn walk_fn_range(int n, std::integer_sequence<int, Ns...>)
{
    static const WalkFn tab[] = {&walk_kernel<V, LO + Ns, K>...};
    const int i = n - LO;
    return (i >= 0 && i < (int)sizeof...(Ns)) ? tab[i] : nullptr;
}

// Defined in the walk_inst_*.hip translation units (compiled in parallel).
WalkFn walk_fn_c128_lo(int n, bool kahan);   // n = 1..24
WalkFn walk_fn_c128_hi(int n, bool kahan);   // n = 25..48
WalkFn walk_fn_f64(int n, bool kahan);
WalkFn walk_fn_modp(int n);
WalkFn walk_fn_mont(int n);
WalkFn walk_fn_fused16_k();
WalkFn walk_fn_fused16_nok();
WalkFn walk_fn_fused26_k();
WalkFn walk_fn_fused26_nok();

}  // namespace permk
