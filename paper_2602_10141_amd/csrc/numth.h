// Host-side number theory for the CRT path (paper Sec. 2.1).
#pragma once
#include <stdint.h>

#include <vector>

namespace permh {

uint64_t powmod(uint64_t b, uint64_t e, uint64_t m);       // m < 2^32
bool is_prime_u32(uint32_t m);
std::vector<uint32_t> prime_factors(uint32_t n);
// Primitive n-th root of unity h^((p-1)/n) mod p for the smallest h >= 2 of
// exact order n; 0 if p != 1 (mod n).
uint32_t root_of_unity(int n, uint32_t p);
// The `count` smallest primes p = 1 (mod n) with 2^30 < p < 2^31, ascending.
std::vector<uint32_t> primes_1_mod_n(int n, int count);
// -p^{-1} mod 2^32 for odd p.
uint32_t mont_pprime(uint32_t p);
// What the F_p finalize step multiplies a residue sum of an order-n walk by:
// inv(2)^(n-1) against Glynn's 2^(n-1) (1 when `scaled` is false), times
// R^(n-1), R = 2^32, for Montgomery sums, whose products leave R^-(n-1).
uint32_t fp_finalize_factor(uint32_t p, int n, bool montgomery, bool scaled);

// Non-negative multi-limb integer, little-endian uint64 limbs, no leading zeros.
struct BigU {
    std::vector<uint64_t> limb;
    static BigU from(uint64_t v);
    void trim();
    void mul_small(uint64_t m);
    void add_small(uint64_t a);
    static BigU mul(const BigU &a, const BigU &b);
    static int cmp(const BigU &a, const BigU &b);
    static BigU sub(const BigU &a, const BigU &b);   // requires a >= b
};

// (prod primes)^2 > 4 n^n, i.e. prod primes > 2 n^{n/2}.
bool schur_bound_ok(int n, const std::vector<uint32_t> &primes);
// Garner: the X with X = res_i (mod p_i) and |X| < M/2; primes distinct odd primes.
bool garner_lift(const uint32_t *res, const uint32_t *primes, int k, BigU &mag, int &sign);
double log2_product(const uint32_t *primes, int k);

}  // namespace permh
