// Host-side number theory for the CRT path (paper Sec. 2.1): primality,
// primes p = 1 (mod n), primitive n-th roots of unity mod p, Schur residue
// matrices, Montgomery constants and the Garner lift of residues to a signed
// multi-limb integer.  Pure C++; no device code.
#include "numth.h"

#include <algorithm>
#include <cmath>

namespace permh {

static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (a * b) % m; }  // m < 2^32

uint64_t powmod(uint64_t b, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    b %= m;
    while (e) {
        if (e & 1) r = mulmod64(r, b, m);
        b = mulmod64(b, b, m);
        e >>= 1;
    }
    return r;
}

uint32_t fp_finalize_factor(uint32_t p, int n, bool montgomery, bool scaled)
{
    if (p < 3) return 0;
    const uint64_t e = n > 1 ? (uint64_t)(n - 1) : 0;
    uint64_t f = 1;
    if (montgomery) f = powmod((1ull << 32) % p, e, p);
    if (scaled) f = mulmod64(f, powmod((p + 1) / 2, e, p), p);
    return (uint32_t)f;
}

// Deterministic Miller-Rabin for m < 2^32 (bases 2, 3, 5, 7 suffice below 3.2e9).
bool is_prime_u32(uint32_t m)
{
    if (m < 2) return false;
    static const uint32_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint32_t q : small) {
        if (m == q) return true;
        if (m % q == 0) return false;
    }
    uint32_t d = m - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; ++s; }
    for (uint32_t a : {2u, 3u, 5u, 7u}) {
        uint64_t x = powmod(a, d, m);
        if (x == 1 || x == m - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod64(x, x, m);
            if (x == m - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

std::vector<uint32_t> prime_factors(uint32_t n)
{
    std::vector<uint32_t> out;
    for (uint32_t d = 2; (uint64_t)d * d <= n; ++d)
        if (n % d == 0) {
            out.push_back(d);
            while (n % d == 0) n /= d;
        }
    if (n > 1) out.push_back(n);
    return out;
}

uint32_t root_of_unity(int n, uint32_t p)
{
    if (n < 1 || (p - 1) % (uint32_t)n) return 0;
    const std::vector<uint32_t> qs = n > 1 ? prime_factors((uint32_t)n) : std::vector<uint32_t>{};
    for (uint64_t h = 2; h < p; ++h) {
        const uint64_t g = powmod(h, (p - 1) / (uint32_t)n, p);
        bool ok = true;
        for (uint32_t q : qs)
            if (powmod(g, (uint32_t)n / q, p) == 1) { ok = false; break; }
        if (ok) return (uint32_t)g;
    }
    return 0;
}

std::vector<uint32_t> primes_1_mod_n(int n, int count)
{
    std::vector<uint32_t> out;
    const uint64_t lo = 1ull << 30, hi = 1ull << 31;
    uint64_t p = lo + 1;
    p += ((uint64_t)n - (p - 1) % (uint64_t)n) % (uint64_t)n;   // p = 1 (mod n)
    for (; p < hi && (int)out.size() < count; p += (uint64_t)n)
        if (p > lo && is_prime_u32((uint32_t)p)) out.push_back((uint32_t)p);
    return out;
}

uint32_t mont_pprime(uint32_t p)
{
    uint32_t inv = p;                       // Newton: correct to 3 bits for odd p
    for (int i = 0; i < 5; ++i) inv *= 2u - p * inv;
    return 0u - inv;                        // -p^{-1} mod 2^32
}

// ------------------------------------------------------------ big integers
void BigU::trim()
{
    while (!limb.empty() && limb.back() == 0) limb.pop_back();
}

BigU BigU::from(uint64_t v)
{
    BigU b;
    if (v) b.limb.push_back(v);
    return b;
}

void BigU::mul_small(uint64_t m)
{
    unsigned __int128 carry = 0;
    for (auto &l : limb) {
        const unsigned __int128 t = (unsigned __int128)l * m + carry;
        l = (uint64_t)t;
        carry = t >> 64;
    }
    if (carry) limb.push_back((uint64_t)carry);
    trim();
}

void BigU::add_small(uint64_t a)
{
    unsigned __int128 carry = a;
    for (size_t i = 0; i < limb.size() && carry; ++i) {
        const unsigned __int128 t = (unsigned __int128)limb[i] + carry;
        limb[i] = (uint64_t)t;
        carry = t >> 64;
    }
    if (carry) limb.push_back((uint64_t)carry);
}

BigU BigU::mul(const BigU &a, const BigU &b)
{
    BigU r;
    if (a.limb.empty() || b.limb.empty()) return r;
    r.limb.assign(a.limb.size() + b.limb.size(), 0);
    for (size_t i = 0; i < a.limb.size(); ++i) {
        unsigned __int128 carry = 0;
        for (size_t j = 0; j < b.limb.size(); ++j) {
            const unsigned __int128 t =
                (unsigned __int128)a.limb[i] * b.limb[j] + r.limb[i + j] + carry;
            r.limb[i + j] = (uint64_t)t;
            carry = t >> 64;
        }
        r.limb[i + b.limb.size()] += (uint64_t)carry;
    }
    r.trim();
    return r;
}

int BigU::cmp(const BigU &a, const BigU &b)
{
    if (a.limb.size() != b.limb.size()) return a.limb.size() < b.limb.size() ? -1 : 1;
    for (size_t i = a.limb.size(); i-- > 0;)
        if (a.limb[i] != b.limb[i]) return a.limb[i] < b.limb[i] ? -1 : 1;
    return 0;
}

BigU BigU::sub(const BigU &a, const BigU &b)   // a >= b
{
    BigU r = a;
    unsigned __int128 borrow = 0;
    for (size_t i = 0; i < r.limb.size(); ++i) {
        const unsigned __int128 bi = (i < b.limb.size() ? b.limb[i] : 0) + borrow;
        const unsigned __int128 ai = r.limb[i];
        if (ai >= bi) { r.limb[i] = (uint64_t)(ai - bi); borrow = 0; }
        else { r.limb[i] = (uint64_t)(((unsigned __int128)1 << 64) + ai - bi); borrow = 1; }
    }
    r.trim();
    return r;
}

bool schur_bound_ok(int n, const std::vector<uint32_t> &primes)
{
    BigU M = BigU::from(1);
    for (uint32_t p : primes) M.mul_small(p);
    BigU lhs = BigU::mul(M, M);
    BigU rhs = BigU::from(4);
    for (int i = 0; i < n; ++i) rhs.mul_small((uint64_t)n);
    return BigU::cmp(lhs, rhs) > 0;
}

bool garner_lift(const uint32_t *res, const uint32_t *primes, int k, BigU &mag, int &sign)
{
    std::vector<uint64_t> v(k);
    for (int i = 0; i < k; ++i) {
        const uint64_t p = primes[i];
        uint64_t x = res[i] % p;
        for (int j = 0; j < i; ++j) {
            const uint64_t pj = primes[j] % p;
            const uint64_t inv = powmod(pj, p - 2, p);        // p prime
            if (!inv) return false;
            x = ((x + p - v[j] % p) % p) * inv % p;
        }
        v[i] = x;
    }
    // X = v0 + v1 p0 + v2 p0 p1 + ...  (Horner from the top digit)
    BigU X = BigU::from(0);
    for (int i = k - 1; i >= 0; --i) {
        if (i < k - 1) X.mul_small(primes[i]);
        X.add_small(v[i]);
    }
    BigU M = BigU::from(1);
    for (int i = 0; i < k; ++i) M.mul_small(primes[i]);
    // X > M/2 (M odd)  <=>  2X > M
    BigU X2 = X;
    X2.mul_small(2);
    if (X.limb.empty()) { mag = X; sign = 0; }
    else if (BigU::cmp(X2, M) > 0) { mag = BigU::sub(M, X); sign = -1; }
    else { mag = X; sign = 1; }
    return true;
}

double log2_product(const uint32_t *primes, int k)
{
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += std::log2((double)primes[i]);
    return s;
}

}  // namespace permh
