/*
 * Oracle: plain single-threaded CPU permanents.  TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  It shares no code, header or table with the GPU path.
 *
 * What it computes
 * ----------------
 * perm(A) = sum over sigma in S_n of prod_i a_{i,sigma(i)}      (paper, Sec. 1)
 *
 * evaluated with Ryser's inclusion-exclusion formula, which the paper cites
 * as the O(n 2^n) algorithm (Sec. 1 and Sec. 2.1) without printing it:
 *
 *   perm(A) = (-1)^n  sum_{S subset {0..n-1}} (-1)^{|S|} prod_i ( sum_{j in S} a_ij )
 *
 * The subsets S are visited in reflected-binary Gray order (S_x = gray(x),
 * x = 1 .. 2^n - 1), so one column enters or leaves S per visit and the n row
 * sums are updated by one add or subtract each; that is the textbook
 * O(n 2^n) form of the formula.  The parity of |S_x| equals the parity of x.
 *
 * Per field:
 *   c128 / f64 : double arithmetic; a complex product is 4 multiplies and
 *                2 adds (the file is compiled with -ffp-contract=off, so no
 *                FMA is formed); the signed sum uses Kahan compensated
 *                summation per real component (paper, Sec. 1 Note) unless
 *                kahan == 0.
 *   c128 long double : the same walk in long double, to audit the double one.
 *   F_p        : residues in [0,p), products as (uint64)a*b % p, no
 *                Montgomery or Barrett form, p odd or even, p < 2^32.
 *
 * It also evaluates, for range checks, the Glynn-form partial sum
 *   G(x0,x1) = sum_{x=x0}^{x1-1} (-1)^x prod_i ( a_i0 + sum_{k>=1} d_k(x) a_ik ),
 *   d_k(x) = 1 - 2 * bit_{k-1}(x XOR (x>>1)),
 * directly from its definition: every x is evaluated from scratch in O(n^2)
 * with no Gray-code update, so it shares neither formula nor walk with the
 * Ryser routine above.  Over the full range x in [0, 2^(n-1)),
 * G / 2^(n-1) = perm(A) (Glynn's identity, which the paper's GPU code uses,
 * Sec. 1 Note).
 *
 * Return value of every entry point: 0 on success, -1 on a bad argument.
 */
#include <stdint.h>
#include <stddef.h>

#define ORACLE_NMAX 48            /* the largest order the library accepts */

static unsigned ctz64(uint64_t x) {
    unsigned k = 0;
    while (!(x & 1u)) { x >>= 1; ++k; }
    return k;
}

/* ---------------------------------------------------------------- c128 */
int oracle_ryser_c128(const double *A, int n, int kahan, double *out)
{
    if (n < 0 || n > ORACLE_NMAX || !out || (n > 0 && !A)) return -1;
    if (n == 0) { out[0] = 1.0; out[1] = 0.0; return 0; }
    double sr[ORACLE_NMAX], si[ORACLE_NMAX];
    for (int i = 0; i < n; ++i) { sr[i] = 0.0; si[i] = 0.0; }
    double tr = 0.0, ti = 0.0, cr = 0.0, ci = 0.0;  /* sums, compensations */
    const uint64_t nsub = (uint64_t)1 << n;
    for (uint64_t x = 1; x < nsub; ++x) {
        unsigned j = ctz64(x);
        uint64_t g = x ^ (x >> 1);
        int enters = (int)((g >> j) & 1u);
        for (int i = 0; i < n; ++i) {
            double ar = A[2 * ((size_t)i * n + j)], ai = A[2 * ((size_t)i * n + j) + 1];
            if (enters) { sr[i] += ar; si[i] += ai; }
            else        { sr[i] -= ar; si[i] -= ai; }
        }
        double pr = sr[0], pi = si[0];
        for (int i = 1; i < n; ++i) {
            double qr = pr * sr[i] - pi * si[i];
            double qi = pr * si[i] + pi * sr[i];
            pr = qr; pi = qi;
        }
        if (x & 1u) { pr = -pr; pi = -pi; }       /* (-1)^{|S|} */
        if (kahan) {
            double y = pr - cr, t = tr + y; cr = (t - tr) - y; tr = t;
            y = pi - ci; t = ti + y; ci = (t - ti) - y; ti = t;
        } else {
            tr += pr; ti += pi;
        }
    }
    if (n & 1) { tr = -tr; ti = -ti; }            /* (-1)^n */
    out[0] = tr; out[1] = ti;
    return 0;
}

/* Same walk in long double (x87 extended precision on x86-64). */
int oracle_ryser_c128_ld(const double *A, int n, double *out)
{
    if (n < 0 || n > ORACLE_NMAX || !out || (n > 0 && !A)) return -1;
    if (n == 0) { out[0] = 1.0; out[1] = 0.0; return 0; }
    long double sr[ORACLE_NMAX], si[ORACLE_NMAX];
    for (int i = 0; i < n; ++i) { sr[i] = 0.0L; si[i] = 0.0L; }
    long double tr = 0.0L, ti = 0.0L, cr = 0.0L, ci = 0.0L;
    const uint64_t nsub = (uint64_t)1 << n;
    for (uint64_t x = 1; x < nsub; ++x) {
        unsigned j = ctz64(x);
        uint64_t g = x ^ (x >> 1);
        int enters = (int)((g >> j) & 1u);
        for (int i = 0; i < n; ++i) {
            long double ar = A[2 * ((size_t)i * n + j)], ai = A[2 * ((size_t)i * n + j) + 1];
            if (enters) { sr[i] += ar; si[i] += ai; }
            else        { sr[i] -= ar; si[i] -= ai; }
        }
        long double pr = sr[0], pi = si[0];
        for (int i = 1; i < n; ++i) {
            long double qr = pr * sr[i] - pi * si[i];
            long double qi = pr * si[i] + pi * sr[i];
            pr = qr; pi = qi;
        }
        if (x & 1u) { pr = -pr; pi = -pi; }
        long double y = pr - cr, t = tr + y; cr = (t - tr) - y; tr = t;
        y = pi - ci; t = ti + y; ci = (t - ti) - y; ti = t;
    }
    if (n & 1) { tr = -tr; ti = -ti; }
    out[0] = (double)tr; out[1] = (double)ti;
    return 0;
}

/* ----------------------------------------------------------------- f64 */
int oracle_ryser_f64(const double *A, int n, int kahan, double *out)
{
    if (n < 0 || n > ORACLE_NMAX || !out || (n > 0 && !A)) return -1;
    if (n == 0) { out[0] = 1.0; return 0; }
    double s[ORACLE_NMAX];
    for (int i = 0; i < n; ++i) s[i] = 0.0;
    double tot = 0.0, c = 0.0;
    const uint64_t nsub = (uint64_t)1 << n;
    for (uint64_t x = 1; x < nsub; ++x) {
        unsigned j = ctz64(x);
        uint64_t g = x ^ (x >> 1);
        int enters = (int)((g >> j) & 1u);
        for (int i = 0; i < n; ++i) {
            if (enters) s[i] += A[(size_t)i * n + j];
            else        s[i] -= A[(size_t)i * n + j];
        }
        double p = s[0];
        for (int i = 1; i < n; ++i) p *= s[i];
        if (x & 1u) p = -p;
        if (kahan) { double y = p - c, t = tot + y; c = (t - tot) - y; tot = t; }
        else tot += p;
    }
    if (n & 1) tot = -tot;
    out[0] = tot;
    return 0;
}

/* --------------------------------------------- float sums over subset ranges */
/* The signed Ryser sums of the two walks above over the Gray-ordered subsets
 * x in [x_begin, x_end) (1 <= x_begin <= x_end <= 2^n), without the final
 * (-1)^n, Kahan-summed per component.  The row sums start as those of the
 * subset gray(x_begin - 1), added up column by column; from there each
 * visit is the whole walk's.  Disjoint ranges covering [1, 2^n) add up to
 * the whole sum (up to the rounding of that addition), so one permanent can
 * be spread over host threads. */
int oracle_ryser_c128_range(const double *A, int n, uint64_t x_begin, uint64_t x_end, double *out)
{
    if (n < 1 || n > ORACLE_NMAX || !A || !out) return -1;
    if (x_begin < 1 || x_begin > x_end || (n < 64 && x_end > ((uint64_t)1 << n))) return -1;
    double sr[ORACLE_NMAX], si[ORACLE_NMAX];
    for (int i = 0; i < n; ++i) { sr[i] = 0.0; si[i] = 0.0; }
    const uint64_t g0 = (x_begin - 1) ^ ((x_begin - 1) >> 1);
    for (int j = 0; j < n; ++j)
        if ((g0 >> j) & 1u)
            for (int i = 0; i < n; ++i) {
                sr[i] += A[2 * ((size_t)i * n + j)];
                si[i] += A[2 * ((size_t)i * n + j) + 1];
            }
    double tr = 0.0, ti = 0.0, cr = 0.0, ci = 0.0;
    for (uint64_t x = x_begin; x < x_end; ++x) {
        unsigned j = ctz64(x);
        uint64_t g = x ^ (x >> 1);
        int enters = (int)((g >> j) & 1u);
        for (int i = 0; i < n; ++i) {
            double ar = A[2 * ((size_t)i * n + j)], ai = A[2 * ((size_t)i * n + j) + 1];
            if (enters) { sr[i] += ar; si[i] += ai; }
            else        { sr[i] -= ar; si[i] -= ai; }
        }
        double pr = sr[0], pi = si[0];
        for (int i = 1; i < n; ++i) {
            double qr = pr * sr[i] - pi * si[i];
            double qi = pr * si[i] + pi * sr[i];
            pr = qr; pi = qi;
        }
        if (x & 1u) { pr = -pr; pi = -pi; }
        double y = pr - cr, t = tr + y; cr = (t - tr) - y; tr = t;
        y = pi - ci; t = ti + y; ci = (t - ti) - y; ti = t;
    }
    out[0] = tr; out[1] = ti;
    return 0;
}

int oracle_ryser_f64_range(const double *A, int n, uint64_t x_begin, uint64_t x_end, double *out)
{
    if (n < 1 || n > ORACLE_NMAX || !A || !out) return -1;
    if (x_begin < 1 || x_begin > x_end || (n < 64 && x_end > ((uint64_t)1 << n))) return -1;
    double s[ORACLE_NMAX];
    for (int i = 0; i < n; ++i) s[i] = 0.0;
    const uint64_t g0 = (x_begin - 1) ^ ((x_begin - 1) >> 1);
    for (int j = 0; j < n; ++j)
        if ((g0 >> j) & 1u)
            for (int i = 0; i < n; ++i) s[i] += A[(size_t)i * n + j];
    double tot = 0.0, c = 0.0;
    for (uint64_t x = x_begin; x < x_end; ++x) {
        unsigned j = ctz64(x);
        uint64_t g = x ^ (x >> 1);
        int enters = (int)((g >> j) & 1u);
        for (int i = 0; i < n; ++i) {
            if (enters) s[i] += A[(size_t)i * n + j];
            else        s[i] -= A[(size_t)i * n + j];
        }
        double p = s[0];
        for (int i = 1; i < n; ++i) p *= s[i];
        if (x & 1u) p = -p;
        double y = p - c, t = tot + y; c = (t - tot) - y; tot = t;
    }
    out[0] = tot;
    return 0;
}

/* ----------------------------------------------------------------- F_p */
/* Signed Ryser sum over the Gray-ordered subsets x = x_begin .. x_end-1
 * (x_begin >= 1), mod p, without the final (-1)^n.  The row sums start as
 * those of the subset gray(x_begin - 1), added up column by column; from
 * there the walk is the same as for the whole sum.  [1, 2^n) is the whole
 * sum. */
static int ryser_modp_span(const uint32_t *A, int n, uint32_t p, uint64_t x_begin, uint64_t x_end,
                           uint64_t *tot_out)
{
    const uint64_t P = p;
    uint64_t s[ORACLE_NMAX];
    for (int i = 0; i < n; ++i) s[i] = 0;
    const uint64_t g0 = (x_begin - 1) ^ ((x_begin - 1) >> 1);
    for (int j = 0; j < n; ++j)
        if ((g0 >> j) & 1u)
            for (int i = 0; i < n; ++i) s[i] = (s[i] + A[(size_t)i * n + j]) % P;
    uint64_t tot = 0;
    for (uint64_t x = x_begin; x < x_end; ++x) {
        unsigned j = ctz64(x);
        uint64_t g = x ^ (x >> 1);
        int enters = (int)((g >> j) & 1u);
        for (int i = 0; i < n; ++i) {
            uint64_t a = A[(size_t)i * n + j];
            if (enters) s[i] = (s[i] + a) % P;
            else        s[i] = (s[i] + P - a) % P;
        }
        uint64_t prod = s[0];
        for (int i = 1; i < n; ++i) prod = (prod * s[i]) % P;
        if (x & 1u) tot = (tot + P - prod) % P;
        else        tot = (tot + prod) % P;
    }
    *tot_out = tot;
    return 0;
}

static int ryser_modp_upto(const uint32_t *A, int n, uint32_t p, uint64_t x_end, uint64_t *tot_out)
{
    return ryser_modp_span(A, n, p, 1, x_end, tot_out);
}

int oracle_ryser_modp(const uint32_t *A, int n, uint32_t p, uint32_t *out)
{
    if (n < 0 || n > ORACLE_NMAX || !out || p < 2 || (n > 0 && !A)) return -1;
    for (int i = 0; i < n * n; ++i) if (A[i] >= p) return -1;
    if (n == 0) { out[0] = 1u % p; return 0; }
    uint64_t tot = 0;
    ryser_modp_upto(A, n, p, (uint64_t)1 << n, &tot);
    if (n & 1) tot = (p - tot) % p;
    out[0] = (uint32_t)tot;
    return 0;
}

/* The first x_end - 1 subsets of the walk above: the same per-subset work on
 * a bounded prefix, used to time the oracle on matrices too large to finish. */
int oracle_ryser_modp_prefix(const uint32_t *A, int n, uint32_t p, uint64_t x_end, uint32_t *out)
{
    if (n < 1 || n > ORACLE_NMAX || !out || p < 2 || !A) return -1;
    if (n < 64 && x_end > ((uint64_t)1 << n)) return -1;
    for (int i = 0; i < n * n; ++i) if (A[i] >= p) return -1;
    uint64_t tot = 0;
    ryser_modp_upto(A, n, p, x_end, &tot);
    out[0] = (uint32_t)tot;
    return 0;
}

/* The signed Ryser sum over the subsets x in [x_begin, x_end) of the walk
 * above (1 <= x_begin <= x_end <= 2^n), mod p, without the final (-1)^n:
 * disjoint ranges that cover [1, 2^n) add up to the whole sum, so one
 * permanent can be split over host threads. */
int oracle_ryser_modp_range(const uint32_t *A, int n, uint32_t p, uint64_t x_begin, uint64_t x_end,
                            uint32_t *out)
{
    if (n < 1 || n > ORACLE_NMAX || !out || p < 2 || !A) return -1;
    if (x_begin < 1 || x_begin > x_end || (n < 64 && x_end > ((uint64_t)1 << n))) return -1;
    for (int i = 0; i < n * n; ++i) if (A[i] >= p) return -1;
    uint64_t tot = 0;
    ryser_modp_span(A, n, p, x_begin, x_end, &tot);
    out[0] = (uint32_t)tot;
    return 0;
}

/* ------------------------------------------- Glynn terms, evaluated directly */
static int glynn_delta(uint64_t x, int k)   /* k >= 1 */
{
    uint64_t g = x ^ (x >> 1);
    return ((g >> (k - 1)) & 1u) ? -1 : 1;
}

int oracle_glynn_range_c128(const double *A, int n, uint64_t x0, uint64_t x1, double *out)
{
    if (n < 1 || n > ORACLE_NMAX || !A || !out || x0 > x1) return -1;
    if (n - 1 < 64 && x1 > ((uint64_t)1 << (n - 1))) return -1;
    double tr = 0.0, ti = 0.0, cr = 0.0, ci = 0.0;
    for (uint64_t x = x0; x < x1; ++x) {
        double pr = 1.0, pi = 0.0;
        for (int i = 0; i < n; ++i) {
            double rr = A[2 * ((size_t)i * n)], ri = A[2 * ((size_t)i * n) + 1];
            for (int k = 1; k < n; ++k) {
                double d = (double)glynn_delta(x, k);
                rr += d * A[2 * ((size_t)i * n + k)];
                ri += d * A[2 * ((size_t)i * n + k) + 1];
            }
            double qr = pr * rr - pi * ri;
            double qi = pr * ri + pi * rr;
            pr = qr; pi = qi;
        }
        if (x & 1u) { pr = -pr; pi = -pi; }
        double y = pr - cr, t = tr + y; cr = (t - tr) - y; tr = t;
        y = pi - ci; t = ti + y; ci = (t - ti) - y; ti = t;
    }
    out[0] = tr; out[1] = ti;
    return 0;
}

int oracle_glynn_range_f64(const double *A, int n, uint64_t x0, uint64_t x1, double *out)
{
    if (n < 1 || n > ORACLE_NMAX || !A || !out || x0 > x1) return -1;
    if (n - 1 < 64 && x1 > ((uint64_t)1 << (n - 1))) return -1;
    double tot = 0.0, c = 0.0;
    for (uint64_t x = x0; x < x1; ++x) {
        double p = 1.0;
        for (int i = 0; i < n; ++i) {
            double r = A[(size_t)i * n];
            for (int k = 1; k < n; ++k) r += (double)glynn_delta(x, k) * A[(size_t)i * n + k];
            p *= r;
        }
        if (x & 1u) p = -p;
        double y = p - c, t = tot + y; c = (t - tot) - y; tot = t;
    }
    out[0] = tot;
    return 0;
}

int oracle_glynn_range_modp(const uint32_t *A, int n, uint32_t p, uint64_t x0, uint64_t x1,
                            uint32_t *out)
{
    if (n < 1 || n > ORACLE_NMAX || !A || !out || p < 2 || x0 > x1) return -1;
    if (n - 1 < 64 && x1 > ((uint64_t)1 << (n - 1))) return -1;
    for (int i = 0; i < n * n; ++i) if (A[i] >= p) return -1;
    const uint64_t P = p;
    uint64_t tot = 0;
    for (uint64_t x = x0; x < x1; ++x) {
        uint64_t prod = 1 % P;
        for (int i = 0; i < n; ++i) {
            uint64_t r = A[(size_t)i * n];
            for (int k = 1; k < n; ++k) {
                uint64_t a = A[(size_t)i * n + k];
                r = (glynn_delta(x, k) > 0) ? (r + a) % P : (r + P - a) % P;
            }
            prod = (prod * r) % P;
        }
        tot = (x & 1u) ? (tot + P - prod) % P : (tot + prod) % P;
    }
    out[0] = (uint32_t)tot;
    return 0;
}

/* Many independent f64/c128 permanents, one after another (the CPU baseline
 * times this; nthreads-fold parallelism is done by the caller with separate
 * processes or threads over disjoint index ranges). */
int oracle_ryser_c128_many(const double *A, int n, int count, int kahan, double *out)
{
    if (count < 0) return -1;
    for (int m = 0; m < count; ++m)
        if (oracle_ryser_c128(A + (size_t)m * 2 * n * n, n, kahan, out + 2 * (size_t)m)) return -1;
    return 0;
}

int oracle_ryser_f64_many(const double *A, int n, int count, int kahan, double *out)
{
    if (count < 0) return -1;
    for (int m = 0; m < count; ++m)
        if (oracle_ryser_f64(A + (size_t)m * n * n, n, kahan, out + (size_t)m)) return -1;
    return 0;
}
