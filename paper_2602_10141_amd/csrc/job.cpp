// Checkpointed exact permanent over Z: per-prime Glynn ranges cut into
// pieces whose unscaled partial sums mod p go to an append-only text file,
// so a run of hours survives interruption and resumes bit-exactly.
//
// File format (text):
//   perm-job 1 n <n> k <k> piece_log2 <c> id <16 hex digits>
//   <prime index> <piece index> <partial mod p>      (one line per piece)
// The id hashes n, the primes and the matrices (FNV-1a over their bytes).
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <chrono>
#include <cmath>
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "numth.h"

using namespace permk;
using namespace permi;

struct perm_job {
    perm_ctx *ctx = nullptr;
    int n = 0, k = 0, piece_log2 = 0;
    double log2_bound = 0;
    std::vector<uint32_t> primes, mats;
    uint64_t pieces = 0;                    // per prime
    std::vector<int64_t> part;              // k * pieces, -1 = not done
    uint64_t done = 0;
    uint64_t next = 0;                      // scan position (piece-major over primes)
    FILE *ck = nullptr;
    uint64_t id = 0;
};

namespace {

uint64_t fnv(uint64_t h, const void *p, size_t b)
{
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < b; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

std::string header(const perm_job *J)
{
    char buf[160];
    snprintf(buf, sizeof buf, "perm-job 1 n %d k %d piece_log2 %d id %016" PRIx64, J->n, J->k,
             J->piece_log2, J->id);
    return buf;
}

// Read an existing checkpoint into J->part.  Returns PERM_OK if the file is
// absent or valid.
int load(perm_job *J, const char *path, bool *exists, size_t *valid_len, size_t *file_len)
{
    *exists = false;
    *valid_len = *file_len = 0;
    FILE *f = fopen(path, "rb");
    if (!f) return PERM_OK;
    *exists = true;
    std::string text;
    char buf[1 << 16];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    *file_len = text.size();
    size_t pos = text.find('\n');
    if (pos == std::string::npos) return fail(PERM_EINVAL, "checkpoint %s has no complete header", path);
    if (text.compare(0, pos, header(J)) != 0)
        return fail(PERM_EINVAL, "checkpoint %s belongs to another job (header '%s', expected '%s')",
                    path, text.substr(0, pos).c_str(), header(J).c_str());
    size_t line = 1;
    *valid_len = pos + 1;
    for (size_t at = pos + 1; at < text.size();) {
        const size_t end = text.find('\n', at);
        if (end == std::string::npos) break;           // torn last line: ignored
        ++line;
        unsigned long long i = 0, j = 0, v = 0;
        int used = 0;
        const std::string ln = text.substr(at, end - at);
        if (sscanf(ln.c_str(), "%llu %llu %llu%n", &i, &j, &v, &used) != 3 || used != (int)ln.size() ||
            i >= (unsigned long long)J->k || j >= J->pieces || v >= J->primes[i])
            return fail(PERM_EINVAL, "checkpoint %s line %zu is malformed: '%s'", path, line, ln.c_str());
        int64_t &slot = J->part[(size_t)i * J->pieces + j];
        if (slot >= 0 && slot != (int64_t)v)
            return fail(PERM_EINVAL, "checkpoint %s line %zu contradicts an earlier line", path, line);
        if (slot < 0) J->done++;
        slot = (int64_t)v;
        at = end + 1;
        *valid_len = at;
    }
    return PERM_OK;
}

}  // namespace

extern "C" int perm_job_create(perm_ctx *ctx, const uint32_t *mats, const uint32_t *primes, int k,
                               int n, double log2_bound, int piece_log2,
                               const char *checkpoint_path, perm_job **out)
{
    if (!ctx || !mats || !out) return fail(PERM_EINVAL, "NULL argument");
    *out = nullptr;
    if (n < 2 || n > PERM_NMAX) return fail(PERM_EINVAL, "n = %d outside [2, %d]", n, PERM_NMAX);
    int rc = check_primes(primes, k, log2_bound);
    if (rc != PERM_OK) return rc;
    if (piece_log2 == 0) piece_log2 = std::max(10, n - 9);
    if (piece_log2 < 10 || piece_log2 > n - 1)
        return fail(PERM_EINVAL, "piece_log2 = %d outside [10, %d]", piece_log2, n - 1);
    const size_t nn = (size_t)n * n;
    for (size_t q = 0; q < nn * (size_t)k; ++q)
        if (mats[q] >= primes[q / nn])
            return fail(PERM_EINVAL, "entry %zu of matrix %zu is not reduced mod %u", q % nn, q / nn,
                        primes[q / nn]);
    perm_job *J = new (std::nothrow) perm_job();
    if (!J) return fail(PERM_ENOMEM, "host allocation failed");
    J->ctx = ctx;
    J->n = n;
    J->k = k;
    J->piece_log2 = piece_log2;
    J->log2_bound = log2_bound;
    J->primes.assign(primes, primes + k);
    J->mats.assign(mats, mats + nn * k);
    J->pieces = 1ull << (n - 1 - piece_log2);
    J->part.assign((size_t)k * J->pieces, -1);
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, &n, sizeof n);
    h = fnv(h, primes, sizeof(uint32_t) * k);
    h = fnv(h, mats, sizeof(uint32_t) * nn * k);
    J->id = h;
    if (checkpoint_path && *checkpoint_path) {
        bool exists = false;
        size_t valid_len = 0, file_len = 0;
        if ((rc = load(J, checkpoint_path, &exists, &valid_len, &file_len)) != PERM_OK) {
            delete J;
            return rc;
        }
        // drop a torn last line so that appending continues on a line boundary
        if (exists && file_len > valid_len && truncate(checkpoint_path, (off_t)valid_len) != 0) {
            delete J;
            return fail(PERM_EINVAL, "cannot truncate the torn end of checkpoint %s", checkpoint_path);
        }
        J->ck = fopen(checkpoint_path, "ab");
        if (!J->ck) {
            delete J;
            return fail(PERM_EINVAL, "cannot open checkpoint %s for appending", checkpoint_path);
        }
        if (!exists) {
            fprintf(J->ck, "%s\n", header(J).c_str());
            if (fflush(J->ck) != 0 || fsync(fileno(J->ck)) != 0) {
                fclose(J->ck);
                delete J;
                return fail(PERM_EINVAL, "cannot write checkpoint %s", checkpoint_path);
            }
        }
    }
    *out = J;
    return PERM_OK;
}

extern "C" int perm_job_run(perm_job *J, double seconds, uint64_t *done, uint64_t *total)
{
    if (!J) return fail(PERM_EINVAL, "job is NULL");
    perm_ctx *ctx = J->ctx;
    const uint64_t all = (uint64_t)J->k * J->pieces;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = ctx->stream;
    const size_t per = (size_t)J->n * J->n * 4;
    const int variant = variant_of(PERM_MODP, 0);
    // A batch covers at least 2^37 Glynn terms (about a second on one
    // device) and at least 8 wave items per resident wave (about 12 per
    // compute unit), so that the last round of long items does not leave
    // most of the device idle.
    const int c = log2_chunk_for(ctx, variant, J->n);
    const double items_min = 8.0 * 12.0 * ctx->num_cus;
    const double terms = std::max(std::ldexp(1.0, 37), items_min * std::ldexp(1.0, c + 6));
    const double want = std::ceil(terms / std::ldexp(1.0, J->piece_log2));
    const uint64_t batch_pieces = (uint64_t)std::min(4096.0, std::max(1.0, want));
    while (J->done < all) {
        std::vector<std::pair<uint32_t, uint64_t>> pick;      // (prime, piece)
        for (uint64_t scan = 0; scan < all && pick.size() < batch_pieces; ++scan) {
            const uint64_t q = (J->next + scan) % all;
            const uint32_t i = (uint32_t)(q % J->k);
            const uint64_t j = q / J->k;
            if (J->part[(size_t)i * J->pieces + j] < 0) pick.emplace_back(i, j);
        }
        int rc = begin_call(ctx, s);
        if (rc != PERM_OK) return rc;
        const void *src = nullptr;
        if ((rc = source_on_device(ctx, J->mats.data(), per * J->k, 0, s, &src)) != PERM_OK) return rc;
        std::vector<MatIn> &in = ctx->scratch_in;
        in.assign(pick.size(), MatIn{});
        for (size_t q = 0; q < pick.size(); ++q) {
            MatIn &m = in[q];
            m.variant = variant;
            m.n = J->n;
            m.p = J->primes[pick[q].first];
            m.src_off = per * pick[q].first;
            m.out_slot = (uint32_t)q;
            m.full = false;
            m.x0 = pick[q].second << J->piece_log2;
            m.x1 = m.x0 + (1ull << J->piece_log2);
            m.no_scale = true;
        }
        Plan &pl = ctx->scratch_plan;
        if ((rc = plan(ctx, in, pl)) != PERM_OK) return rc;
        if ((rc = ensure(ctx, ctx->outs, pick.size() * 16)) != PERM_OK) return rc;
        if ((rc = execute(ctx, pl, src, ctx->outs.p, pick.size(), s)) != PERM_OK) return rc;
        std::vector<uint32_t> slots(pick.size() * 4);
        if (hipMemcpyAsync(slots.data(), ctx->outs.p, pick.size() * 16, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
            return fail(PERM_EDEVICE, "result copy failed");
        if ((rc = end_call(ctx, s)) != PERM_OK) return rc;
        if (hipStreamSynchronize(s) != hipSuccess) return fail(PERM_EDEVICE, "job batch failed");
        for (size_t q = 0; q < pick.size(); ++q) {
            J->part[(size_t)pick[q].first * J->pieces + pick[q].second] = slots[4 * q];
            J->done++;
            if (J->ck)
                fprintf(J->ck, "%u %" PRIu64 " %u\n", pick[q].first, pick[q].second, slots[4 * q]);
        }
        if (J->ck && (fflush(J->ck) != 0 || fsync(fileno(J->ck)) != 0))
            return fail(PERM_EINVAL, "checkpoint write failed");
        const uint64_t last = (uint64_t)pick.back().second * J->k + pick.back().first;
        J->next = (last + 1) % all;
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (el >= seconds) break;
    }
    if (done) *done = J->done;
    if (total) *total = all;
    return PERM_OK;
}

extern "C" int perm_job_result(perm_job *J, uint32_t *residues, uint64_t *limbs, int max_limbs,
                               int *nlimbs, int *sign)
{
    if (!J || !limbs || !nlimbs || !sign) return fail(PERM_EINVAL, "NULL argument");
    const uint64_t all = (uint64_t)J->k * J->pieces;
    if (J->done < all)
        return fail(PERM_EAGAIN, "%" PRIu64 " of %" PRIu64 " pieces done", J->done, all);
    std::vector<uint32_t> res(J->k);
    for (int i = 0; i < J->k; ++i) {
        const uint64_t p = J->primes[i];
        uint64_t sum = 0;
        for (uint64_t j = 0; j < J->pieces; ++j) sum = (sum + (uint64_t)J->part[(size_t)i * J->pieces + j]) % p;
        // perm = 2^-(n-1) * (sum of the unscaled Glynn partials)
        const uint64_t inv2 = (p + 1) / 2;
        res[i] = (uint32_t)(sum * permh::powmod(inv2, (uint64_t)(J->n - 1), p) % p);
    }
    permh::BigU mag;
    int sg = 0;
    if (!permh::garner_lift(res.data(), J->primes.data(), J->k, mag, sg))
        return fail(PERM_EINVAL, "lift failed");
    int rc = write_limbs(mag, sg, limbs, max_limbs, nlimbs, sign);
    if (rc != PERM_OK) return rc;
    if (residues) std::memcpy(residues, res.data(), sizeof(uint32_t) * J->k);
    return PERM_OK;
}

extern "C" void perm_job_destroy(perm_job *J)
{
    if (!J) return;
    if (J->ck) fclose(J->ck);
    delete J;
}
