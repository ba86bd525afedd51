// Replays a serving stream through the request loop on the CPU test double:
// 64 complex requests at each odd n in 11..25 and six F_p requests at each
// of the large orders, shuffled, submitted at once or with exponential gaps,
// some cancelled; every completed result must carry its matrix's hash and no
// bad partial slot.  Settings come from the environment (SIM_*).
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

extern std::atomic<long> sim_desync, sim_bad_parts, sim_items;
uint64_t sim_hash(const unsigned char *p, size_t b);

namespace {

double env_f(const char *k, double d) { const char *v = getenv(k); return v ? atof(v) : d; }

struct Request {
    perm_item it{};
    std::vector<unsigned char> m;
};

}  // namespace

int main()
{
    const double rate = env_f("SIM_RATE", 0);                 // requests per second, 0 = at once
    const int reps = (int)env_f("SIM_REPS", 1);
    const int cancel_every = (int)env_f("SIM_CANCEL_EVERY", 0);
    // with fault injection on, requests may fail with PERM_EDEVICE; all
    // others must still complete with their own results
    const bool faults = getenv("SIM_FAIL_WALK") || getenv("SIM_FAIL_EVENT_SYNC");
    std::vector<int> big;
    {
        std::stringstream ss(getenv("SIM_BIG") ? getenv("SIM_BIG") : "32,34,36");
        std::string tok;
        while (std::getline(ss, tok, ',')) big.push_back(atoi(tok.c_str()));
    }
    std::mt19937_64 g((uint64_t)env_f("SIM_SEED", 1));
    std::vector<Request> reqs;
    for (int n = 11; n <= 25; n += 2)
        for (int t = 0; t < 64; ++t) {
            Request r;
            r.it.n = n;
            r.it.field = PERM_C128;
            r.m.resize((size_t)n * n * 16);
            for (auto &b : r.m) b = (unsigned char)g();
            reqs.push_back(std::move(r));
        }
    for (int n : big)
        for (int k = 0; k < 6; ++k) {
            Request r;
            r.it.n = n;
            r.it.field = PERM_MODP;
            r.it.p = 2147483647u - 2 * k;
            r.m.resize((size_t)n * n * 4);
            for (auto &b : r.m) b = (unsigned char)g();
            reqs.push_back(std::move(r));
        }
    std::shuffle(reqs.begin(), reqs.end(), g);
    perm_ctx ctx;
    ctx.num_cus = 256;
    long wrong = 0;
    for (int rep = 0; rep < reps && !wrong; ++rep) {
        long failed = 0;
        perm_srv_cfg cfg{};
        cfg.hbm_budget = (size_t)env_f("SIM_BUDGET_MB", 512) << 20;
        cfg.max_inflight = (int)env_f("SIM_MAX_INFLIGHT", 0);
        cfg.slice_us = env_f("SIM_SLICE_US", 2000);
        perm_srv *S = nullptr;
        if (perm_srv_create(&ctx, &cfg, &S) != PERM_OK) return 2;
        std::vector<std::atomic<uint64_t>> tickets(reqs.size());
        for (auto &t : tickets) t = 0;
        std::exponential_distribution<double> gap(rate > 0 ? rate : 1.0);
        std::vector<double> gaps(reqs.size());
        for (double &x : gaps) x = rate > 0 ? gap(g) : 0.0;
        std::atomic<bool> sub_failed{false};
        std::thread sub([&] {
            const auto t0 = std::chrono::steady_clock::now();
            double t = 0;
            for (size_t i = 0; i < reqs.size(); ++i) {
                t += gaps[i];
                if (rate > 0) std::this_thread::sleep_until(t0 + std::chrono::duration<double>(t));
                uint64_t tk = 0;
                if (perm_srv_submit(S, &reqs[i].it, reqs[i].m.data(), &tk) != PERM_OK) {
                    sub_failed = true;
                    return;
                }
                if (cancel_every && i % cancel_every == 0) perm_srv_cancel(S, tk);
                tickets[i] = tk;
            }
        });
        for (size_t i = 0; i < reqs.size() && !sub_failed; ++i) {
            while (!tickets[i] && !sub_failed) std::this_thread::sleep_for(std::chrono::microseconds(100));
            if (sub_failed) break;
            unsigned char out[16];
            int done = 0;
            double lat = 0;
            perm_srv_times tm{};
            // odd requests report the phases of their latency
            const int rc = (i & 1) ? perm_srv_wait_times(S, tickets[i], 30.0, out, &done, &tm)
                                   : perm_srv_wait(S, tickets[i], 30.0, out, &done, &lat);
            if (!done) {
                fprintf(stderr, "request %zu (n=%d) not done after 30 s\n", i, reqs[i].it.n);
                fflush(stderr);
                _Exit(3);
            }
            if (i & 1) {
                const double sum = tm.queued_us + tm.admitted_us + tm.running_us;
                const bool unstarted = rc == PERM_ECANCELED && tm.running_us == 0;
                if (tm.queued_us < 0 || tm.admitted_us < 0 || tm.running_us < 0 ||
                    std::fabs(sum - tm.latency_us) > 1e-6 * std::max(1.0, tm.latency_us) ||
                    (rc == PERM_OK && tm.admitted_us + tm.running_us <= 0 && !unstarted)) {
                    fprintf(stderr, "request %zu: phases %.3f %.3f %.3f us, latency %.3f us\n", i,
                            tm.queued_us, tm.admitted_us, tm.running_us, tm.latency_us);
                    ++wrong;
                }
            }
            if (cancel_every && i % cancel_every == 0 && rc == PERM_ECANCELED) continue;
            if (faults && rc == PERM_EDEVICE) {
                ++failed;
                continue;
            }
            uint64_t h, bad;
            memcpy(&h, out, 8);
            memcpy(&bad, out + 8, 8);
            if (rc != PERM_OK || h != sim_hash(reqs[i].m.data(), reqs[i].m.size()) || bad) {
                if (wrong < 5)
                    fprintf(stderr, "request %zu (n=%d): status %d, bad slots %llu\n", i, reqs[i].it.n,
                            rc, (unsigned long long)bad);
                ++wrong;
            }
        }
        sub.join();
        if (sub_failed) {
            fprintf(stderr, "a submit failed\n");
            wrong++;
        }
        perm_srv_stats st{};
        perm_srv_get_stats(S, &st);
        perm_srv_destroy(S);
        // every request is counted once: completed, failed or cancelled
        if (st.completed + st.failed + st.canceled != st.submitted) {
            fprintf(stderr, "stats: %llu completed + %llu failed + %llu canceled != %llu submitted\n",
                    (unsigned long long)st.completed, (unsigned long long)st.failed,
                    (unsigned long long)st.canceled, (unsigned long long)st.submitted);
            wrong++;
        }
        if (st.failed != (uint64_t)failed) {
            fprintf(stderr, "stats count %llu failed, the results %ld\n",
                    (unsigned long long)st.failed, failed);
            wrong++;
        }
        printf("rep %d: wrong %ld desync %ld bad_slots %ld items %ld slices %llu completed %llu canceled %llu failed %ld\n",
               rep, wrong, sim_desync.load(), sim_bad_parts.load(), sim_items.load(),
               (unsigned long long)st.slices, (unsigned long long)st.completed,
               (unsigned long long)st.canceled, failed);
    }
    fflush(stdout);
    fflush(stderr);
    // skip static destruction: the device thread is still polling its queues
    _Exit(wrong || sim_desync || sim_bad_parts ? 1 : 0);
}
