// Command-queue implementation of the HIP runtime test double.
#include "hip/hip_runtime.h"

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

namespace {

struct Cmd {
    std::function<void()> fn;
    SimEvent *wait_ev = nullptr;   // wait for this record of the event
    uint64_t wait_gen = 0;
};

}  // namespace

struct SimStream { std::deque<Cmd> q; };
struct SimEvent { uint64_t recorded = 0, completed = 0; double t_ms = 0; };

namespace {

// Leaked on purpose: the device thread may outlive static destruction.
std::mutex &mu = *new std::mutex;
std::vector<SimStream *> &streams = *new std::vector<SimStream *>;
SimStream *null_stream = nullptr;
std::mt19937_64 rng(getenv("SIM_SEED") ? strtoull(getenv("SIM_SEED"), nullptr, 10) : 12345);
bool started = false;

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

void device_loop()
{
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        std::vector<SimStream *> ready;
        for (SimStream *s : streams) {
            if (s->q.empty()) continue;
            const Cmd &c = s->q.front();
            if (c.wait_ev && c.wait_ev->completed < c.wait_gen) continue;
            ready.push_back(s);
        }
        if (ready.empty()) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
            continue;
        }
        SimStream *s = ready[rng() % ready.size()];
        Cmd c = std::move(s->q.front());
        s->q.pop_front();
        const bool nap = rng() % 8 == 0;
        const long nap_us = (long)(rng() % 200);
        lk.unlock();
        if (nap) std::this_thread::sleep_for(std::chrono::microseconds(nap_us));
        if (c.fn) c.fn();
        lk.lock();
    }
}

// with mu held
void start_locked()
{
    if (started) return;
    started = true;
    null_stream = new SimStream();
    streams.push_back(null_stream);
    std::thread(device_loop).detach();
}

void push_locked(hipStream_t s, Cmd c)
{
    start_locked();
    (s ? s : null_stream)->q.push_back(std::move(c));
}

// Block until every command enqueued on `s` so far has run.
void drain(hipStream_t s)
{
    SimEvent ev;
    {
        std::lock_guard<std::mutex> lk(mu);
        Cmd c;
        c.fn = [&ev] { std::lock_guard<std::mutex> l2(mu); ev.completed = 1; };
        push_locked(s, std::move(c));
    }
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (ev.completed) return;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

void sim_enqueue(hipStream_t s, std::function<void()> fn)
{
    std::lock_guard<std::mutex> lk(mu);
    Cmd c;
    c.fn = std::move(fn);
    push_locked(s, std::move(c));
}

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceCount(int *n)
{
    *n = 1;
    return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int)
{
    p->multiProcessorCount = 256;
    strcpy(p->gcnArchName, "simulated");
    p->totalGlobalMem = (size_t)1 << 36;
    return hipSuccess;
}
hipError_t hipMemcpy(void *d, const void *src, size_t n, hipMemcpyKind)
{
    drain(nullptr);
    memcpy(d, src, n);
    return hipSuccess;
}
hipError_t hipDeviceSynchronize()
{
    std::vector<SimStream *> all;
    {
        std::lock_guard<std::mutex> lk(mu);
        all = streams;
    }
    for (SimStream *s : all) drain(s == null_stream ? nullptr : s);
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    std::lock_guard<std::mutex> lk(mu);
    start_locked();
    *s = new SimStream();
    streams.push_back(*s);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) { drain(s); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }   // kept: the device thread may look at it
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned)
{
    std::lock_guard<std::mutex> lk(mu);
    Cmd c;
    c.wait_ev = e;
    c.wait_gen = e->recorded;
    push_locked(s, std::move(c));
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n)
{
    *p = aligned_alloc(256, (n + 255) & ~(size_t)255);
    if (!*p) return hipErrorInvalidValue;
    memset(*p, 0xA5, n);          // stale contents are visible, never zero by luck
    return hipSuccess;
}
hipError_t hipFree(void *p) { free(p); return hipSuccess; }
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void *p) { free(p); return hipSuccess; }
hipError_t hipHostGetDevicePointer(void **d, void *h, unsigned)
{
    *d = h;                        // one address space here
    return hipSuccess;
}
hipError_t hipMemset(void *p, int v, size_t n)
{
    sim_enqueue(nullptr, [=] { memset(p, v, n); });
    return hipSuccess;             // asynchronous like the real call may be
}
hipError_t hipMemsetAsync(void *p, int v, size_t n, hipStream_t s)
{
    sim_enqueue(s, [=] { memset(p, v, n); });
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *src, size_t n, hipMemcpyKind, hipStream_t s)
{
    sim_enqueue(s, [=] { memcpy(d, src, n); });
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) { *e = new SimEvent(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = new SimEvent(); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(mu);
    const uint64_t g = ++e->recorded;
    Cmd c;
    c.fn = [e, g] {
        std::lock_guard<std::mutex> l2(mu);
        if (e->completed < g) e->completed = g;
        e->t_ms = now_ms();
    };
    push_locked(s, std::move(c));
    return hipSuccess;
}
// Fault injection: SIM_FAIL_EVENT_SYNC=k makes the k-th hipEventSynchronize
// report an error once the event has completed (a device error noticed when
// the host waits for a slice).
hipError_t hipEventSynchronize(hipEvent_t e)
{
    static std::atomic<long> calls{0};
    static const long fail_at = getenv("SIM_FAIL_EVENT_SYNC") ? atol(getenv("SIM_FAIL_EVENT_SYNC")) : 0;
    const bool fail = fail_at > 0 && ++calls == fail_at;
    uint64_t g;
    {
        std::lock_guard<std::mutex> lk(mu);
        g = e->recorded;
    }
    const double t0 = now_ms();
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (e->completed >= g) return fail ? hipErrorInvalidValue : hipSuccess;
        }
        if (now_ms() - t0 > 30000) {
            fprintf(stderr, "SIM: an event wait took 30 s: the command queues are stuck\n");
            fflush(stderr);
            _Exit(3);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}
hipError_t hipEventQuery(hipEvent_t e)
{
    std::lock_guard<std::mutex> lk(mu);
    return e->completed >= e->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    std::lock_guard<std::mutex> lk(mu);
    *ms = (float)(b->t_ms - a->t_ms);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipRuntimeGetVersion(int *v)
{
    *v = 70200000;
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "simulated runtime error"; }
