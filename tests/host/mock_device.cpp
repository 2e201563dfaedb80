// A CPU stand-in for the device calls the serving loop makes, so that its
// host logic (admission, batching, completion, release, shutdown)
// runs on the CPU under AddressSanitizer.  Each stream is a worker thread that
// runs its queued operations in order; an event completes when its stream
// reaches it.  The tile "kernel" takes tiles in table order and copies each
// tile's input columns into the request's result, so a test can see which
// columns ran and where they went.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>

#include "internal.h"

struct ihipEvent_t {
    std::atomic<int> pending{0};
};

struct ihipStream_t {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> ops;
    bool stop = false, running = false;
    std::thread th;
    ihipStream_t() {
        th = std::thread([this] {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                cv.wait(lk, [&] { return stop || !ops.empty(); });
                if (ops.empty()) break;
                auto f = std::move(ops.front());
                ops.pop_front();
                running = true;
                lk.unlock();
                f();
                lk.lock();
                running = false;
                cv.notify_all();
            }
        });
    }
    void push(std::function<void()> f) {
        std::lock_guard<std::mutex> lk(mu);
        ops.push_back(std::move(f));
        cv.notify_all();
    }
    void drain() {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return ops.empty() && !running; });
    }
};

extern "C" {
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n) {
    const size_t bytes = (n + 255) / 256 * 256;  // device allocations are 256-byte aligned
    *p = aligned_alloc(256, bytes ? bytes : 256);
    if (*p) memset(*p, 0, bytes ? bytes : 256);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
    free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipHostGetDevicePointer(void **d, void *h, unsigned int) {
    *d = h;  // one address space on the CPU
    return hipSuccess;
}
hipError_t hipHostFree(void *p) { return hipFree(p); }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    *s = new ihipStream_t();
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    s->drain();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    s->th.join();
    delete s;
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
    *e = new ihipEvent_t();
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    e->pending.fetch_add(1);
    s->push([e] { e->pending.fetch_sub(1); });
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) { return e->pending.load() ? hipErrorNotReady : hipSuccess; }
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
    memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t s) {
    if (!s) {
        memcpy(dst, src, n);
        return hipSuccess;
    }
    s->push([=] { memcpy(dst, src, n); });
    return hipSuccess;
}
}  // extern "C"

namespace sbs {
// The tile kernel's completion protocol as the device runs it: after its
// tile a "wave" takes one from the request's count of tiles left (acquire and
// release), and the one that takes the last raises the request's flag with a
// release store; the host reads the flag with an acquire load.
hipError_t launch_tiles(int kind, int prec, const Tile *tiles, int ntiles, int *counter, int *left, int *done, int,
                        hipStream_t s) {
    s->push([=] {
        for (int t = 0; t < ntiles; ++t) {
            const Tile &tl = tiles[t];
            if (tl.kind != kind || tl.prec != prec) std::abort();  // a launch holds one (kind, prec) group
            // FP32 requests: the refined tiles use their scratch, the FP64-sweep tiles have none
            if ((prec == 1) != (tl.scratch != nullptr)) std::abort();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            const int64_t j1 = tl.col0 + 64 < tl.m ? tl.col0 + 64 : tl.m;
            for (int64_t i = 0; i < tl.n; ++i)
                for (int64_t j = tl.col0; j < j1; ++j) {
                    const int64_t k = i * tl.m + j;
                    tl.x[k] = tl.prec ? (double)static_cast<const float *>(tl.in)[k]
                                      : static_cast<const double *>(tl.in)[k];
                }
            const int before = __atomic_fetch_sub(&left[tl.req], 1, __ATOMIC_ACQ_REL);
            if (before < 1) std::abort();  // more tiles than the request was given
            if (before == 1) __atomic_store_n(&done[tl.req], 1, __ATOMIC_RELEASE);
        }
        *counter = ntiles;
    });
    return hipSuccess;
}
}  // namespace sbs
