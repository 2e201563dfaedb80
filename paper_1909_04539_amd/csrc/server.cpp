// Serving loop: continuous batching of shared-LHS solves.
//
// Requests arrive on any thread (sbs_server_submit) and join a FIFO queue.
// One scheduler thread
//   1. retires finished requests and stamps their latencies: a request is
//      done when the wave that finishes its last tile raises the request's
//      flag in host memory (so a small request completes while the rest of
//      its launch still runs); a launch is retired when its event completes,
//   2. admits queued requests, in arrival order, while their result and
//      scratch bytes fit in the device arena (the HBM budget),
//   3. coalesces every admitted request into the next launch on a free
//      stream slot: each request is cut into tiles of 64 systems, the tiles
//      of one kind and precision go to one persistent tile kernel.
// Several slots (streams) run at once, so requests admitted while earlier
// launches are still running start at once and overlap them on the GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace sbs;
using Clock = std::chrono::steady_clock;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxTilesPerLaunch = 1 << 16;
constexpr int kGroups = 6;  // (tri, penta) x (fp64, fp32 refined, fp32 as one fp64 sweep)
constexpr int kPersistentWaves = 1024;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
   public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

   private:
    std::map<size_t, size_t> free_;
};

enum State { QUEUED, ADMITTED, RUNNING, DONE };

struct Req {
    uint64_t ticket = 0;
    int32_t lhs = 0;
    const void *rhs = nullptr;
    int64_t m = 0;
    int32_t dtype = SBS_F64;
    int32_t prec = 0;  // the tiles' prec (Tile): fixed at submission
    size_t bytes = 0, off = 0;
    double *x = nullptr;
    float *scratch = nullptr;
    State state = QUEUED;
    sbs_status status = SBS_OK;
    Clock::time_point t_submit, t_done;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    unsigned char *host = nullptr;  // pinned staging: tile counters, tiles left per request, tiles
    unsigned char *dev = nullptr;
    int *flag_host = nullptr;       // per request of the launch: set to 1 by the device when it is done
    int *flag_dev = nullptr;        // the same memory as the device addresses it
    // requests of the running launch, by their index in the flag array;
    // nullptr once a request has completed (it may then be released and freed
    // while the launch still runs)
    std::vector<Req *> reqs;
    bool busy = false;
};

// Staging layout of a slot: kGroups tile counters (one 64-byte line each),
// the tiles left of each request (max_batch ints), then the tiles.
size_t left_offset() { return kGroups * 64; }
size_t tiles_offset(int max_batch) { return round_up(left_offset() + (size_t)max_batch * 4, 64); }

}  // namespace

struct sbs_server {
    int device = 0;
    size_t budget = 0;
    unsigned char *arena_base = nullptr;
    Arena arena{0};
    int max_batch = 4096;
    int32_t fp32_mode = SBS_SERVE_F32_REFINED;  // how FP32 requests submitted from now on are solved
    std::vector<sbs_lhs *> lhs;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req *> queue;
    std::deque<Req *> ready;
    std::unordered_map<uint64_t, Req *> reqs;
    uint64_t next_ticket = 1;
    uint64_t kicks = 0;  // bumped by submit / release / destroy to wake the scheduler
    bool stop = false;
    std::thread worker;

    uint64_t submitted = 0, completed = 0, rejected = 0, launches = 0, in_flight = 0;
    size_t reserved = 0;
    double unknowns = 0;
    std::vector<double> lat_us;

    void loop();
    void finish(Req *r, sbs_status st, Clock::time_point now);
    void retire();
    void admit();
    bool launch(Slot &s);
};

void sbs_server::finish(Req *r, sbs_status st, Clock::time_point now) {
    r->state = DONE;
    r->t_done = now;
    r->status = st;
    lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
    ++completed;
    --in_flight;
    unknowns += (double)lhs[r->lhs]->n * (double)r->m;
}

void sbs_server::retire() {
    bool any = false;
    for (Slot &s : slots) {
        if (!s.busy) continue;
        // the event is queried first: if it has completed, every flag it
        // covers has been written
        const hipError_t q = hipEventQuery(s.done);
        const auto now = Clock::now();
        for (size_t k = 0; k < s.reqs.size(); ++k) {
            Req *r = s.reqs[k];
            if (!r) continue;
            if (__atomic_load_n(&s.flag_host[k], __ATOMIC_ACQUIRE) == 1) {
                finish(r, SBS_OK, now);
            } else if (q != hipErrorNotReady) {
                // launch over without this request's flag: only a failed launch
                finish(r, q == hipSuccess ? SBS_ERR_DEVICE : SBS_ERR_DEVICE, now);
            } else {
                continue;
            }
            s.reqs[k] = nullptr;
            any = true;
        }
        if (q != hipErrorNotReady) {
            s.reqs.clear();
            s.busy = false;
            any = true;
        }
    }
    if (any) cv_done.notify_all();
}

void sbs_server::admit() {
    while (!queue.empty()) {
        Req *r = queue.front();
        size_t off;
        if (!arena.alloc(r->bytes, &off)) break;  // FIFO: later requests wait too
        queue.pop_front();
        r->off = off;
        const sbs_lhs *h = lhs[r->lhs];
        r->x = reinterpret_cast<double *>(arena_base + off);
        r->scratch = r->prec == 1
                         ? reinterpret_cast<float *>(arena_base + off + round_up((size_t)h->n * r->m * 8, kAlign))
                         : nullptr;
        r->state = ADMITTED;
        reserved += r->bytes;
        ++in_flight;
        ready.push_back(r);
    }
}

bool sbs_server::launch(Slot &s) {
    // Take admitted requests in order until the tile table is full.
    std::vector<Req *> take;
    int tiles = 0;
    while (!ready.empty() && (int)take.size() < max_batch) {
        Req *r = ready.front();
        const int t = (int)((r->m + kWave - 1) / kWave);
        if (!take.empty() && tiles + t > kMaxTilesPerLaunch) break;
        take.push_back(r);
        tiles += t;
        ready.pop_front();
    }
    if (take.empty()) return false;

    // Group tiles by (kind, precision); inside a group, longest systems first.
    std::vector<Tile> grp[kGroups];
    int *left = reinterpret_cast<int *>(s.host + left_offset());
    for (size_t k = 0; k < take.size(); ++k) {
        Req *r = take[k];
        const sbs_lhs *h = lhs[r->lhs];
        const int g = (h->kind == SBS_PENTA ? 3 : 0) + r->prec;
        left[k] = (int)((r->m + kWave - 1) / kWave);
        s.flag_host[k] = 0;  // the slot's previous launch has completed: nothing writes it now
        for (int64_t c = 0; c < r->m; c += kWave) {
            Tile t;
            t.fac = r->prec == 1 ? h->fac32 : h->fac64;
            t.bands = h->bands;
            t.in = r->rhs;
            t.x = r->x;
            t.scratch = r->scratch;
            t.n = h->n;
            t.m = r->m;
            t.col0 = c;
            t.kind = h->kind;
            t.prec = r->prec;
            t.req = (int32_t)k;
            t.pad = 0;
            grp[g].push_back(t);
        }
        r->state = RUNNING;
    }
    size_t at = tiles_offset(max_batch);
    size_t offs[kGroups];
    for (int g = 0; g < kGroups; ++g) {
        std::stable_sort(grp[g].begin(), grp[g].end(), [](const Tile &a, const Tile &b) { return a.n > b.n; });
        offs[g] = at;
        if (!grp[g].empty()) std::memcpy(s.host + at, grp[g].data(), grp[g].size() * sizeof(Tile));
        at += grp[g].size() * sizeof(Tile);
    }
    std::memset(s.host, 0, kGroups * 64);
    hipError_t e = hipMemcpyAsync(s.dev, s.host, at, hipMemcpyHostToDevice, s.stream);
    for (int g = 0; g < kGroups && e == hipSuccess; ++g) {
        if (grp[g].empty()) continue;
        const int kind = g >= 3 ? SBS_PENTA : SBS_TRI;
        e = launch_tiles(kind, g % 3, reinterpret_cast<const Tile *>(s.dev + offs[g]), (int)grp[g].size(),
                         reinterpret_cast<int *>(s.dev + g * 64), reinterpret_cast<int *>(s.dev + left_offset()),
                         s.flag_dev, kPersistentWaves, s.stream);
    }
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    s.reqs = std::move(take);
    s.busy = true;
    ++launches;
    if (e != hipSuccess) {
        // Nothing will signal these requests: fail them now.  The slot
        // stays busy until its stream has drained whatever was queued.
        const auto now = Clock::now();
        for (Req *&r : s.reqs) {
            finish(r, SBS_ERR_DEVICE, now);
            r = nullptr;
        }
        if (hipStreamSynchronize(s.stream) == hipSuccess) {
            s.reqs.clear();
            s.busy = false;
        }
        cv_done.notify_all();
    }
    return true;
}

void sbs_server::loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    uint64_t seen = kicks;
    for (;;) {
        seen = kicks;
        retire();
        if (!stop) admit();
        bool any_busy = false;
        for (Slot &s : slots) {
            if (!s.busy && !ready.empty()) launch(s);
            any_busy |= s.busy;
        }
        if (stop && !any_busy && ready.empty()) break;
        if (any_busy)
            cv_sched.wait_for(lk, std::chrono::microseconds(20));
        else
            cv_sched.wait(lk, [&] { return stop || kicks != seen; });
    }
}

extern "C" {

sbs_status sbs_server_create(size_t budget_bytes, int32_t max_streams, int32_t max_batch_requests,
                             sbs_server **out) {
    if (!out) return SBS_ERR_INVALID_ARG;
    *out = nullptr;
    if (budget_bytes < kAlign || max_streams < 0 || max_streams > 16 || max_batch_requests < 0)
        return SBS_ERR_INVALID_ARG;
    sbs_server *s = new (std::nothrow) sbs_server();
    if (!s) return SBS_ERR_NO_MEMORY;
    s->budget = budget_bytes / kAlign * kAlign;
    s->arena = Arena(s->budget);
    s->max_batch = max_batch_requests ? max_batch_requests : 4096;
    const int ns = max_streams ? max_streams : 4;
    sbs_status st = SBS_OK;
    if (hipGetDevice(&s->device) != hipSuccess) st = SBS_ERR_DEVICE;
    if (st == SBS_OK && hipMalloc(reinterpret_cast<void **>(&s->arena_base), s->budget) != hipSuccess)
        st = SBS_ERR_NO_MEMORY;
    const size_t table = tiles_offset(s->max_batch) + (size_t)kMaxTilesPerLaunch * sizeof(Tile);
    s->slots.resize(ns);
    for (Slot &sl : s->slots) {
        if (st != SBS_OK) break;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            st = SBS_ERR_DEVICE;
        else if (hipHostMalloc(reinterpret_cast<void **>(&sl.host), table, hipHostMallocDefault) != hipSuccess ||
                 hipMalloc(reinterpret_cast<void **>(&sl.dev), table) != hipSuccess ||
                 hipHostMalloc(reinterpret_cast<void **>(&sl.flag_host), (size_t)s->max_batch * sizeof(int),
                               hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
            st = SBS_ERR_NO_MEMORY;
        else if (hipHostGetDevicePointer(reinterpret_cast<void **>(&sl.flag_dev), sl.flag_host, 0) != hipSuccess)
            st = SBS_ERR_DEVICE;
    }
    if (st == SBS_OK) {
        // no exception crosses the C ABI: a thread that cannot be started is
        // reported as a lack of resources
        try {
            s->worker = std::thread([s] { s->loop(); });
        } catch (...) {
            st = SBS_ERR_NO_MEMORY;
        }
    }
    if (st != SBS_OK) {
        for (Slot &sl : s->slots) {
            if (sl.dev) (void)hipFree(sl.dev);
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.flag_host) (void)hipHostFree(sl.flag_host);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        if (s->arena_base) (void)hipFree(s->arena_base);
        delete s;
        return st;
    }
    *out = s;
    return SBS_OK;
}

sbs_status sbs_server_register(sbs_server *srv, sbs_handle h, int32_t *lhs_id) {
    if (!srv || !h || !lhs_id) return SBS_ERR_INVALID_ARG;
    if (h->kind != SBS_TRI && h->kind != SBS_PENTA) return SBS_ERR_INVALID_ARG;  // tiles cover the banded kinds
    std::lock_guard<std::mutex> lk(srv->mu);
    try {
        srv->lhs.push_back(h);
    } catch (...) {  // no exception crosses the C ABI
        return SBS_ERR_NO_MEMORY;
    }
    *lhs_id = (int32_t)srv->lhs.size() - 1;
    return SBS_OK;
}

sbs_status sbs_server_set_fp32_mode(sbs_server *srv, int32_t mode) {
    if (!srv || (mode != SBS_SERVE_F32_REFINED && mode != SBS_SERVE_F32_FP64_SWEEP)) return SBS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->fp32_mode = mode;
    return SBS_OK;
}

sbs_status sbs_server_submit(sbs_server *srv, int32_t lhs_id, const void *rhs, int64_t m, int32_t dtype,
                             uint64_t *ticket) {
    if (!srv || !ticket || m < 1 || (dtype != SBS_F64 && dtype != SBS_F32) || !rhs) return SBS_ERR_INVALID_ARG;
    if ((m + kWave - 1) / kWave > kMaxTilesPerLaunch) return SBS_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(rhs) % (dtype == SBS_F64 ? 8 : 4)) return SBS_ERR_INVALID_ARG;
    Req *r = new (std::nothrow) Req();
    if (!r) return SBS_ERR_NO_MEMORY;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) {
        delete r;
        return SBS_ERR_SHUTDOWN;
    }
    if (lhs_id < 0 || lhs_id >= (int32_t)srv->lhs.size()) {
        delete r;
        return SBS_ERR_INVALID_ARG;
    }
    const sbs_lhs *h = srv->lhs[lhs_id];
    const size_t nm = (size_t)h->n * (size_t)m;
    const int32_t prec = dtype == SBS_F64 ? 0 : (srv->fp32_mode == SBS_SERVE_F32_FP64_SWEEP ? 2 : 1);
    // refined FP32 requests: three FP32 scratch arrays (x0, d1, r / d2) besides x
    r->bytes = round_up(nm * 8, kAlign) + (prec == 1 ? round_up(nm * 12, kAlign) : 0);
    if (r->bytes > srv->budget) {
        ++srv->rejected;
        delete r;
        return SBS_ERR_BUDGET;
    }
    r->ticket = srv->next_ticket++;
    r->lhs = lhs_id;
    r->rhs = rhs;
    r->m = m;
    r->dtype = dtype;
    r->prec = prec;
    r->t_submit = Clock::now();
    try {
        srv->reqs[r->ticket] = r;
        srv->queue.push_back(r);
    } catch (...) {  // no exception crosses the C ABI
        srv->reqs.erase(r->ticket);
        delete r;
        return SBS_ERR_NO_MEMORY;
    }
    ++srv->submitted;
    *ticket = r->ticket;
    ++srv->kicks;
    srv->cv_sched.notify_one();
    return SBS_OK;
}

sbs_status sbs_server_wait(sbs_server *srv, uint64_t ticket, int64_t timeout_us, const double **x_device,
                           double *latency_us) {
    if (!srv) return SBS_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return SBS_ERR_NOT_FOUND;
    Req *r = it->second;
    auto done = [&] { return r->state == DONE; };
    if (timeout_us < 0)
        srv->cv_done.wait(lk, done);
    else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done))
        return SBS_ERR_TIMEOUT;
    if (x_device) *x_device = r->status == SBS_OK ? r->x : nullptr;
    if (latency_us) *latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
    return r->status;
}

sbs_status sbs_server_fetch(sbs_server *srv, uint64_t ticket, double *dst, void *stream) {
    if (!srv || !dst) return SBS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return SBS_ERR_NOT_FOUND;
    Req *r = it->second;
    if (r->state != DONE || r->status != SBS_OK) return SBS_ERR_INVALID_ARG;
    const size_t bytes = (size_t)srv->lhs[r->lhs]->n * (size_t)r->m * sizeof(double);
    const hipError_t e = hipMemcpyAsync(dst, r->x, bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBS_OK : SBS_ERR_DEVICE;
}

sbs_status sbs_server_release(sbs_server *srv, uint64_t ticket) {
    if (!srv) return SBS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return SBS_ERR_NOT_FOUND;
    Req *r = it->second;
    if (r->state != DONE) return SBS_ERR_INVALID_ARG;  // only finished requests give bytes back
    if (r->bytes && r->x) {
        srv->arena.release(r->off, r->bytes);
        srv->reserved -= r->bytes;
    }
    srv->reqs.erase(it);
    delete r;
    ++srv->kicks;
    srv->cv_sched.notify_one();
    return SBS_OK;
}

sbs_status sbs_server_replay(sbs_server *srv, int64_t count, const int32_t *lhs_ids, const void *const *rhs,
                             const int64_t *m, const int32_t *dtype, const double *arrival_us, double *latency_us,
                             double *elapsed_s) {
    if (!srv || count < 0 || (count > 0 && (!lhs_ids || !rhs || !m || !dtype))) return SBS_ERR_INVALID_ARG;
    std::vector<uint64_t> ticket;
    try {
        ticket.assign((size_t)count, 0);
    } catch (...) {  // no exception crosses the C ABI
        return SBS_ERR_NO_MEMORY;
    }
    std::unique_ptr<std::atomic<int>[]> posted(new (std::nothrow) std::atomic<int>[(size_t)count]);
    if (count > 0 && !posted) return SBS_ERR_NO_MEMORY;
    for (int64_t k = 0; k < count; ++k) posted[k].store(0, std::memory_order_relaxed);
    std::atomic<int> first_error{SBS_OK};
    auto note = [&](sbs_status st) {
        int ok = SBS_OK;
        if (st != SBS_OK) first_error.compare_exchange_strong(ok, (int)st);
    };
    const auto t0 = Clock::now();
    Clock::time_point t_end = t0;
    // waits for and releases the requests in order, as the submitter posts them
    std::thread waiter;
    auto wait_all = [&] {
        for (int64_t k = 0; k < count; ++k) {
            int p;
            while ((p = posted[k].load(std::memory_order_acquire)) == 0) std::this_thread::yield();
            if (p < 0) {
                if (latency_us) latency_us[k] = -1.0;
                continue;
            }
            double lat = -1.0;
            note(sbs_server_wait(srv, ticket[k], -1, nullptr, &lat));
            note(sbs_server_release(srv, ticket[k]));
            if (latency_us) latency_us[k] = lat;
        }
        t_end = Clock::now();
    };
    try {
        waiter = std::thread(wait_all);
    } catch (...) {  // no exception crosses the C ABI
        return SBS_ERR_NO_MEMORY;
    }
    for (int64_t k = 0; k < count; ++k) {
        if (arrival_us) {
            const auto due = t0 + std::chrono::duration_cast<Clock::duration>(
                                      std::chrono::duration<double, std::micro>(arrival_us[k]));
            while (Clock::now() < due) {
            }
        }
        const sbs_status st = sbs_server_submit(srv, lhs_ids[k], rhs[k], m[k], dtype[k], &ticket[k]);
        note(st);
        posted[k].store(st == SBS_OK ? 1 : -1, std::memory_order_release);
    }
    waiter.join();
    if (elapsed_s) *elapsed_s = std::chrono::duration<double>(t_end - t0).count();
    return (sbs_status)first_error.load();
}

sbs_status sbs_server_stats_get(sbs_server *srv, sbs_server_stats *out) {
    if (!srv || !out) return SBS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->launches = srv->launches;
    out->queued = srv->queue.size();
    out->in_flight = srv->in_flight;
    out->bytes_reserved = srv->reserved;
    out->budget_bytes = srv->budget;
    out->unknowns = srv->unknowns;
    if (!srv->lat_us.empty()) {
        std::vector<double> v = srv->lat_us;
        auto pct = [&](double p) {
            const size_t k = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
            std::nth_element(v.begin(), v.begin() + k, v.end());
            return v[k];
        };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
        out->max_us = *std::max_element(v.begin(), v.end());
    }
    return SBS_OK;
}

sbs_status sbs_server_destroy(sbs_server *srv) {
    if (!srv) return SBS_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        // Requests still waiting for admission will never run.
        for (Req *r : srv->queue) {
            r->state = DONE;
            r->status = SBS_ERR_SHUTDOWN;
            r->t_done = Clock::now();
        }
        srv->queue.clear();
        ++srv->kicks;
        srv->cv_sched.notify_all();
        srv->cv_done.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();  // drains admitted and running work
    sbs_status st = SBS_OK;
    for (Slot &sl : srv->slots) {
        if (sl.stream && hipStreamSynchronize(sl.stream) != hipSuccess) st = SBS_ERR_DEVICE;
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.flag_host) (void)hipHostFree(sl.flag_host);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (srv->arena_base && hipFree(srv->arena_base) != hipSuccess) st = SBS_ERR_DEVICE;
    for (auto &kv : srv->reqs) delete kv.second;
    delete srv;
    return st;
}

}  // extern "C"
