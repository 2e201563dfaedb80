// Scenarios for the serving loop's host logic, run against the CPU stand-in
// for the device.  Usage: scenarios <mix|budget|errors|shutdown>; exit 0 on
// success, otherwise prints what failed.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "internal.h"

#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                \
        }                                                                \
    } while (0)

namespace {

struct Input {
    std::vector<double> f64;
    std::vector<float> f32;
    int dtype = SBS_F64;
    int64_t n = 0, m = 0;
    const void *ptr() const { return dtype == SBS_F64 ? (const void *)f64.data() : (const void *)f32.data(); }
    double at(int64_t k) const { return dtype == SBS_F64 ? f64[k] : (double)f32[k]; }
};

Input make_input(std::mt19937_64 &g, int64_t n, int64_t m, int dtype) {
    Input in;
    in.dtype = dtype;
    in.n = n;
    in.m = m;
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    if (dtype == SBS_F64) {
        in.f64.resize(n * m);
        for (double &v : in.f64) v = u(g);
    } else {
        in.f32.resize(n * m);
        for (float &v : in.f32) v = (float)u(g);
    }
    return in;
}

// Every column of the result was written by its own tile, from its own input.
bool result_matches(const double *x, const Input &in) {
    for (int64_t k = 0; k < in.n * in.m; ++k)
        if (x[k] != in.at(k)) return false;
    return true;
}

struct Lhs {
    std::vector<sbs_lhs> h;
    std::vector<int32_t> id;
    Lhs(sbs_server *srv, std::vector<int64_t> ns) : h(ns.size()), id(ns.size()) {
        for (size_t k = 0; k < ns.size(); ++k) {
            h[k] = sbs_lhs();
            h[k].kind = k & 1 ? SBS_PENTA : SBS_TRI;
            h[k].n = ns[k];
            CHECK(sbs_server_register(srv, &h[k], &id[k]) == SBS_OK);
        }
    }
};

// Many overlapping requests of mixed size, matrix and precision, each
// released as soon as it is done while later ones still run.
void mix() {
    sbs_server *srv = nullptr;
    CHECK(sbs_server_create(64u << 20, 4, 0, &srv) == SBS_OK);
    Lhs L(srv, {40, 77, 114, 151});
    std::mt19937_64 g(7);
    const int count = 600;
    std::vector<Input> in;
    std::vector<uint64_t> tk(count);
    std::vector<int> which(count);
    for (int r = 0; r < count; ++r) {
        which[r] = (int)(g() % 4);
        in.push_back(make_input(g, L.h[which[r]].n, 1 + (int64_t)(g() % 300), g() % 3 ? SBS_F64 : SBS_F32));
    }
    for (int r = 0; r < count; ++r)
        CHECK(sbs_server_submit(srv, L.id[which[r]], in[r].ptr(), in[r].m, in[r].dtype, &tk[r]) == SBS_OK);
    for (int r = 0; r < count; ++r) {
        const double *x = nullptr;
        double lat = -1;
        CHECK(sbs_server_wait(srv, tk[r], 20000000, &x, &lat) == SBS_OK);
        CHECK(x && lat >= 0);
        CHECK(result_matches(x, in[r]));
        CHECK(sbs_server_release(srv, tk[r]) == SBS_OK);
        CHECK(sbs_server_wait(srv, tk[r], 0, &x, &lat) == SBS_ERR_NOT_FOUND);
    }
    sbs_server_stats st;
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK);
    CHECK(st.submitted == (uint64_t)count && st.completed == (uint64_t)count);
    CHECK(st.in_flight == 0 && st.queued == 0 && st.bytes_reserved == 0);
    CHECK(st.launches >= 1 && st.launches < (uint64_t)count);  // requests were coalesced
    CHECK(st.p50_us > 0 && st.p99_us >= st.p50_us && st.max_us >= st.p99_us);
    CHECK(sbs_server_destroy(srv) == SBS_OK);
    std::printf("mix: %d requests in %lu launches\n", count, (unsigned long)st.launches);
}

// Admission follows the byte budget in arrival order; a request larger than
// the whole budget is refused at submission.
void budget() {
    const int64_t n = 200, m = 64;
    const size_t per = (size_t)n * m * 8;
    sbs_server *srv = nullptr;
    CHECK(sbs_server_create(3 * per, 2, 0, &srv) == SBS_OK);
    Lhs L(srv, {n});
    std::mt19937_64 g(3);
    Input big = make_input(g, n, 1000, SBS_F64);
    uint64_t t = 0;
    CHECK(sbs_server_submit(srv, L.id[0], big.ptr(), big.m, SBS_F64, &t) == SBS_ERR_BUDGET);
    std::vector<Input> in;
    std::vector<uint64_t> tk(8);
    for (int r = 0; r < 8; ++r) in.push_back(make_input(g, n, m, SBS_F64));
    for (int r = 0; r < 8; ++r) CHECK(sbs_server_submit(srv, L.id[0], in[r].ptr(), m, SBS_F64, &tk[r]) == SBS_OK);
    const double *x;
    double lat;
    for (int r = 0; r < 3; ++r) CHECK(sbs_server_wait(srv, tk[r], 20000000, &x, &lat) == SBS_OK);
    // nobody has released anything: the fourth cannot be admitted
    CHECK(sbs_server_wait(srv, tk[3], 50000, &x, &lat) == SBS_ERR_TIMEOUT);
    sbs_server_stats st;
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK);
    CHECK(st.completed == 3 && st.queued == 5 && st.rejected == 1 && st.bytes_reserved == 3 * per);
    for (int r = 0; r < 8; ++r) {
        CHECK(sbs_server_wait(srv, tk[r], 20000000, &x, &lat) == SBS_OK);
        CHECK(result_matches(x, in[r]));
        CHECK(sbs_server_release(srv, tk[r]) == SBS_OK);
    }
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK);
    CHECK(st.completed == 8 && st.bytes_reserved == 0);
    CHECK(sbs_server_destroy(srv) == SBS_OK);
    std::printf("budget: ok\n");
}

// Argument checks, unknown tickets, and release of an unfinished request.
void errors() {
    sbs_server *srv = nullptr;
    CHECK(sbs_server_create(0, 1, 0, &srv) == SBS_ERR_INVALID_ARG && !srv);
    CHECK(sbs_server_create(1 << 20, 17, 0, &srv) == SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_create(64u << 20, 1, 0, &srv) == SBS_OK);
    Lhs L(srv, {40});
    std::mt19937_64 g(5);
    Input in = make_input(g, 40, 64 * 2000, SBS_F64);
    uint64_t t = 0;
    CHECK(sbs_server_submit(srv, 5, in.ptr(), in.m, SBS_F64, &t) == SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_submit(srv, L.id[0], in.ptr(), 0, SBS_F64, &t) == SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_submit(srv, L.id[0], in.ptr(), 8, 7, &t) == SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_submit(srv, L.id[0], nullptr, 8, SBS_F64, &t) == SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_submit(srv, L.id[0], (const char *)in.ptr() + 4, 8, SBS_F64, &t) == SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_submit(srv, L.id[0], in.ptr(), in.m, SBS_F64, &t) == SBS_OK);
    // 2000 tiles take tens of milliseconds: the request is not done yet
    CHECK(sbs_server_release(srv, t) == SBS_ERR_INVALID_ARG);
    const double *x;
    double lat;
    CHECK(sbs_server_wait(srv, t + 1, 0, &x, &lat) == SBS_ERR_NOT_FOUND);
    CHECK(sbs_server_wait(srv, t, 20000000, &x, &lat) == SBS_OK);
    CHECK(result_matches(x, in));
    CHECK(sbs_server_release(srv, t) == SBS_OK);
    CHECK(sbs_server_release(srv, t) == SBS_ERR_NOT_FOUND);
    CHECK(sbs_server_destroy(srv) == SBS_OK);
    std::printf("errors: ok\n");
}

// Shutdown with requests running, finished-but-unreleased and still queued:
// everything admitted drains, queued requests are dropped, nothing leaks.
void shutdown() {
    const int64_t n = 100, m = 640;
    sbs_server *srv = nullptr;
    CHECK(sbs_server_create(2 * (size_t)n * m * 8, 2, 0, &srv) == SBS_OK);
    Lhs L(srv, {n});
    std::mt19937_64 g(9);
    std::vector<Input> in;
    std::vector<uint64_t> tk(6);
    for (int r = 0; r < 6; ++r) in.push_back(make_input(g, n, m, SBS_F64));
    for (int r = 0; r < 6; ++r) CHECK(sbs_server_submit(srv, L.id[0], in[r].ptr(), m, SBS_F64, &tk[r]) == SBS_OK);
    const double *x;
    double lat;
    CHECK(sbs_server_wait(srv, tk[0], 20000000, &x, &lat) == SBS_OK);
    CHECK(sbs_server_destroy(srv) == SBS_OK);
    std::printf("shutdown: ok\n");
}

// Per-request completion: one launch holds a long pentadiagonal request
// and short tridiagonal ones (the tridiagonal tiles run first); each short
// request is reported done, fetched and released while the long one is still
// running in the same launch, and its arena bytes are reused by a request
// admitted after it.
void early() {
    sbs_server *srv = nullptr;
    CHECK(sbs_server_create(64u << 20, 1, 0, &srv) == SBS_OK);
    Lhs L(srv, {64, 300});  // id 0 tridiagonal, id 1 pentadiagonal
    std::mt19937_64 g(11);
    Input big = make_input(g, 300, 64 * 400, SBS_F64);  // 400 tiles: about 8 ms
    std::vector<Input> small;
    for (int r = 0; r < 4; ++r) small.push_back(make_input(g, 64, 5 + r, r % 2 ? SBS_F32 : SBS_F64));
    uint64_t tb = 0;
    std::vector<uint64_t> ts(small.size());
    CHECK(sbs_server_submit(srv, L.id[1], big.ptr(), big.m, SBS_F64, &tb) == SBS_OK);
    for (size_t r = 0; r < small.size(); ++r)
        CHECK(sbs_server_submit(srv, L.id[0], small[r].ptr(), small[r].m, small[r].dtype, &ts[r]) == SBS_OK);
    const double *x;
    double lat;
    int early_done = 0;
    for (size_t r = 0; r < small.size(); ++r) {
        CHECK(sbs_server_wait(srv, ts[r], 20000000, &x, &lat) == SBS_OK);
        CHECK(result_matches(x, small[r]));
        if (sbs_server_wait(srv, tb, 0, &x, &lat) == SBS_ERR_TIMEOUT) ++early_done;
        CHECK(sbs_server_release(srv, ts[r]) == SBS_OK);
    }
    sbs_server_stats st;
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK);
    // all of them in the first launch (one slot, submitted together) ...
    CHECK(st.launches <= 2);
    // ... and finished while the long request still ran
    CHECK(early_done == (int)small.size());
    // a request admitted now reuses the released bytes and runs next
    Input again = make_input(g, 64, 9, SBS_F64);
    uint64_t ta = 0;
    CHECK(sbs_server_submit(srv, L.id[0], again.ptr(), again.m, SBS_F64, &ta) == SBS_OK);
    CHECK(sbs_server_wait(srv, tb, 20000000, &x, &lat) == SBS_OK);
    CHECK(result_matches(x, big));
    CHECK(sbs_server_wait(srv, ta, 20000000, &x, &lat) == SBS_OK);
    CHECK(result_matches(x, again));
    CHECK(sbs_server_release(srv, tb) == SBS_OK);
    CHECK(sbs_server_release(srv, ta) == SBS_OK);
    CHECK(sbs_server_destroy(srv) == SBS_OK);
    std::printf("early: %d short requests done while the long one ran\n", early_done);
}

// Many launches on several slots with requests released the moment each
// completes, in random order of completion checks: every request completes
// exactly once with its own columns, and nothing is touched after release.
void churn() {
    sbs_server *srv = nullptr;
    // the budget holds every request at once: results are waited for in a
    // shuffled order, so a request may be held (done, unreleased) while a
    // later one waits for admission
    CHECK(sbs_server_create(256u << 20, 3, 7, &srv) == SBS_OK);
    Lhs L(srv, {40, 90, 130, 260});
    std::mt19937_64 g(13);
    const int count = 400;
    std::vector<Input> in;
    std::vector<uint64_t> tk(count);
    for (int r = 0; r < count; ++r)
        in.push_back(make_input(g, L.h[r % 4].n, 1 + (int64_t)(g() % 200), g() % 2 ? SBS_F64 : SBS_F32));
    for (int r = 0; r < count; ++r)
        CHECK(sbs_server_submit(srv, L.id[r % 4], in[r].ptr(), in[r].m, in[r].dtype, &tk[r]) == SBS_OK);
    std::vector<int> order(count);
    for (int r = 0; r < count; ++r) order[r] = r;
    std::shuffle(order.begin(), order.end(), g);
    for (int r : order) {
        const double *x;
        double lat;
        CHECK(sbs_server_wait(srv, tk[r], 20000000, &x, &lat) == SBS_OK);
        CHECK(result_matches(x, in[r]));
        CHECK(sbs_server_release(srv, tk[r]) == SBS_OK);
    }
    sbs_server_stats st;
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK);
    CHECK(st.completed == (uint64_t)count && st.in_flight == 0 && st.bytes_reserved == 0);
    CHECK(sbs_server_destroy(srv) == SBS_OK);
    std::printf("churn: %d requests in %lu launches\n", count, (unsigned long)st.launches);
}

// FP32 requests submitted before and after sbs_server_set_fp32_mode keep the
// mode they were submitted with: the refined ones reserve three FP32 scratch
// arrays next to x and run as prec-1 tiles with them, the FP64-sweep ones reserve x
// only and run as prec-2 tiles without scratch (the mock device checks the
// tiles' prec and scratch).
void modes() {
    const int64_t n = 100, m = 70;
    const size_t x_bytes = (size_t)((n * m * 8 + 255) / 256 * 256), s_bytes = (size_t)((n * m * 12 + 255) / 256 * 256);
    sbs_server *srv = nullptr;
    CHECK(sbs_server_create(64u << 20, 2, 0, &srv) == SBS_OK);
    CHECK(sbs_server_set_fp32_mode(srv, 2) == SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_set_fp32_mode(srv, -1) == SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_set_fp32_mode(nullptr, SBS_SERVE_F32_REFINED) == SBS_ERR_INVALID_ARG);
    Lhs L(srv, {n, n});
    std::mt19937_64 g(11);
    std::vector<Input> in;
    std::vector<uint64_t> tk;
    for (int r = 0; r < 12; ++r) in.push_back(make_input(g, n, m, r % 3 == 2 ? SBS_F64 : SBS_F32));
    for (int r = 0; r < 12; ++r) {
        if (r == 6) CHECK(sbs_server_set_fp32_mode(srv, SBS_SERVE_F32_FP64_SWEEP) == SBS_OK);
        uint64_t t = 0;
        CHECK(sbs_server_submit(srv, L.id[r % 2], in[r].ptr(), m, in[r].dtype, &t) == SBS_OK);
        tk.push_back(t);
    }
    size_t want = 0;
    for (int r = 0; r < 12; ++r) want += x_bytes + (in[r].dtype == SBS_F32 && r < 6 ? s_bytes : 0);
    const double *x;
    double lat;
    for (int r = 0; r < 12; ++r) {
        CHECK(sbs_server_wait(srv, tk[r], 20000000, &x, &lat) == SBS_OK);
        CHECK(result_matches(x, in[r]));
    }
    sbs_server_stats st;
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK);
    CHECK(st.completed == 12 && st.bytes_reserved == want);
    for (int r = 0; r < 12; ++r) CHECK(sbs_server_release(srv, tk[r]) == SBS_OK);
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK && st.bytes_reserved == 0);
    CHECK(sbs_server_destroy(srv) == SBS_OK);
    std::printf("modes: 12 requests, %zu bytes reserved at the peak\n", want);
}

// The native trace replay: requests submitted at their arrival times by the
// calling thread, waited for and released in order by a second one; every
// latency filled in, nothing left reserved, a refused request reported as the
// first error with latency -1 while the others still run.
void replay() {
    sbs_server *srv = nullptr;
    CHECK(sbs_server_create(64u << 20, 3, 0, &srv) == SBS_OK);
    Lhs L(srv, {50, 90, 130});
    std::mt19937_64 g(5);
    const int count = 300;
    std::vector<Input> in;
    std::vector<int32_t> ids(count), dts(count);
    std::vector<const void *> ptrs(count);
    std::vector<int64_t> ms(count);
    std::vector<double> arr(count), lat(count, -2.0);
    for (int r = 0; r < count; ++r) {
        in.push_back(make_input(g, L.h[r % 3].n, 1 + (int64_t)(g() % 150), r % 2 ? SBS_F32 : SBS_F64));
        ids[r] = L.id[r % 3];
        ptrs[r] = in[r].ptr();
        ms[r] = in[r].m;
        dts[r] = in[r].dtype;
        arr[r] = 50.0 * r;
    }
    double el = -1;
    CHECK(sbs_server_replay(srv, count, ids.data(), ptrs.data(), ms.data(), dts.data(), arr.data(), lat.data(),
                            &el) == SBS_OK);
    CHECK(el >= 50e-6 * (count - 1));
    for (int r = 0; r < count; ++r) CHECK(lat[r] >= 0);
    sbs_server_stats st;
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK);
    CHECK(st.completed == (uint64_t)count && st.bytes_reserved == 0 && st.in_flight == 0);
    // closed loop, with one request refused (m = 0)
    ms[7] = 0;
    CHECK(sbs_server_replay(srv, count, ids.data(), ptrs.data(), ms.data(), dts.data(), nullptr, lat.data(), &el) ==
          SBS_ERR_INVALID_ARG);
    CHECK(lat[7] == -1.0);
    for (int r = 0; r < count; ++r)
        if (r != 7) CHECK(lat[r] >= 0);
    CHECK(sbs_server_stats_get(srv, &st) == SBS_OK);
    CHECK(st.completed == (uint64_t)(2 * count - 1) && st.bytes_reserved == 0);
    CHECK(sbs_server_replay(srv, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &el) == SBS_OK);
    CHECK(sbs_server_replay(nullptr, 1, ids.data(), ptrs.data(), ms.data(), dts.data(), nullptr, nullptr, nullptr) ==
          SBS_ERR_INVALID_ARG);
    CHECK(sbs_server_destroy(srv) == SBS_OK);
    std::printf("replay: %d requests, %.3f s\n", count, el);
}

}  // namespace

int main(int argc, char **argv) {
    const std::string s = argc > 1 ? argv[1] : "";
    if (s == "mix") mix();
    else if (s == "budget") budget();
    else if (s == "errors") errors();
    else if (s == "shutdown") shutdown();
    else if (s == "early") early();
    else if (s == "churn") churn();
    else if (s == "modes") modes();
    else if (s == "replay") replay();
    else {
        std::fprintf(stderr, "unknown scenario '%s'\n", s.c_str());
        return 2;
    }
    return 0;
}
