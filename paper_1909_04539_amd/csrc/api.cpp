// C-ABI entry points: argument checking, the host-side FP64 factorisation of
// the shared matrix, its upload, and dispatch to the HIP kernels.
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "factor_rows.h"
#include "internal.h"

using namespace sbs;

namespace {

// Coefficient k of row i of a row-aligned band array, 0 outside the matrix.
double coef(const double *bands, int kind, int64_t n, int k, int64_t i) {
    const int64_t col = i + k - kind / 2;
    if (col < 0 || col >= n) return 0.0;
    return bands[(int64_t)k * n + i];
}

template <typename Row32, typename Row64>
Row32 narrow(const Row64 &r);
template <>
TriRow<float> narrow(const TriRow<double> &r) {
    return {(float)r.a_s, (float)r.chat, (float)r.inv, 0.0f};
}
template <>
PentaRow<float> narrow(const PentaRow<double> &r) {
    return {(float)r.eps_s, (float)r.beta_s, (float)r.inv, (float)r.gamma, (float)r.delta, 0.f, 0.f, 0.f};
}
template <>
PeriodicRow<float> narrow(const PeriodicRow<double> &r) {
    return {(float)r.a_s, (float)r.chat, (float)r.inv, (float)r.wt, (float)r.z, 0.f, 0.f, 0.f};
}

int nbands(int kind) { return kind == SBS_TRI_PERIODIC ? 3 : kind; }

// Whether each band holds one value wherever it lies inside the matrix (every
// row of a periodic matrix); if so, those values.  A band with no entry inside
// (a penta band of a 1-row matrix) counts as constant 0.
bool constant_bands(const double *bands, int kind, int64_t n, BandCoef *c) {
    const int nb = nbands(kind), H = nb / 2;
    for (int k = 0; k < nb; ++k) {
        bool have = false;
        c->c[k] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t col = i + k - H;
            if (kind != SBS_TRI_PERIODIC && (col < 0 || col >= n)) continue;
            const double v = bands[(int64_t)k * n + i];
            if (!have) {
                c->c[k] = v;
                have = true;
            } else if (v != c->c[k]) {
                return false;
            }
        }
    }
    return true;
}

// Band k of row i as the matrix uses it: 0 outside a banded matrix; every
// entry (the corners a_0 and c_{n-1} included) for a periodic one.
double entry(const double *bands, int kind, int64_t n, int k, int64_t i) {
    return kind == SBS_TRI_PERIODIC ? bands[(int64_t)k * n + i] : coef(bands, kind, n, k, i);
}

template <typename Row64, typename Row32>
sbs_status upload(sbs_lhs *h, const std::vector<Row64> &r64, const double *B) {
    const int64_t rows = h->rows;
    const size_t b64 = sizeof(Row64) * rows, b32 = sizeof(Row32) * rows, bb = sizeof(BandRow) * rows;
    const size_t total = b64 + b32 + bb;
    std::vector<unsigned char> host(total, 0);  // padding rows stay zero
    std::memcpy(host.data(), r64.data(), sizeof(Row64) * h->n);
    Row32 *p32 = reinterpret_cast<Row32 *>(host.data() + b64);
    for (int64_t i = 0; i < h->n; ++i) p32[i] = narrow<Row32>(r64[i]);
    BandRow *pb = reinterpret_cast<BandRow *>(host.data() + b64 + b32);
    for (int64_t i = 0; i < h->n; ++i)
        for (int k = 0; k < nbands(h->kind); ++k) pb[i].c[k] = entry(B, h->kind, h->n, k, i);

    if (hipGetDevice(&h->device) != hipSuccess) return SBS_ERR_DEVICE;
    void *dev = nullptr;
    if (hipMalloc(&dev, total) != hipSuccess) return SBS_ERR_NO_MEMORY;
    if (hipMemcpy(dev, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dev);
        return SBS_ERR_DEVICE;
    }
    h->dev = dev;
    h->fac64 = dev;
    h->fac32 = static_cast<unsigned char *>(dev) + b64;
    h->bands = reinterpret_cast<BandRow *>(static_cast<unsigned char *>(dev) + b64 + b32);
    h->device_bytes = (int64_t)total;
    return SBS_OK;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Which partitioned form runs: the separator kernel when it fills the GPU
// with whole row runs from a plan in LDS; else the pair kernel; else a
// separator shape (for AUTO only one whose plan sits in LDS or whose row
// runs are at least 128 bytes: a plan read from global memory with shorter
// runs loses to the chunked sweep).  A plan read from global memory loses
// to the pair form (random-band pentadiagonal n = 1024: 263.6 us against
// 225.6 us), so it runs only where the pair form has no plan.
// 0: none (AUTO then runs the sweeps), 1: separator, 2: pair.
int pick_uncached(const sbs_lhs *h, int t, int64_t m, const void *rhs, bool for_auto, sbs::SepChoice *sc,
                  sbs::PartChoice *pc) {
    const bool sep = sbs::choose_sep(h, t, m, rhs, sc);
    const bool part = sbs::choose_partition(h, t, m, pc);
    if (sep && !sc->gf && sbs::sep_fills(h, t, m, *sc)) return 1;
    // too few systems to fill the chip with whole row runs: where the pair
    // form would take 64-row blocks of at most 16 systems (128-byte runs),
    // the separator form's 32-row blocks with two systems per lane and 16
    // per workgroup (plan in LDS) finish sooner (tridiagonal n = 2048,
    // m = 2048: 15.4 against 19.0 us; pentadiagonal n = 1024, m = 2048: 11.7
    // against 16.5 us; tridiagonal n = 2048, m = 8192: 63.7 against
    // 67.8 us); against shorter pair blocks it was not faster throughout,
    // and where the pair form has 256-byte runs those are worth more
    if (part && t == 0 && h->part[pc->plan].lb == 64 && pc->S <= 16) {
        sbs::SepChoice alt;
        if (sbs::sep_shape(h, t, m, rhs, 32, 2, 16, 0, &alt) && !alt.gf) {
            *sc = alt;
            return 1;
        }
    }
    // pentadiagonal, where the pair form would take 32-row blocks of at most
    // 16 systems: 16-row separator blocks, one system per lane, 16 per
    // workgroup (n = 512, m = 4096: 10.0 against 11.7 us; n = 384,
    // m = 2048: 8.7 against 10.2 us; n = 512, m = 1024: 8.9 against 9.5 us;
    // for tridiagonal matrices the two were even)
    if (part && t == 0 && h->kind == SBS_PENTA && h->part[pc->plan].lb == 32 && pc->S <= 16) {
        sbs::SepChoice alt;
        if (sbs::sep_shape(h, t, m, rhs, 16, 1, 16, 0, &alt) && !alt.gf) {
            *sc = alt;
            return 1;
        }
    }
    if (part) return 2;
    const size_t elem = t == 0 ? 8 : 4;
    if (sep && (!for_auto || !sc->gf || (size_t)sc->S * elem >= 128)) return 1;
    return 0;
}

// The choice depends on the handle, the dtype, m, whether rhs is aligned for
// two systems per lane and AUTO or not; it is made once and kept (weighing
// every shape costs several microseconds, as much as a small solve).
int pick_partition(const sbs_lhs *h, int t, int64_t m, const void *rhs, bool for_auto, sbs::SepChoice *sc,
                   sbs::PartChoice *pc) {
    struct Pick {
        int form;
        sbs::SepChoice sc;
        sbs::PartChoice pc;
    };
    static std::mutex mu;
    static std::map<std::tuple<uint64_t, int, int64_t, bool, bool>, Pick> known;
    const bool al = reinterpret_cast<uintptr_t>(rhs) % (2 * (t == 0 ? 8 : 4)) == 0;
    const auto key = std::make_tuple(h->id, t, m, al, for_auto);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = known.find(key);
        if (it != known.end()) {
            *sc = it->second.sc;
            *pc = it->second.pc;
            return it->second.form;
        }
    }
    const int form = pick_uncached(h, t, m, rhs, for_auto, sc, pc);
    std::lock_guard<std::mutex> g(mu);
    if (known.size() >= 4096) known.clear();  // bounded: many batch sizes only cost a new choice
    known[key] = Pick{form, *sc, *pc};
    return form;
}

}  // namespace

namespace sbs {

int device_cus(int device) {
    static std::mutex mu;
    static std::map<int, int> known;
    std::lock_guard<std::mutex> g(mu);
    auto it = known.find(device);
    if (it != known.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
        return 256;  // not kept: asked again next time
    known[device] = cus;
    return cus;
}

int occupancy(const void *fn, int threads, size_t lds) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t, int>, int> known;
    const auto key = std::make_tuple(fn, threads, lds, dev);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = known.find(key);
        if (it != known.end()) return it->second;
    }
    int wgs = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&wgs, fn, threads, lds) != hipSuccess) return 0;
    std::lock_guard<std::mutex> g(mu);
    known[key] = wgs;
    return wgs;
}

sbs_status refined_check(const sbs_lhs *h, const float *b, const double *x, int64_t m, int32_t sweeps) {
    if (!h || m < 0 || sweeps < 0 || sweeps > 8 || h->kind == SBS_TRI_PERIODIC) return SBS_ERR_INVALID_ARG;
    if (m == 0) return SBS_OK;
    if (!b || !x || !aligned(b, 8) || !aligned(x, 16)) return SBS_ERR_INVALID_ARG;
    const size_t nb = (size_t)h->n * (size_t)m;
    const char *bx = reinterpret_cast<const char *>(x), *bbp = reinterpret_cast<const char *>(b);
    if (bx < bbp + nb * 4 && bbp < bx + nb * 8) return SBS_ERR_INVALID_ARG;  // b and x overlap
    return SBS_OK;
}

bool refined_fused(const sbs_lhs *h, int64_t m) {
    RefwChoice rc;
    PartChoice pc;
    return choose_refine_wave(h, m, &rc) || choose_partition_refine(h, m, &pc);
}

sbs_status refined_run(const sbs_lhs *h, const float *b, double *x, int64_t m, int32_t sweeps, float *r,
                       hipStream_t s) {
    // Fused paths: one kernel keeps each block of b and x on chip through all
    // passes (needs a partition plan); r is not touched.  First the
    // one-wave-per-block kernel on the separator plan, then the pair form.
    RefwChoice rc;
    if (choose_refine_wave(h, m, &rc))
        return launch_refine_wave(h, rc, b, x, m, sweeps, s) == hipSuccess ? SBS_OK : SBS_ERR_DEVICE;
    PartChoice pc;
    if (choose_partition_refine(h, m, &pc))
        return launch_partition_refine(h, pc, b, x, m, sweeps, s) == hipSuccess ? SBS_OK : SBS_ERR_DEVICE;
    // x0 = FP32 solve of b, written as FP64.  r is written in full by the
    // first residual pass before anything reads it.
    hipError_t e = launch_sweep(h, SBS_VARIANT_AUTO, 1, 1, 0, b, x, m, s);
    for (int k = 0; k < sweeps && e == hipSuccess; ++k) {
        // r = fl32(b - A x)   (on later passes fused with x += delta)
        e = launch_refine_step(h, k == 0 ? 0 : 1, b, x, r, r, m, s);
        if (e == hipSuccess) e = launch_sweep(h, SBS_VARIANT_AUTO, 1, 1, 1, r, r, m, s);  // delta
    }
    if (e == hipSuccess && sweeps > 0) e = launch_refine_step(h, 2, b, x, r, nullptr, m, s);  // x += delta
    return e == hipSuccess ? SBS_OK : SBS_ERR_DEVICE;
}

}  // namespace sbs

extern "C" {

const char *sbs_status_str(sbs_status s) {
    switch (s) {
        case SBS_OK: return "ok";
        case SBS_ERR_INVALID_ARG: return "invalid argument";
        case SBS_ERR_ZERO_PIVOT: return "zero or non-finite pivot";
        case SBS_ERR_NONFINITE: return "non-finite matrix coefficient";
        case SBS_ERR_DEVICE: return "device error";
        case SBS_ERR_NO_MEMORY: return "out of memory";
        case SBS_ERR_BUDGET: return "request exceeds the memory budget";
        case SBS_ERR_NOT_FOUND: return "not found";
        case SBS_ERR_TIMEOUT: return "timed out";
        case SBS_ERR_SHUTDOWN: return "server shutting down";
    }
    return "unknown status";
}

const char *sbs_version(void) { return "sbs 0.1 (gfx950)"; }

sbs_status sbs_factor_shared_lhs(int32_t kind, int64_t n, const double *bands, sbs_handle *out,
                                 int64_t *bad_row) {
    int64_t bad = -1;
    if (bad_row) *bad_row = -1;
    if (out) *out = nullptr;
    if (!out || !bands || n < 1 || (kind != SBS_TRI && kind != SBS_PENTA && kind != SBS_TRI_PERIODIC))
        return SBS_ERR_INVALID_ARG;
    // the kernels index rows with 32-bit integers
    if (n > (int64_t)INT32_MAX || (kind == SBS_TRI_PERIODIC && n < 3)) return SBS_ERR_INVALID_ARG;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < nbands(kind); ++k)
            if (!std::isfinite(entry(bands, kind, n, k, i))) {
                if (bad_row) *bad_row = i;
                return SBS_ERR_NONFINITE;
            }
    sbs_lhs *h = new (std::nothrow) sbs_lhs();
    if (!h) return SBS_ERR_NO_MEMORY;
    static std::atomic<uint64_t> next_id{1};
    h->id = next_id++;
    h->kind = kind;
    h->n = n;
    h->rows = (n + kRowPad - 1) / kRowPad * kRowPad;
    sbs_status st;
    try {
        auto cf = [&](int k, int64_t i) { return entry(bands, kind, n, k, i); };
        if (kind == SBS_TRI) {
            std::vector<TriRow<double>> r(n);
            st = factor_tri_rows(n, cf, r.data(), &bad) ? SBS_OK : SBS_ERR_ZERO_PIVOT;
            if (st == SBS_OK) st = upload<TriRow<double>, TriRow<float>>(h, r, bands);
        } else if (kind == SBS_PENTA) {
            std::vector<PentaRow<double>> r(n);
            st = factor_penta_rows(n, cf, r.data(), &bad) ? SBS_OK : SBS_ERR_ZERO_PIVOT;
            if (st == SBS_OK) st = upload<PentaRow<double>, PentaRow<float>>(h, r, bands);
        } else {
            std::vector<PeriodicRow<double>> r(n);
            st = factor_periodic_rows(n, cf, r.data(), &bad) ? SBS_OK : SBS_ERR_ZERO_PIVOT;
            if (st == SBS_OK) st = upload<PeriodicRow<double>, PeriodicRow<float>>(h, r, bands);
        }
        if (st == SBS_OK) st = build_partitions(h, bands);
        h->constant_bands = constant_bands(bands, kind, n, &h->coef);
    } catch (const std::bad_alloc &) {
        st = SBS_ERR_NO_MEMORY;
    }
    if (st != SBS_OK) {
        if (bad_row) *bad_row = bad;
        sbs_release(h);
        return st;
    }
    *out = h;
    return SBS_OK;
}

sbs_status sbs_factor_uniform(int32_t kind, int64_t n, const double *coeffs, sbs_handle *out, int64_t *bad_row) {
    if (bad_row) *bad_row = -1;
    if (out) *out = nullptr;
    if (!out || !coeffs || n < 1 || n > (int64_t)INT32_MAX) return SBS_ERR_INVALID_ARG;
    if (kind != SBS_TRI && kind != SBS_PENTA && kind != SBS_TRI_PERIODIC) return SBS_ERR_INVALID_ARG;
    const int nb = nbands(kind);
    std::vector<double> bands;
    try {
        bands.resize((size_t)nb * n);
    } catch (const std::bad_alloc &) {
        return SBS_ERR_NO_MEMORY;
    }
    for (int k = 0; k < nb; ++k)
        for (int64_t i = 0; i < n; ++i) bands[(size_t)k * n + i] = coeffs[k];
    return sbs_factor_shared_lhs(kind, n, bands.data(), out, bad_row);
}

sbs_status sbs_release(sbs_handle h) {
    if (!h) return SBS_OK;
    sbs_status st = SBS_OK;
    if (h->dev && hipFree(h->dev) != hipSuccess) st = SBS_ERR_DEVICE;
    if (h->pdev && hipFree(h->pdev) != hipSuccess) st = SBS_ERR_DEVICE;
    delete h;
    return st;
}

sbs_status sbs_handle_info(sbs_handle h, int32_t *kind, int64_t *n, int64_t *device_bytes) {
    if (!h) return SBS_ERR_INVALID_ARG;
    if (kind) *kind = h->kind;
    if (n) *n = h->n;
    if (device_bytes) *device_bytes = h->device_bytes;
    return SBS_OK;
}

sbs_status sbs_solve_batch_variant(sbs_handle h, void *rhs, int64_t m, int32_t dtype, int32_t variant,
                                   void *stream) {
    if (!h || m < 0 || (dtype != SBS_F64 && dtype != SBS_F32)) return SBS_ERR_INVALID_ARG;
    if (variant < SBS_VARIANT_AUTO || variant > SBS_VARIANT_PARTITION) return SBS_ERR_INVALID_ARG;
    if (variant == SBS_VARIANT_RESIDENT && h->n > 64) return SBS_ERR_INVALID_ARG;
    if (m == 0) return SBS_OK;
    if (!rhs || !aligned(rhs, dtype == SBS_F64 ? 8 : 4)) return SBS_ERR_INVALID_ARG;
    if (m > (int64_t)0x7fffffff * kWave) return SBS_ERR_INVALID_ARG;
    if (variant == SBS_VARIANT_CHUNKED && chunked_lds_bytes(h, dtype == SBS_F64 ? 0 : 1) > kMaxLdsBytes)
        return SBS_ERR_INVALID_ARG;
    const int t = dtype == SBS_F64 ? 0 : 1;
    hipError_t e;
    if (variant == SBS_VARIANT_AUTO || variant == SBS_VARIANT_PARTITION) {
        SepChoice sc;
        PartChoice pc;
        const int form = pick_partition(h, t, m, rhs, variant == SBS_VARIANT_AUTO, &sc, &pc);
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (form == 1)
            e = launch_sep(h, sc, t, rhs, m, s);
        else if (form == 2)
            e = launch_partition(h, pc, t, t, t, rhs, rhs, m, s);
        else if (variant == SBS_VARIANT_PARTITION)
            return SBS_ERR_INVALID_ARG;
        else
            e = launch_sweep(h, variant, t, t, t, rhs, rhs, m, s);
        return e == hipSuccess ? SBS_OK : SBS_ERR_DEVICE;
    }
    e = launch_sweep(h, variant, t, t, t, rhs, rhs, m, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBS_OK : SBS_ERR_DEVICE;
}

sbs_status sbs_solve_batch_partition(sbs_handle h, void *rhs, int64_t m, int32_t dtype, int32_t form, int32_t lb,
                                     int32_t vec, int32_t S, int32_t flags, void *stream) {
    if (!h || m < 0 || (dtype != SBS_F64 && dtype != SBS_F32) || (form != 0 && form != 1)) return SBS_ERR_INVALID_ARG;
    if (m == 0) return SBS_OK;
    if (!rhs || !aligned(rhs, dtype == SBS_F64 ? 8 : 4) || m > (int64_t)0x7fffffff * kWave) return SBS_ERR_INVALID_ARG;
    const int t = dtype == SBS_F64 ? 0 : 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (form == 1) {
        SepChoice sc;
        if (flags < 0 || flags > 0xffff || !sep_shape(h, t, m, rhs, lb, vec, S, flags, &sc)) return SBS_ERR_INVALID_ARG;
        e = launch_sep(h, sc, t, rhs, m, s);
    } else {
        PartChoice pc;
        if (vec != 1 || flags != 0 || !part_shape(h, t, m, lb, S, &pc)) return SBS_ERR_INVALID_ARG;
        e = launch_partition(h, pc, t, t, t, rhs, rhs, m, s);
    }
    return e == hipSuccess ? SBS_OK : SBS_ERR_DEVICE;
}

sbs_status sbs_partition_shape(sbs_handle h, int64_t m, int32_t dtype, const void *rhs, int32_t *form, int32_t *lb,
                               int32_t *vec, int32_t *S) {
    if (!h || m < 1 || (dtype != SBS_F64 && dtype != SBS_F32) || !form || !lb || !vec || !S)
        return SBS_ERR_INVALID_ARG;
    const int t = dtype == SBS_F64 ? 0 : 1;
    SepChoice sc;
    PartChoice pc;
    const int pick = pick_partition(h, t, m, rhs, true, &sc, &pc);
    if (pick == 1) {
        *form = 1;
        *lb = h->sep[sc.plan].lb;
        *vec = sc.vec;
        *S = sc.S;
    } else if (pick == 2) {
        *form = 0;
        *lb = h->part[pc.plan].lb;
        *vec = 1;
        *S = pc.S;
    } else {
        *form = *lb = *vec = *S = 0;
        return SBS_ERR_NOT_FOUND;
    }
    return SBS_OK;
}

sbs_status sbs_auto_variant(sbs_handle h, int64_t m, int32_t dtype, int32_t *variant) {
    if (!h || !variant || m < 1 || (dtype != SBS_F64 && dtype != SBS_F32)) return SBS_ERR_INVALID_ARG;
    const int t = dtype == SBS_F64 ? 0 : 1;
    PartChoice pc;
    SepChoice sc;
    // (shapes for right-hand sides aligned to 16 bytes)
    *variant = pick_partition(h, t, m, nullptr, true, &sc, &pc) ? SBS_VARIANT_PARTITION : choose_variant(h, t);
    return SBS_OK;
}

sbs_status sbs_solve_batch(sbs_handle h, void *rhs, int64_t m, int32_t dtype, void *stream) {
    return sbs_solve_batch_variant(h, rhs, m, dtype, SBS_VARIANT_AUTO, stream);
}

size_t sbs_refined_workspace_bytes(sbs_handle h, int64_t m) {
    if (!h || m < 0) return 0;
    // One FP32 residual / correction array of n*m, rounded to 256 bytes.
    return ((size_t)h->n * (size_t)m * sizeof(float) + 255) / 256 * 256;
}

sbs_status sbs_solve_batch_refined(sbs_handle h, const float *b, double *x, int64_t m, int32_t sweeps, void *work,
                                   size_t work_bytes, void *stream) {
    const sbs_status st = refined_check(h, b, x, m, sweeps);
    if (st != SBS_OK || m == 0) return st;
    if (!work || work_bytes < sbs_refined_workspace_bytes(h, m) || !aligned(work, 8)) return SBS_ERR_INVALID_ARG;
    return refined_run(h, b, x, m, sweeps, static_cast<float *>(work), static_cast<hipStream_t>(stream));
}

sbs_status sbs_cn_step(sbs_handle h, void *c, int64_t m, int32_t dtype, int32_t steps, void *stream) {
    if (!h || m < 0 || steps < 0 || (dtype != SBS_F64 && dtype != SBS_F32)) return SBS_ERR_INVALID_ARG;
    if (m == 0 || steps == 0) return SBS_OK;
    if (!c || !aligned(c, dtype == SBS_F64 ? 8 : 4)) return SBS_ERR_INVALID_ARG;
    if (m > (int64_t)0x7fffffff * kWave) return SBS_ERR_INVALID_ARG;
    const int t = dtype == SBS_F64 ? 0 : 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // pentadiagonal, constant bands and a separator shape that fills every CU
    // with whole row runs: the separator kernel's step (coefficients by
    // value).  Hyperdiffusion n = 1024, m = 65536: 234.4 us against 246.2 us
    // in the pair form; for tridiagonal matrices the pair form's step is the
    // faster (periodic diffusion, same size: 221.6 us against 233.5 us).
    if (h->constant_bands && h->kind == SBS_PENTA) {
        SepChoice sc;
        if (choose_sep(h, t, m, c, &sc, true) && sep_fills(h, t, m, sc)) {
            for (int k = 0; k < steps; ++k)
                if (launch_sep(h, sc, t, c, m, s) != hipSuccess) return SBS_ERR_DEVICE;
            return SBS_OK;
        }
    }
    PartChoice pc;
    const int cn = h->constant_bands ? 2 : 1;  // constant bands: coefficients by value, no band rows in LDS
    const bool part = choose_partition(h, t, m, &pc, cn);
    for (int k = 0; k < steps; ++k) {
        const hipError_t e = part ? launch_partition(h, pc, t, t, t, c, c, m, s, cn) : launch_cn(h, t, c, m, s);
        if (e != hipSuccess) return SBS_ERR_DEVICE;
    }
    return SBS_OK;
}

sbs_status sbs_transpose(const void *src, void *dst, int64_t rows, int64_t cols, int32_t dtype, void *stream) {
    if (rows < 0 || cols < 0 || (dtype != SBS_F64 && dtype != SBS_F32)) return SBS_ERR_INVALID_ARG;
    if (rows == 0 || cols == 0) return SBS_OK;
    if (!src || !dst) return SBS_ERR_INVALID_ARG;
    const size_t eb = dtype == SBS_F64 ? 8 : 4;
    const size_t bytes = (size_t)rows * (size_t)cols * eb;
    const char *s = static_cast<const char *>(src), *d = static_cast<const char *>(dst);
    if (s < d + bytes && d < s + bytes) return SBS_ERR_INVALID_ARG;
    if (!aligned(src, eb) || !aligned(dst, eb)) return SBS_ERR_INVALID_ARG;
    hipError_t e = launch_transpose(src, dst, rows, cols, (int)eb, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBS_OK : SBS_ERR_DEVICE;
}

sbs_status sbs_adi_step(sbs_handle hy, sbs_handle hx, double *grid, double *work, int64_t ny, int64_t nx,
                        void *stream) {
    if (!hy || !hx || ny < 1 || nx < 1 || hy->n != ny || hx->n != nx) return SBS_ERR_INVALID_ARG;
    if (!grid || !work) return SBS_ERR_INVALID_ARG;
    sbs_status st = sbs_solve_batch(hy, grid, nx, SBS_F64, stream);          // along y
    if (st != SBS_OK) return st;
    // Along x the systems are the grid's rows.  With a partition plan they
    // are solved where they are (each lane reads its block of a row as one
    // contiguous run); otherwise through the interleaved layout of the
    // transpose.
    PartChoice pc;
    if (choose_partition(hx, 0, ny, &pc, false, true))
        return launch_partition_rows(hx, pc, grid, ny, static_cast<hipStream_t>(stream)) == hipSuccess
                   ? SBS_OK
                   : SBS_ERR_DEVICE;
    st = sbs_transpose(grid, work, ny, nx, SBS_F64, stream);                   // (ny, nx) -> (nx, ny)
    if (st == SBS_OK) st = sbs_solve_batch(hx, work, ny, SBS_F64, stream);      // along x
    if (st == SBS_OK) st = sbs_transpose(work, grid, nx, ny, SBS_F64, stream);  // back
    return st;
}

}  // extern "C"
