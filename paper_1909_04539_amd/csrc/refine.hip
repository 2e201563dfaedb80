// Mixed-precision solve on the separator partition, one wave per block.
//
// A workgroup holds 64 systems (one per lane) x P blocks of LB rows (one
// wave per block).  Every lane of a wave works on the same rows of the same
// block, so every coefficient it reads -- the FP32 block factor, the spikes,
// the separator rows, the rows of S^{-1} and the FP64 band rows of the
// residual -- is wave-uniform and comes through scalar loads (from a copy
// of the plan laid out pass by pass, so that a run of rows is a few wide
// loads); LDS holds only
// per-lane data (the group's FP32 right-hand sides), the separator
// right-hand sides and the block edges of x exchanged for the residual.
//
// Per group of 64 systems, with b the stored FP32 right-hand sides:
//   x = fl64(solve32(b));
//   repeated `sweeps` times:  r = fl32(b - A x)  (FP64 arithmetic, original
//                             bands),  x += fl64(solve32(r));
// where solve32 is the separator-partitioned solve in FP32: the block sweeps
// (Sections 3.1 / 4.1 recurrences with the block's interior factor), the
// separator right-hand sides, the separators z = S^{-1} yhat (per-lane dot
// products, S^{-1} from scalar loads) and the interior correction
// x_I = g - V z_own - W z_prev.  b is read from HBM once (4 bytes per
// unknown) and x written once (8 bytes).
#include <algorithm>

#include "internal.h"

namespace sbs {
namespace {

template <int KIND>
struct R32;
template <>
struct R32<SBS_TRI> {
    using type = TriRow<float>;
};
template <>
struct R32<SBS_PENTA> {
    using type = PentaRow<float>;
};

struct RefArgs {
    int fac_bytes, spk_bytes, scf_bytes, sinv_bytes;
    int rec_fwd, rec_bwd, rec_spk, rec_band, rec_sinv, ldsinv;  // the kernel's copy of the plan
    int n, P, Nr, ngroups, sweeps;
    int64_t m;
};

// Stride (in floats) between the systems' columns of the separator buffers:
// odd, so that the 64 lanes' accesses fall in distinct banks, and above Nr
// rounded up to 8 (the separators are read 8 at a time).
__host__ __device__ __forceinline__ int refw_ldr(int Nr) { return (Nr + 7) / 8 * 8 + 1; }

// LDS: b [P*LB][64] FP32, edges [P][2H][64] FP64, yhat in two parts
// [2][64][ldr] FP32.
__host__ __device__ __forceinline__ size_t refw_lds(int KIND, int LB, int P, int Nr) {
    const int H = KIND / 2;
    return (size_t)P * LB * 64 * 4 + (size_t)P * 2 * H * 64 * 8 + (size_t)2 * 64 * refw_ldr(Nr) * 4;
}

// Compiler-only fence (emits nothing): the value is computed here.
__device__ __forceinline__ void fence(float &v) { asm volatile("" : "+v"(v) : : "memory"); }

// Pointers with their address space spelled out: the asm statements below
// hide where a pointer came from, and a pointer of unknown space is read and
// written through flat (vector) instructions.  The plan is read through the
// constant space (read-only for the kernel's life: uniform reads become
// scalar loads), the right-hand sides and solutions through the global one.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

// The next row's address, stepped one add at a time and made opaque, so
// that the addresses of all rows are not formed up front and kept live.
template <typename P>
__device__ __forceinline__ P step(P p, int64_t m) {
    p += m;
    asm volatile("" : "+v"(p));
    return p;
}

// A wave-uniform pointer made opaque to the compiler here: the scalar loads
// through it are issued at this point.  The plan is read-only, so without it
// the compiler hoists every row's coefficients to the start of the kernel
// (out of the group loop), runs out of scalar registers, and then waits on
// one scalar load per row.
// `after`: a value the loads must wait for (without it the compiler may move
// every batch's pointer, and so its loads, to the start).
template <typename P>
__device__ __forceinline__ cptr<P> here(cptr<P> p, float after) {
    asm volatile("" : "+s"(p) : "v"(after));
    return p;
}

// The block's forward and backward sweeps in FP32 (Sections 3.1 / 4.1
// recurrences with the block's interior factor).  Coefficients come from the
// plan's contiguous per-pass arrays in batches of G rows through wide scalar
// loads, the next batch in flight while the current one is used.
template <int KIND, int LB>
__device__ __forceinline__ void sweeps32(cptr<float> fwd, cptr<float> bwd, float (&w)[LB]) {
    constexpr int F = KIND == SBS_TRI ? 2 : 3, Bk = KIND == SBS_TRI ? 1 : 2;
    constexpr int G = 8, NG = LB / G;
    float c[2][G * F];
    auto getf = [&](int k, float(&d)[G * F], float after) {
        cptr<float> f = here(fwd, after) + k * G * F;
#pragma unroll
        for (int i = 0; i < G * F; ++i) d[i] = f[i];
    };
    float cb[2][G * Bk];
    auto getb = [&](int k, float(&d)[G * Bk], float after) {
        cptr<float> f = here(bwd, after) + k * G * Bk;
#pragma unroll
        for (int i = 0; i < G * Bk; ++i) d[i] = f[i];
    };
    getf(0, c[0], w[0]);
    if constexpr (KIND == SBS_TRI) {
        float y = 0.0f;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            if (k + 1 < NG) getf(k + 1, c[(k + 1) & 1], y);
#pragma unroll
            for (int u = 0; u < G; ++u) {  // y_i = d_i / den_i - (a_i / den_i) y_{i-1}
                const int t = k * G + u;
                y = w[t] = fmaf(-c[k & 1][2 * u], y, w[t] * c[k & 1][2 * u + 1]);
            }
        }
        getb(NG - 1, cb[(NG - 1) & 1], y);
        float x1 = 0.0f;
#pragma unroll
        for (int k = NG - 1; k >= 0; --k) {
            if (k > 0) getb(k - 1, cb[(k - 1) & 1], x1);
#pragma unroll
            for (int u = G - 1; u >= 0; --u) {  // x_i = y_i - chat_i x_{i+1}
                const int t = k * G + u;
                x1 = w[t] = fmaf(-cb[k & 1][u], x1, w[t]);
            }
        }
    } else {
        float g1 = 0.0f, g2 = 0.0f;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            if (k + 1 < NG) getf(k + 1, c[(k + 1) & 1], g1);
#pragma unroll
            for (int u = 0; u < G; ++u) {  // g_i = (f_i - eps_i g_{i-2} - beta_i g_{i-1}) / alpha_i
                const int t = k * G + u;
                const float *e = c[k & 1] + 3 * u;
                const float gg = fmaf(-e[1], g1, fmaf(-e[0], g2, w[t] * e[2]));
                g2 = g1;
                g1 = w[t] = gg;
            }
        }
        getb(NG - 1, cb[(NG - 1) & 1], g1);
        float x1 = 0.0f, x2 = 0.0f;
#pragma unroll
        for (int k = NG - 1; k >= 0; --k) {
            if (k > 0) getb(k - 1, cb[(k - 1) & 1], x1);
#pragma unroll
            for (int u = G - 1; u >= 0; --u) {  // x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2}
                const int t = k * G + u;
                const float xx = fmaf(-cb[k & 1][2 * u], x1, fmaf(-cb[k & 1][2 * u + 1], x2, w[t]));
                x2 = x1;
                x1 = w[t] = xx;
            }
        }
    }
}

template <int KIND, int LB, int MAXT>
__global__ __launch_bounds__(MAXT) void k_refine_wave(const unsigned char *__restrict__ blob, RefArgs a,
                                                      const unsigned char *__restrict__ rec,
                                                      const float *__restrict__ b32, double *__restrict__ x64) {
    constexpr int H = KIND / 2, NB = 2 * H + 1, NI = LB - H;
    constexpr int F = KIND == SBS_TRI ? 2 : 3, Bk = KIND == SBS_TRI ? 1 : 2;
    extern __shared__ __align__(16) unsigned char lds[];
    const int P = a.P, Nr = a.Nr, n = a.n, ldr = refw_ldr(Nr);
    const int64_t m = a.m;
    const float *__restrict__ scf = reinterpret_cast<const float *>(blob + a.fac_bytes + a.spk_bytes);
    const int *__restrict__ map =
        reinterpret_cast<const int *>(blob + a.fac_bytes + a.spk_bytes + a.scf_bytes + a.sinv_bytes);

    const int lane = threadIdx.x % kWave;
    const int p = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // the wave's block
    const int r0 = p * LB;
    const bool has_sep = p < P - 1, has_prev = p > 0;
    const bool full = r0 + LB <= n;  // no rows of the block past the end
    const int pp = has_prev ? p - 1 : p;
    const int q = map[p], qp = map[pp];
    const cptr<float> fwd = (cptr<float>)(reinterpret_cast<const float *>(rec + a.rec_fwd) + q * LB * F);
    const cptr<float> bwd = (cptr<float>)(reinterpret_cast<const float *>(rec + a.rec_bwd) + q * LB * Bk);
    const cptr<float> sk = (cptr<float>)(reinterpret_cast<const float *>(rec + a.rec_spk) + q * LB * 2 * H);
    // rows of S^{-1} of the own and the previous separator (a block without
    // one reads the other's and discards the result)
    const int lsv = a.ldsinv;
    const float *psinv = reinterpret_cast<const float *>(rec + a.rec_sinv);
    const cptr<float> rr = (cptr<float>)(psinv + (size_t)H * (has_sep ? p : pp) * lsv);
    const cptr<float> rl = (cptr<float>)(psinv + (size_t)H * (has_prev ? pp : p) * lsv);
    const cptr<double> br = (cptr<double>)(reinterpret_cast<const double *>(rec + a.rec_band) + (size_t)r0 * NB);

    float *lb32 = reinterpret_cast<float *>(lds) + (size_t)r0 * kWave + lane;  // [t * 64]
    double *ledge = reinterpret_cast<double *>(lds + (size_t)P * LB * kWave * 4);
    float *lredl = reinterpret_cast<float *>(lds + (size_t)P * LB * kWave * 4 + (size_t)P * 2 * H * kWave * 8);
    float *lredr = lredl + kWave * ldr;
    float *myl = lredl + lane * ldr, *myr = lredr + lane * ldr;

    // the separator rows' couplings to interior rows: the own separator's to
    // this block's last rows, the previous separator's to this block's first
    float cl[H][H], cr[H][H];
#pragma unroll
    for (int c = 0; c < H; ++c)
#pragma unroll
        for (int d = 0; d < H; ++d) {
            cl[c][d] = (c + d < H) ? scf[(q * H + c) * NB + d] : 0.0f;
            cr[c][d] = (2 * H - c + d < NB) ? scf[(qp * H + c) * NB + 2 * H - c + d] : 0.0f;
        }

    // solve32 of w in place; `fresh`: the separator buffers may still be read
    // by the previous group's waves, so wait for them first
    auto solve32 = [&](float(&w)[LB], bool fresh) {
        sweeps32<KIND, LB>(fwd, bwd, w);
        if (fresh) __syncthreads();
        if (has_prev) {
#pragma unroll
            for (int c = 0; c < H; ++c) {
                float yh = 0.0f;
#pragma unroll
                for (int e = 0; e + 2 * H - c < NB; ++e) yh = fmaf(-cr[c][e], w[e], yh);
                myr[H * pp + c] = yh;
            }
        }
        if (has_sep) {
#pragma unroll
            for (int c = 0; c < H; ++c) {
                float yh = w[NI + c];
#pragma unroll
                for (int d = 0; d + c < H; ++d) yh = fmaf(-cl[c][d], w[NI + c + d - H], yh);
                myl[H * p + c] = yh;
            }
        }
        __syncthreads();
        float zr[H], zl[H];
#pragma unroll
        for (int c = 0; c < H; ++c) zr[c] = zl[c] = 0.0f;
        // separators: KB separator unknowns at a time, the LDS reads of yhat
        // waited for before the scalar loads of the S^{-1} rows are issued
        // (scalar loads return out of order: any wait for one waits for all)
        constexpr int KB = 8;
        for (int k0 = 0; k0 < Nr; k0 += KB) {
            float y[KB];
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                // inside the lane's column (ldr > Nr rounded up to KB)
                const float v = myl[k0 + u] + myr[k0 + u];
                y[u] = k0 + u < Nr ? v : 0.0f;
            }
            fence(y[KB - 1]);
            // (rows padded with zeros to a multiple of KB)
            const cptr<float> a = here(rr, y[KB - 1]) + k0, b = here(rl, y[KB - 1]) + k0;
#pragma unroll
            for (int u = 0; u < KB; ++u)
#pragma unroll
                for (int c = 0; c < H; ++c) {
                    zr[c] = fmaf(a[c * lsv + u], y[u], zr[c]);
                    zl[c] = fmaf(b[c * lsv + u], y[u], zl[c]);
                }
        }
#pragma unroll
        for (int c = 0; c < H; ++c) {
            zr[c] = has_sep ? zr[c] : 0.0f;
            zl[c] = has_prev ? zl[c] : 0.0f;
        }
        // correction, the spikes of GS rows per scalar batch
        constexpr int GS = KIND == SBS_TRI ? 8 : 4;
        float sb[2][GS][2 * H];
        auto spikes = [&](int k, float(&d)[GS][2 * H], float after) {
            cptr<float> f = here(sk, after) + k * GS * 2 * H;
#pragma unroll
            for (int u = 0; u < GS; ++u)
#pragma unroll
                for (int e = 0; e < 2 * H; ++e) d[u][e] = f[u * 2 * H + e];
        };
        spikes(0, sb[0], zr[0] + zl[0]);
#pragma unroll
        for (int k = 0; k < LB / GS; ++k) {
            if (k + 1 < LB / GS) spikes(k + 1, sb[(k + 1) & 1], k > 0 ? w[k * GS - 1] : zr[0]);
#pragma unroll
            for (int u = 0; u < GS; ++u) {
                const int t = k * GS + u;
                float v = w[t];
#pragma unroll
                for (int c = 0; c < H; ++c) {
                    v = fmaf(-sb[k & 1][u][c], zr[c], v);
                    v = fmaf(-sb[k & 1][u][H + c], zl[c], v);
                }
                if (t >= NI && has_sep) v = zr[t >= NI ? t - NI : 0];
                w[t] = v;
            }
        }
    };

    float w[LB];
    auto load_b = [&](int g) {
        const int64_t j = std::min((int64_t)g * kWave + lane, m - 1);
        gptr<const float> src = (gptr<const float>)(b32 + (int64_t)r0 * m + j);
        if (full) {
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                w[t] = *src;
                src = step(src, m);
            }
        } else {
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                w[t] = r0 + t < n ? *src : 0.0f;
                src = step(src, m);
            }
        }
    };
    int g = blockIdx.x;
    if (g < a.ngroups) load_b(g);
    for (; g < a.ngroups; g += gridDim.x) {
#pragma unroll
        for (int t = 0; t < LB; ++t) lb32[t * kWave] = w[t];
        solve32(w, true);
        double x[LB];
#pragma unroll
        for (int t = 0; t < LB; ++t) x[t] = (double)w[t];
        for (int k = 0; k < a.sweeps; ++k) {
            // the block's first and last H values of x, for the neighbours' residuals
#pragma unroll
            for (int c = 0; c < H; ++c) {
                ledge[(p * 2 * H + c) * kWave + lane] = x[c];
                ledge[(p * 2 * H + H + c) * kWave + lane] = x[LB - H + c];
            }
            __syncthreads();
            double lo[H], hi[H];  // x of rows r0 - H .. r0 - 1 and r0 + LB .. r0 + LB + H - 1
#pragma unroll
            for (int c = 0; c < H; ++c) {
                lo[c] = has_prev ? ledge[((p - 1) * 2 * H + H + c) * kWave + lane] : 0.0;
                hi[c] = has_sep ? ledge[((p + 1) * 2 * H + c) * kWave + lane] : 0.0;
            }
            // r = fl32(b - A x), FP64, the row's coefficients summed left to
            // right; b from LDS into w first, then the band rows GB at a time
#pragma unroll
            for (int t = 0; t < LB; ++t) w[t] = lb32[t * kWave];
            fence(w[LB - 1]);
            constexpr int GB = KIND == SBS_TRI ? 4 : 2;
            double bb[2][GB][NB];
            auto brows = [&](int k, double(&d)[GB][NB], float after) {
                cptr<double> f = here(br, after) + k * GB * NB;
#pragma unroll
                for (int u = 0; u < GB; ++u)
#pragma unroll
                    for (int e = 0; e < NB; ++e) d[u][e] = f[u * NB + e];
            };
            brows(0, bb[0], w[LB - 1]);
#pragma unroll
            for (int k = 0; k < LB / GB; ++k) {
                if (k + 1 < LB / GB) brows(k + 1, bb[(k + 1) & 1], k > 0 ? w[k * GB - 1] : w[LB - 1]);
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    const int t = k * GB + u;
                    double ax = 0.0;
#pragma unroll
                    for (int e = 0; e < NB; ++e) {
                        const int i = t - H + e;
                        const double xv = i < 0 ? lo[i + H] : (i >= LB ? hi[i - LB] : x[i]);
                        ax = e == 0 ? bb[k & 1][u][0] * xv : fma(bb[k & 1][u][e], xv, ax);
                    }
                    w[t] = (float)((double)w[t] - ax);
                }
            }
            solve32(w, false);
#pragma unroll
            for (int t = 0; t < LB; ++t) x[t] += (double)w[t];
        }
        const int64_t j = std::min((int64_t)g * kWave + lane, m - 1);
        gptr<double> dst = (gptr<double>)(x64 + (int64_t)r0 * m + j);
        if (full) {
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                __builtin_nontemporal_store(x[t], dst);
                dst = step(dst, m);
            }
        } else {
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                if (r0 + t < n) __builtin_nontemporal_store(x[t], dst);
                dst = step(dst, m);
            }
        }
        if (g + (int)gridDim.x < a.ngroups) load_b(g + gridDim.x);
    }
}

template <int KIND, int LB>
constexpr int refw_maxt() {
    // x (FP64) and the work copy (FP32) of LB rows stay in registers
    return LB <= 32 ? 1024 : 512;
}

template <int KIND, int LB>
hipError_t refw_kernel() {
    auto kern = k_refine_wave<KIND, LB, refw_maxt<KIND, LB>()>;
    // once per instantiation (thread-safe static initialisation)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kMaxPartLdsBytes);
    return attr;
}

template <int KIND, int LB>
hipError_t go_refw(const sbs_lhs *h, const RefwChoice &c, const float *b, double *x, int64_t m, int sweeps,
                   hipStream_t s) {
    const SepPlan &sp = h->sep[c.plan];
    if (hipError_t e = refw_kernel<KIND, LB>(); e != hipSuccess) return e;
    RefArgs a;
    a.fac_bytes = (int)sp.fac_bytes32;
    a.spk_bytes = (int)sp.spk_bytes32;
    a.scf_bytes = (int)sp.scf_bytes32;
    a.sinv_bytes = (int)sp.sinv_bytes32;
    a.rec_fwd = (int)sp.refine.fwd;
    a.rec_bwd = (int)sp.refine.bwd;
    a.rec_spk = (int)sp.refine.spk;
    a.rec_band = (int)sp.refine.band;
    a.rec_sinv = (int)sp.refine.sinv;
    a.ldsinv = sp.refine.ldsinv;
    a.n = (int)h->n;
    a.P = sp.P;
    a.Nr = sp.Nr;
    a.ngroups = (int)((m + kWave - 1) / kWave);
    a.sweeps = sweeps;
    a.m = m;
    const int cus = device_cus(h->device);
    const int grid = std::min(a.ngroups, cus);
    hipLaunchKernelGGL((k_refine_wave<KIND, LB, refw_maxt<KIND, LB>()>), dim3(grid), dim3(sp.P * kWave), c.lds, s,
                       static_cast<const unsigned char *>(sp.blob32), a,
                       static_cast<const unsigned char *>(sp.refine.base), b, x);
    return hipGetLastError();
}

}  // namespace

// The one-wave-per-block mixed-precision kernel: a separator plan of a
// non-periodic matrix with at most one wave per block within the thread
// limit, and the group's right-hand sides, the edge exchange and the
// separator buffers within the LDS.  The longest block that fits is taken
// first among 32 and 64 rows (16-row blocks: too many waves per row).
bool choose_refine_wave(const sbs_lhs *h, int64_t m, RefwChoice *out) {
    if (m < 1 || (h->kind != SBS_TRI && h->kind != SBS_PENTA)) return false;
    for (int q : {1, 2}) {
        const SepPlan &sp = h->sep[q];
        if (!sp.ok || sp.periodic || !sp.refine.base) continue;
        const int maxt = sp.lb <= 32 ? 1024 : 512;
        if (sp.P * kWave > maxt) continue;
        const size_t lds = refw_lds(h->kind, sp.lb, sp.P, sp.Nr);
        if (lds > kMaxPartLdsBytes) continue;
        out->plan = q;
        out->lds = lds;
        return true;
    }
    return false;
}

hipError_t launch_refine_wave(const sbs_lhs *h, const RefwChoice &c, const float *b, double *x, int64_t m,
                              int sweeps, hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    const int lb = h->sep[c.plan].lb;
    if (h->kind == SBS_TRI)
        return lb == 32 ? go_refw<SBS_TRI, 32>(h, c, b, x, m, sweeps, stream)
                        : go_refw<SBS_TRI, 64>(h, c, b, x, m, sweeps, stream);
    return lb == 32 ? go_refw<SBS_PENTA, 32>(h, c, b, x, m, sweeps, stream)
                    : go_refw<SBS_PENTA, 64>(h, c, b, x, m, sweeps, stream);
}

}  // namespace sbs
