// HIP kernels for gfx950: the per-system forward / backward sweeps (resident,
// chunked, stream; plain, periodic and Crank-Nicolson forms), the partitioned
// solve with several lanes per system (plain, Crank-Nicolson, row layout and
// the fused mixed-precision form), the residual and update passes of the
// multi-pass refinement, the serving tile kernel and the tiled transpose.
//
// Execution model of the sweeps (Section 2 of the paper, re-done for CDNA4):
// one lane of a 64-wide wavefront owns one system, and each workgroup is one
// wavefront.  Row i of the interleaved right-hand sides is contiguous across
// the wave's 64 systems, so each row is one coalesced 512-byte (FP64) access;
// the shared factor row i is the same for every lane and is staged in LDS and
// broadcast.  The partitioned kernels give each system P lanes (one block of
// rows each) in workgroups of S systems x P blocks.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace sbs {
namespace {

enum { MODE_RESIDENT = 1, MODE_CHUNKED = 2, MODE_STREAM = 3 };

// ---------------------------------------------------------------------------
// The two recurrences.  Each forward step carries the previous results of
// the system (one for tri, two for penta); each backward step carries the
// next solution values.

template <int KIND, typename T>
struct Rec;

template <typename T>
struct Rec<SBS_TRI, T> {
    using Row = TriRow<T>;
    static constexpr int S = 1;  // values a checkpoint holds
    struct Fwd {
        T y1 = T(0);
    };
    struct Bwd {
        T x1 = T(0);
    };
    struct FC {  // forward coefficients of a row
        T a_s, inv;
    };
    struct BC {  // backward coefficients of a row
        T chat;
    };
    static __device__ __forceinline__ FC fc(const Row *f, int i) { return {f[i].a_s, f[i].inv}; }
    static __device__ __forceinline__ BC bc(const Row *f, int i) { return {f[i].chat}; }
    // y_i = d_i / den_i - (a_i / den_i) y_{i-1}          (Section 3.1, forward)
    static __device__ __forceinline__ T fwd(const FC &c, T d, Fwd &s) {
        const T y = fma(-c.a_s, s.y1, d * c.inv);
        s.y1 = y;
        return y;
    }
    // the same step when a chunk is recomputed from its checkpoint
    static __device__ __forceinline__ T refwd(const FC &c, T d, Fwd &s) { return fwd(c, d, s); }
    // x_i = y_i - chat_i x_{i+1}                          (Section 3.1, backward)
    static __device__ __forceinline__ T bwd(const BC &c, T y, Bwd &s) {
        const T x = fma(-c.chat, s.x1, y);
        s.x1 = x;
        return x;
    }
    static __device__ __forceinline__ void put(const Fwd &s, T *p) { p[0] = s.y1; }
    static __device__ __forceinline__ void get(Fwd &s, const T *p) { s.y1 = p[0]; }
    // what the backward sweep takes over from the finished forward sweep
    static __device__ __forceinline__ void link(const Fwd &, Bwd &) {}
};

template <typename T>
struct Rec<SBS_PENTA, T> {
    using Row = PentaRow<T>;
    static constexpr int S = 2;
    struct Fwd {
        T g2 = T(0), g1 = T(0);
    };
    struct Bwd {
        T x1 = T(0), x2 = T(0);
    };
    struct FC {
        T eps_s, beta_s, inv;
    };
    struct BC {
        T gamma, delta;
    };
    static __device__ __forceinline__ FC fc(const Row *f, int i) { return {f[i].eps_s, f[i].beta_s, f[i].inv}; }
    static __device__ __forceinline__ BC bc(const Row *f, int i) { return {f[i].gamma, f[i].delta}; }
    // g_i = (f_i - eps_i g_{i-2} - beta_i g_{i-1}) / alpha_i   (Section 4.1, L g = f)
    static __device__ __forceinline__ T fwd(const FC &c, T v, Fwd &s) {
        const T g = fma(-c.beta_s, s.g1, fma(-c.eps_s, s.g2, v * c.inv));
        s.g2 = s.g1;
        s.g1 = g;
        return g;
    }
    static __device__ __forceinline__ T refwd(const FC &c, T v, Fwd &s) { return fwd(c, v, s); }
    // x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2}            (Section 4.1, R x = g)
    static __device__ __forceinline__ T bwd(const BC &c, T g, Bwd &s) {
        const T x = fma(-c.gamma, s.x1, fma(-c.delta, s.x2, g));
        s.x2 = s.x1;
        s.x1 = x;
        return x;
    }
    static __device__ __forceinline__ void put(const Fwd &s, T *p) {
        p[0] = s.g2;
        p[kWave] = s.g1;
    }
    static __device__ __forceinline__ void get(Fwd &s, const T *p) {
        s.g2 = p[0];
        s.g1 = p[kWave];
    }
    static __device__ __forceinline__ void link(const Fwd &, Bwd &) {}
};

// Periodic tridiagonal (Section 3.3) through A = A' + u v^T: the sweeps of
// A' (same steps as Rec<SBS_TRI>) plus, in the forward sweep, the running dot
// product acc = sum wt_i d_i, which at the end equals (v.y) / (1 + v.z) for
// y = A'^{-1} d.  The backward sweep carries y and stores x_i = y_i - acc z_i.
template <typename T>
struct Rec<SBS_TRI_PERIODIC, T> {
    using Row = PeriodicRow<T>;
    static constexpr int S = 1;
    struct Fwd {
        T y1 = T(0), acc = T(0);
    };
    struct Bwd {
        T x1 = T(0);  // carried y_{i+1} (of A'^{-1} d, before the correction)
        T s = T(0);
    };
    struct FC {
        T a_s, inv, wt;
    };
    struct BC {
        T chat, z;
    };
    static __device__ __forceinline__ FC fc(const Row *f, int i) { return {f[i].a_s, f[i].inv, f[i].wt}; }
    static __device__ __forceinline__ BC bc(const Row *f, int i) { return {f[i].chat, f[i].z}; }
    static __device__ __forceinline__ T fwd(const FC &c, T d, Fwd &s) {
        const T y = fma(-c.a_s, s.y1, d * c.inv);
        s.acc = fma(c.wt, d, s.acc);
        // Keep the dot product in row order: left free, the scheduler runs
        // the y chain of a whole chunk first and holds every d of the chunk
        // live for the deferred products (about 70 more registers).
        asm volatile("" : "+v"(s.acc));
        s.y1 = y;
        return y;
    }
    // recomputing a chunk from its checkpoint: the dot product is complete
    static __device__ __forceinline__ T refwd(const FC &c, T d, Fwd &s) {
        const T y = fma(-c.a_s, s.y1, d * c.inv);
        s.y1 = y;
        return y;
    }
    static __device__ __forceinline__ T bwd(const BC &c, T yh, Bwd &s) {
        const T y = fma(-c.chat, s.x1, yh);
        s.x1 = y;
        return fma(-c.z, s.s, y);
    }
    static __device__ __forceinline__ void put(const Fwd &s, T *p) { p[0] = s.y1; }
    static __device__ __forceinline__ void get(Fwd &s, const T *p) { s.y1 = p[0]; }
    static __device__ __forceinline__ void link(const Fwd &f, Bwd &b) { b.s = f.acc; }
};

// Addressing.  Row r of a wave's 64 columns starts at base + r * rs bytes
// (`base` is the wave's first system, uniform; rs = m * element size); a lane
// adds its own 32-bit byte offset `lo`.  Walking rows by adding rs to a
// uniform pointer keeps every address a scalar base plus a vector offset.
//
// Lanes past the last system (m not a multiple of 64) take the offset of the
// last real system: they read its column, compute bit-identical values and
// store them to the same addresses in the same instructions, which is
// harmless and avoids masking every access.
template <typename E>
__device__ __forceinline__ E ld(const char *p, uint32_t lo) {
    return *reinterpret_cast<const E *>(p + lo);
}
template <typename E>
__device__ __forceinline__ void st(char *p, uint32_t lo, E v) {
    *reinterpret_cast<E *>(p + lo) = v;
}

// Rows of a chunk are read and written with buffer instructions: a uniform
// resource at the chunk's first row, a uniform row offset and the lane's
// byte offset -- no per-lane 64-bit address arithmetic.  BIG selects one
// resource per row for batches whose chunk span exceeds 31-bit offsets.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRawBufferFlags = 0x00020000;  // raw (untyped) buffer, gfx9-family word 3

__device__ __forceinline__ Rsrc rsrc_at(const char *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, -1, kRawBufferFlags);
}
template <typename E>
__device__ __forceinline__ E bld(Rsrc r, uint32_t vo, uint32_t so) {
    if constexpr (sizeof(E) == 8)
        return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    else
        return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
// Results are written with the non-temporal policy (they are not read again
// by the kernel; on the 1024-row pentadiagonal batch the partitioned solve
// went from 272 to 247 us).  Values that are read back soon, such as the
// stream variant's forward results, use the default policy.
constexpr int kStoreNT = 2;  // cache-policy bits of a buffer store: nt

template <typename E, int POLICY = 0>
__device__ __forceinline__ void bst(E v, Rsrc r, uint32_t vo, uint32_t so) {
    if constexpr (sizeof(E) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, vo, so, POLICY);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, vo, so, POLICY);
}

// Wave-uniform copies of values that may arrive in vector registers (the
// arguments of out-of-line device functions): buffer resources must be built
// from scalar registers.
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <typename P>
__device__ __forceinline__ P *uni(P *p) {
    return reinterpret_cast<P *>(uni64(reinterpret_cast<uint64_t>(p)));
}

// Row offsets are stepped one add at a time and passed through an empty
// asm, so the compiler cannot precompute all L of them into live registers.
__device__ __forceinline__ uint32_t step_off(uint32_t so, uint32_t d) {
    so += d;
    asm volatile("" : "+s"(so));
    return so;
}

template <typename T, typename Tin, int L, bool BIG>
__device__ __forceinline__ void load_rows(T (&buf)[L], const char *base, uint32_t lo, int r0,
                                          int n, int64_t rs) {
    const char *p = base + r0 * rs;
    const Rsrc r = rsrc_at(p);
    uint32_t so = 0;
    if (r0 + L <= n) {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if constexpr (BIG)
                buf[t] = static_cast<T>(bld<Tin>(rsrc_at(p + t * rs), lo, 0));
            else
                buf[t] = static_cast<T>(bld<Tin>(r, lo, so));
            so = step_off(so, (uint32_t)rs);
        }
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (r0 + t < n) {
                if constexpr (BIG)
                    buf[t] = static_cast<T>(bld<Tin>(rsrc_at(p + t * rs), lo, 0));
                else
                    buf[t] = static_cast<T>(bld<Tin>(r, lo, so));
            } else {
                buf[t] = T(0);
            }
            so = step_off(so, (uint32_t)rs);
        }
    }
}

template <typename T, typename Tout, int L, bool BIG>
__device__ __forceinline__ void store_rows(const T (&buf)[L], char *base, uint32_t lo, int r0,
                                           int n, int64_t rs) {
    char *p = base + r0 * rs;
    const Rsrc r = rsrc_at(p);
    uint32_t so = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (r0 + t < n) {
            if constexpr (BIG)
                bst<Tout>(static_cast<Tout>(buf[t]), rsrc_at(p + t * rs), lo, 0);
            else
                bst<Tout>(static_cast<Tout>(buf[t]), r, lo, so);
        }
        so = step_off(so, (uint32_t)rs);
    }
}

// The factor coefficients of a chunk are read from LDS four rows at a time,
// one group ahead of the rows being computed; scheduling barriers keep the
// compiler from hoisting every read of the chunk to its start (which would
// hold L rows of coefficients in registers at once).
constexpr int kGroup = 4;

// Compiler-only fence: `v` must be computed here, and no memory access moves
// across (emits no instruction).
template <typename T>
__device__ __forceinline__ void pin(T &v) {
    asm volatile("" : "+v"(v) : : "memory");
}

// Backward sweep over one chunk held in registers, writing the solution.
// `fr` points at the chunk's factor rows (staged in LDS).
template <int KIND, typename T, typename Tout, int L, bool BIG>
__device__ __forceinline__ void back_chunk(const typename Rec<KIND, T>::Row *__restrict__ fr,
                                           const T (&buf)[L], typename Rec<KIND, T>::Bwd &bs,
                                           char *base, uint32_t lo, int r0, int n,
                                           int64_t rs) {
    using R = Rec<KIND, T>;
    constexpr int G = L < kGroup ? L : kGroup, NG = L / G;
    char *p = base + r0 * rs;
    const Rsrc r = rsrc_at(p);
    const bool full = r0 + L <= n;
    uint32_t so = (uint32_t)((L - 1) * rs);
    typename R::BC c[2][G];
#pragma unroll
    for (int u = 0; u < G; ++u) c[(NG - 1) & 1][u] = R::bc(fr, L - 1 - u);
    // Rows at or beyond n meet zero factor rows and a zero input, so they
    // produce exact zeros and leave the carried values at zero.
#pragma unroll
    for (int g = NG - 1; g >= 0; --g) {
        if (g > 0) {
#pragma unroll
            for (int u = 0; u < G; ++u) c[(g - 1) & 1][u] = R::bc(fr, g * G - 1 - u);
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int t = g * G + G - 1 - u;
            const T x = R::bwd(c[g & 1][u], buf[t], bs);
            if (full || r0 + t < n) {
                if constexpr (BIG)
                    bst<Tout, kStoreNT>(static_cast<Tout>(x), rsrc_at(p + t * rs), lo, 0);
                else
                    bst<Tout, kStoreNT>(static_cast<Tout>(x), r, lo, so);
            }
            so = step_off(so, (uint32_t)(-rs));
        }
        pin(bs.x1);
    }
}

template <int KIND, typename T, int L>
__device__ __forceinline__ void fwd_chunk(const typename Rec<KIND, T>::Row *__restrict__ fr,
                                          T (&buf)[L], typename Rec<KIND, T>::Fwd &st, bool again = false) {
    using R = Rec<KIND, T>;
    constexpr int G = L < kGroup ? L : kGroup, NG = L / G;
    typename R::FC c[2][G];
#pragma unroll
    for (int u = 0; u < G; ++u) c[0][u] = R::fc(fr, u);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG) {
#pragma unroll
            for (int u = 0; u < G; ++u) c[(g + 1) & 1][u] = R::fc(fr, (g + 1) * G + u);
        }
#pragma unroll
        for (int u = 0; u < G; ++u)
            buf[g * G + u] = again ? R::refwd(c[g & 1][u], buf[g * G + u], st) : R::fwd(c[g & 1][u], buf[g * G + u], st);
        pin(buf[g * G + G - 1]);
    }
}

// Backward sweep over one chunk held in registers, leaving the solution in
// `buf` (for passes that still need the chunk's values).
template <int KIND, typename T, int L>
__device__ __forceinline__ void bwd_regs(const typename Rec<KIND, T>::Row *__restrict__ fr, T (&buf)[L],
                                         typename Rec<KIND, T>::Bwd &bs) {
    using R = Rec<KIND, T>;
    constexpr int G = L < kGroup ? L : kGroup, NG = L / G;
    typename R::BC c[2][G];
#pragma unroll
    for (int u = 0; u < G; ++u) c[(NG - 1) & 1][u] = R::bc(fr, L - 1 - u);
#pragma unroll
    for (int g = NG - 1; g >= 0; --g) {
        if (g > 0) {
#pragma unroll
            for (int u = 0; u < G; ++u) c[(g - 1) & 1][u] = R::bc(fr, g * G - 1 - u);
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int t = g * G + G - 1 - u;
            buf[t] = R::bwd(c[g & 1][u], buf[t], bs);
            // in row order: a solution value off the carried chain (periodic:
            // y - s z) would otherwise be deferred with every z kept live
            asm volatile("" : "+v"(buf[t]));
        }
        pin(bs.x1);
    }
}

// A wave's share of one factor chunk (CB bytes = L rows): lane l carries
// bytes [l*PB, (l+1)*PB).  Chunks move global -> registers -> LDS, so that
// the sweeps read every factor row with a broadcast LDS read instead of a
// scalar load whose latency would stall each row.
template <int CB>
struct FacPiece {
    static constexpr int PB = CB >= 256 ? CB / kWave : 4;  // bytes per lane
    static constexpr int NL = CB / PB;                      // lanes taking part
    static constexpr int NQ = PB >= 16 ? PB / 16 : 1;       // 16-byte words per lane (or one small word)
    static_assert(PB == 4 || PB == 8 || PB == 16 || PB == 32 || PB == 64, "factor chunk size");
    // Native vector types: plain vector loads and stores (HIP's uint4 is a
    // struct whose copies become memcpy and pin the value in private memory).
    typedef unsigned int U4 __attribute__((ext_vector_type(4)));
    typedef unsigned int U2 __attribute__((ext_vector_type(2)));
    using W = typename std::conditional<PB >= 16, U4, typename std::conditional<PB == 8, U2, uint32_t>::type>::type;
};

// A factor piece lives in up to four named 16-byte registers (never an
// array, so it cannot be demoted to private memory).
template <int CB>
struct FacRegs {
    using P = FacPiece<CB>;
    typename P::W w0, w1, w2, w3;
    __device__ __forceinline__ void load(const void *rows, int lane) {
        const typename P::W *src =
            reinterpret_cast<const typename P::W *>(static_cast<const char *>(rows) + lane * P::PB);
        if (P::NL == kWave || lane < P::NL) {
            w0 = src[0];
            if constexpr (P::NQ >= 2) w1 = src[1];
            if constexpr (P::NQ >= 4) {
                w2 = src[2];
                w3 = src[3];
            }
        }
    }
    __device__ __forceinline__ void stage(unsigned char *dst, int lane) const {
        typename P::W *d = reinterpret_cast<typename P::W *>(dst + lane * P::PB);
        if (P::NL == kWave || lane < P::NL) {
            d[0] = w0;
            if constexpr (P::NQ >= 2) d[1] = w1;
            if constexpr (P::NQ >= 4) {
                d[2] = w2;
                d[3] = w3;
            }
        }
    }
};

// LDS a wave needs: checkpoints (CHUNKED) then two factor-chunk buffers.
template <int KIND, typename T, int L, int MODE>
__host__ __device__ constexpr size_t ck_bytes(int K) {
    return MODE == 2 ? ((size_t)K * Rec<KIND, T>::S * kWave * sizeof(T) + 15) / 16 * 16 : 0;
}
template <int KIND, typename T, int L, int MODE, bool CN = false>
__host__ __device__ constexpr size_t wave_lds_bytes(int K) {
    return ck_bytes<KIND, T, L, MODE>(K) + 2 * L * sizeof(typename Rec<KIND, T>::Row) +
           (CN ? 2 * L * sizeof(BandRow) : 0);
}

// ---------------------------------------------------------------------------
// Crank-Nicolson steps (Sections 3.2 and 4.2).  Both schemes solve
// A C' = (2I - A) C; since A^{-1} and 2I - A commute, C' = (2I - A) u with
// u = A^{-1} C, so the explicit half is applied to the solution as the
// backward sweep produces it, from the last row to the first, with the
// matrix's own rows: x_q = 2 u_q - sum_k A[q][q+k-H] u_{q+k-H}.  Output row q
// needs u down to row q - H, so a chunk's pass forms rows r0 + H .. r0 + L + H - 1
// (the last H of them belong to the chunk above) and the first H rows of the
// matrix are formed after the last chunk.  No extra HBM traffic.
template <typename T>
struct CnWrap {  // periodic tridiagonal: the corner terms, finished at the end
    T xlast = T(0), ulast = T(0), cl = T(0);
};

template <int H, typename T, typename Tout, int L, bool BIG, bool PERIODIC>
__device__ __forceinline__ void cn_pass(const BandRow *bhere, const BandRow *babove, const T (&u)[L], T (&up)[2 * H],
                                        char *base, uint32_t lo, int r0, int n, int64_t rs, CnWrap<T> &wrap) {
    char *p = base + r0 * rs;
    const Rsrc r = rsrc_at(p);
    uint32_t so = (uint32_t)(H * rs);
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int lq = H + t;  // output row r0 + lq
        const BandRow &b = lq < L ? bhere[lq] : babove[lq - L];
        auto uat = [&](int li) -> T { return li < L ? u[li] : up[li - L]; };
        T ax = T(b.c[0]) * uat(t);
#pragma unroll
        for (int k = 1; k <= 2 * H; ++k) ax = fma(T(b.c[k]), uat(t + k), ax);
        const T x = T(2) * uat(lq) - ax;
        const int q = r0 + lq;
        if (PERIODIC && q == n - 1) {  // its wrap term needs u_0: finished at the end
            wrap.xlast = x;
            wrap.cl = T(b.c[2]);
        } else if (q < n) {
            if constexpr (BIG)
                bst<Tout, kStoreNT>(static_cast<Tout>(x), rsrc_at(p + lq * rs), lo, 0);
            else
                bst<Tout, kStoreNT>(static_cast<Tout>(x), r, lo, so);
        }
        so = step_off(so, (uint32_t)rs);
        if (t % kGroup == kGroup - 1) pin(ax);
    }
    if (PERIODIC && r0 + L >= n && r0 < n) {
        // u_{n-1} (the wrap term of row 0) lies in this, the top, chunk
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (r0 + t == n - 1) wrap.ulast = u[t];
    }
#pragma unroll
    for (int i = 0; i < 2 * H; ++i) up[i] = u[i];
}

// Rows 0 .. H-1 once the whole column is solved (`up` holds u_0 .. u_{2H-1},
// `b0` the band rows of the first chunk); for the periodic matrix also the
// corner terms of rows 0 and n-1.
template <int H, typename T, typename Tout, bool PERIODIC>
__device__ __forceinline__ void cn_finish(const BandRow *b0, const T (&up)[2 * H], char *base, uint32_t lo, int n,
                                          int64_t rs, const CnWrap<T> &wrap) {
#pragma unroll
    for (int q = 0; q < H; ++q) {
        if (q >= n) break;
        const BandRow &b = b0[q];
        auto uat = [&](int i) -> T { return i < 0 ? (PERIODIC ? wrap.ulast : T(0)) : up[i]; };
        T ax = T(b.c[0]) * uat(q - H);
#pragma unroll
        for (int k = 1; k <= 2 * H; ++k) ax = fma(T(b.c[k]), uat(q + k - H), ax);
        const T x = T(2) * up[q] - ax;
        st<Tout>(base + q * rs, lo, static_cast<Tout>(x));
    }
    if (PERIODIC) st<Tout>(base + (int64_t)(n - 1) * rs, lo, static_cast<Tout>(fma(-wrap.cl, up[0], wrap.xlast)));
}

// ---------------------------------------------------------------------------
// One wave solves 64 systems.
//
//  RESIDENT (n <= L): the whole column stays in registers; every right-hand
//    side crosses HBM once in and once out.
//  CHUNKED: the forward sweep stores only the carried values at the start of
//    every L-row chunk (in LDS) and keeps the last chunk in registers.  The
//    backward sweep walks the chunks from last to first, re-reads a chunk's
//    right-hand side, recomputes its forward values from the checkpoint and
//    back-substitutes.  In place is safe: a chunk is read before it is
//    written and lower chunks are untouched until their turn.
//  STREAM: the forward values of every chunk but the last are written over
//    the output and read back by the backward sweep.
//
// Pipelining: while chunk k is computed, the right-hand side of chunk k+1
// and the factor rows of chunk k+2 are in flight, and the factor rows of
// chunk k+1 (which arrived during chunk k-1) are copied into the LDS buffer
// that chunk k+1 will read.  A wave thus keeps about L * 512 B (FP64) of
// loads outstanding, close to the hardware limit of 63 per wave.
// The body works on the wave's systems j0 .. j0+63 of an (n, m) array; `lds`
// is the wave's private LDS area of wave_lds_bytes(K) bytes.
//
// CN: a Crank-Nicolson step instead of a solve (in == out): the backward
// sweep leaves each chunk's solution in registers and cn_pass forms the
// output rows from it with the band rows (`bands`), staged like the factor.
template <int KIND, typename T, typename Tin, typename Tout, int L, int MODE, bool BIG = false, bool CN = false>
__device__ __forceinline__ void sweep_wave(const typename Rec<KIND, T>::Row *__restrict__ fac, int n,
                                           const Tin *in, Tout *out, int64_t m, int64_t j0,
                                           unsigned char *lds, const BandRow *__restrict__ bands = nullptr) {
    using R = Rec<KIND, T>;
    using Row = typename R::Row;
    constexpr int CB = L * (int)sizeof(Row);
    constexpr int H = KIND == SBS_PENTA ? 2 : 1;
    constexpr bool PER = KIND == SBS_TRI_PERIODIC;
    constexpr int CBB = L * (int)sizeof(BandRow);
    const int lane = threadIdx.x;
    in = uni(in);
    out = uni(out);
    m = (int64_t)uni64((uint64_t)m);
    j0 = (int64_t)uni64((uint64_t)j0);
    n = __builtin_amdgcn_readfirstlane(n);
    const int jl = (j0 + lane < m) ? lane : (int)(m - 1 - j0);
    const char *bin = reinterpret_cast<const char *>(in + j0);
    char *bout = reinterpret_cast<char *>(out + j0);
    const uint32_t lin = (uint32_t)jl * sizeof(Tin), lout = (uint32_t)jl * sizeof(Tout);
    const int64_t rsi = m * (int64_t)sizeof(Tin), rso = m * (int64_t)sizeof(Tout);
    const int K = (n + L - 1) / L;
    T *ckp = reinterpret_cast<T *>(lds) + lane;
    unsigned char *fb = lds + ck_bytes<KIND, T, L, MODE>(K);
    auto frow = [&](int k) { return reinterpret_cast<const Row *>(fb + (k & 1) * CB); };
    FacRegs<CB> fv;
    // CN only: band rows of the chunks, double-buffered after the factor's
    unsigned char *bb = fb + 2 * CB;
    auto brow = [&](int k) { return reinterpret_cast<const BandRow *>(bb + (k & 1) * CBB); };
    FacRegs<CBB> bv;
    T up[2 * H] = {};
    CnWrap<T> wrap;
    if constexpr (CN) bands = uni(bands);

    T cur[L];
    typename R::Fwd st;
    fv.load(fac, lane);                                   // factor chunk 0
    load_rows<T, Tin, L, BIG>(cur, bin, lin, 0, n, rsi);
    fv.stage(fb, lane);

    if constexpr (MODE == MODE_RESIDENT) {
        if constexpr (CN) bv.load(bands, lane);
        fwd_chunk<KIND, T, L>(frow(0), cur, st);
        typename R::Bwd bs;
        R::link(st, bs);
        if constexpr (CN) {
            bv.stage(bb, lane);
            bwd_regs<KIND, T, L>(frow(0), cur, bs);
            cn_pass<H, T, Tout, L, BIG, PER>(brow(0), brow(0), cur, up, bout, lout, 0, n, rso, wrap);
            cn_finish<H, T, Tout, PER>(brow(0), up, bout, lout, n, rso, wrap);
        } else {
            back_chunk<KIND, T, Tout, L, BIG>(frow(0), cur, bs, bout, lout, 0, n, rso);
        }
        return;
    } else {
        T nxt[L];
        if (K > 1) fv.load(fac + L, lane);                // factor chunk 1
        // Forward sweep.
        for (int k = 0; k < K; ++k) {
            if constexpr (MODE == MODE_CHUNKED) R::put(st, ckp + k * (R::S * kWave));
            const bool more = k + 1 < K;
            if (more) load_rows<T, Tin, L, BIG>(nxt, bin, lin, (k + 1) * L, n, rsi);
            fwd_chunk<KIND, T, L>(frow(k), cur, st);
            if (more) {
                if constexpr (MODE == MODE_STREAM) store_rows<T, Tout, L, BIG>(cur, bout, lout, k * L, n, rso);
                fv.stage(fb + ((k + 1) & 1) * CB, lane);  // chunk k+1's factor, loaded one chunk ago
                if (k + 2 < K) fv.load(fac + (k + 2) * L, lane);
#pragma unroll
                for (int t = 0; t < L; ++t) cur[t] = nxt[t];
            }
        }
        // Backward sweep; cur holds the forward values of the last chunk and
        // buffer (K-1)&1 its factor rows.
        typename R::Bwd bs;
        R::link(st, bs);
        if constexpr (CN) {
            bv.load(bands + (K - 1) * L, lane);
            bv.stage(bb + ((K - 1) & 1) * CBB, lane);
        }
        if (K >= 2) {
            fv.load(fac + (K - 2) * L, lane);
            if constexpr (CN) bv.load(bands + (K - 2) * L, lane);
            if constexpr (MODE == MODE_CHUNKED)
                load_rows<T, Tin, L, BIG>(nxt, bin, lin, (K - 2) * L, n, rsi);
            else
                load_rows<T, Tout, L, BIG>(nxt, bout, lout, (K - 2) * L, n, rso);
        }
        if constexpr (CN) {
            bwd_regs<KIND, T, L>(frow(K - 1), cur, bs);
            // nothing lies above the top chunk: its rows past n are not stored
            cn_pass<H, T, Tout, L, BIG, PER>(brow(K - 1), brow(K - 1), cur, up, bout, lout, (K - 1) * L, n, rso, wrap);
        } else {
            back_chunk<KIND, T, Tout, L, BIG>(frow(K - 1), cur, bs, bout, lout, (K - 1) * L, n, rso);
        }
        for (int k = K - 2; k >= 0; --k) {
            fv.stage(fb + (k & 1) * CB, lane);
            if constexpr (CN) bv.stage(bb + (k & 1) * CBB, lane);  // chunk k+2's rows are no longer needed
#pragma unroll
            for (int t = 0; t < L; ++t) cur[t] = nxt[t];
            if (k >= 1) {
                fv.load(fac + (k - 1) * L, lane);
                if constexpr (CN) bv.load(bands + (k - 1) * L, lane);
                if constexpr (MODE == MODE_CHUNKED)
                    load_rows<T, Tin, L, BIG>(nxt, bin, lin, (k - 1) * L, n, rsi);
                else
                    load_rows<T, Tout, L, BIG>(nxt, bout, lout, (k - 1) * L, n, rso);
            }
            if constexpr (MODE == MODE_CHUNKED) {
                R::get(st, ckp + k * (R::S * kWave));
                fwd_chunk<KIND, T, L>(frow(k), cur, st, true);  // recompute from the checkpoint
            }
            if constexpr (CN) {
                bwd_regs<KIND, T, L>(frow(k), cur, bs);
                cn_pass<H, T, Tout, L, BIG, PER>(brow(k), brow(k + 1), cur, up, bout, lout, k * L, n, rso, wrap);
            } else {
                back_chunk<KIND, T, Tout, L, BIG>(frow(k), cur, bs, bout, lout, k * L, n, rso);
            }
        }
        if constexpr (CN) cn_finish<H, T, Tout, PER>(brow(0), up, bout, lout, n, rso, wrap);
    }
}

template <int KIND, typename T, int L, int MODE, bool BIG>
__global__ __launch_bounds__(kWave) void k_cn(const typename Rec<KIND, T>::Row *__restrict__ fac,
                                              const BandRow *__restrict__ bands, int n, T *c, int64_t m) {
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_wave<KIND, T, T, T, L, MODE, BIG, true>(fac, n, c, c, m, (int64_t)blockIdx.x * kWave, smem, bands);
}

template <int KIND, typename T, typename Tin, typename Tout, int L, int MODE, bool BIG>
__global__ __launch_bounds__(kWave) void k_sweep(const typename Rec<KIND, T>::Row *__restrict__ fac,
                                                 int n, const Tin *in, Tout *out, int64_t m) {
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_wave<KIND, T, Tin, Tout, L, MODE, BIG>(fac, n, in, out, m, (int64_t)blockIdx.x * kWave, smem);
}

// ---------------------------------------------------------------------------
// Partitioned solve: several lanes per system.  A workgroup holds S systems
// times P blocks (lane l: block p = l / S, system s = l % S).  Every lane
// loads its block's lb rows of its system (for each block, S consecutive
// systems of a row are contiguous, so the accesses stay whole cache lines),
// solves its block with the block's own factor, publishes the top and bottom
// values, and after one barrier computes the interface unknowns it needs --
// the first h unknowns of block p+1 and the last h of block p-1 -- as dot
// products with rows of the stored inverse of the interface system; then
// x = g - V xt - W xb and one store.  Each right-hand side crosses HBM once in
// and once out.  The block factors, spikes and inverse (shared by every
// system) are copied into LDS once per persistent workgroup.

// Interface step of the partitioned solve: publishes this block's interface
// values and computes, from the stored inverse of the interface system, the
// first H unknowns of block p+1 (xt) and the last H of block p-1 (xb); the
// block's solution is then x = g - V xt - W xb.
template <int KIND, typename T, int LB>
__device__ __forceinline__ void part_interface(const T (&x)[LB], T *red, const T *rt, const T *rb, int p, int pp,
                                               bool has_next, bool has_prev, int Nr, T (&xt)[KIND / 2],
                                               T (&xb)[KIND / 2]) {
    // Pair q of the interface holds (bottom H of block q, top H of the next
    // block); block p's bottom is in pair p, its top in pair pp (the previous
    // block's pair: p - 1, or P - 1 for block 0 of a periodic matrix).
    constexpr int H = KIND / 2;
    if (has_next) {
#pragma unroll
        for (int c = 0; c < H; ++c) red[2 * H * p + c] = x[LB - H + c];
    }
    if (has_prev) {
#pragma unroll
        for (int c = 0; c < H; ++c) red[2 * H * pp + H + c] = x[c];
    }
    __syncthreads();
    // All 2H dot products in one pass over the system's interface values, so
    // each is read from LDS once (the rows of the inverse are shared by the
    // block's systems and broadcast).  Blocks at the ends use a row of the
    // other side in place of the missing one and discard it.
    const T *ra = has_next ? rt : rb, *rz = has_prev ? rb : rt;
    T at[H], az[H];
#pragma unroll
    for (int c = 0; c < H; ++c) at[c] = az[c] = T(0);
    for (int k = 0; k < Nr; ++k) {
        const T v = red[k];
#pragma unroll
        for (int c = 0; c < H; ++c) {
            at[c] = fma(ra[c * Nr + k], v, at[c]);
            az[c] = fma(rz[c * Nr + k], v, az[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < H; ++c) {
        xt[c] = has_next ? at[c] : T(0);
        xb[c] = has_prev ? az[c] : T(0);
    }
    __syncthreads();  // red is rewritten next time
}

// FP64 form of the interface step on the matrix cores.  For a group of S
// systems the interface unknowns are Z = R^{-1} Y, with Y (Nr x S) the
// published interface values (column s at red + s * ldr): a dense product
// that the waves share in 16 x 16 tiles of v_mfma_f64_16x16x4f64 (lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; item r of the result is
// D[4 r + l / 16][l % 16]).  Each operand is read from LDS once per tile
// instead of once per lane and product, which is what bounds the per-lane
// dot products.  The tiles go to zb (same layout as red), and after one
// barrier each lane takes its 2H values.  Two barriers per group, as in the
// per-lane form: red is not rewritten before every wave has passed the
// second one, nor zb before the first barrier of the next group.
template <int KIND, int LB>
__device__ __forceinline__ void part_interface_mma(const double (&x)[LB], double *red_all, double *zb,
                                                   const double *rinv, int s, int p, int pp, bool has_next,
                                                   bool has_prev, int Nr, int S, int ldr, double (&xt)[KIND / 2],
                                                   double (&xb)[KIND / 2]) {
    typedef double D4 __attribute__((ext_vector_type(4)));
    constexpr int H = KIND / 2;
    double *red = red_all + s * ldr;
    if (has_next) {
#pragma unroll
        for (int c = 0; c < H; ++c) red[2 * H * p + c] = x[LB - H + c];
    }
    if (has_prev) {
#pragma unroll
        for (int c = 0; c < H; ++c) red[2 * H * pp + H + c] = x[c];
    }
    __syncthreads();
    // whole waves only (blockDim.x a multiple of 64, so nwaves >= 1)
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
    const int mt = (Nr + 15) / 16, ntiles = mt * ((S + 15) / 16);
    const int lr = lane % 16, lk = lane / 16;
    for (int tile = wave; tile < ntiles; tile += nwaves) {
        const int i0 = (tile % mt) * 16, j0 = (tile / mt) * 16;
        const int i = i0 + lr, j = j0 + lr;
        const double *arow = rinv + (size_t)min(i, Nr - 1) * Nr;
        const double *bcol = red_all + min(j, S - 1) * ldr;
        D4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < Nr; k0 += 4) {
            const int k = k0 + lk, kc = min(k, Nr - 1);
            const bool kin = k < Nr;
            const double a = (kin && i < Nr) ? arow[kc] : 0.0;
            const double b = (kin && j < S) ? bcol[kc] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = i0 + 4 * r + lk;
            if (row < Nr && j < S) zb[j * ldr + row] = acc[r];
        }
    }
    __syncthreads();
    const double *z = zb + s * ldr;
#pragma unroll
    for (int c = 0; c < H; ++c) {
        xt[c] = has_next ? z[2 * H * p + H + c] : 0.0;
        xb[c] = has_prev ? z[2 * H * pp + c] : 0.0;
    }
}

template <int KIND, typename T>
__device__ __forceinline__ T part_correct(T v, const T *spt, const T (&xt)[KIND / 2], const T (&xb)[KIND / 2]) {
    constexpr int H = KIND / 2;
#pragma unroll
    for (int c = 0; c < H; ++c) v = fma(-spt[c], xt[c], v);
#pragma unroll
    for (int c = 0; c < H; ++c) v = fma(-spt[H + c], xb[c], v);
    return v;
}

// Bytes of a plan's block map (P ints, 16-byte aligned) at the end of its blob.
__device__ __forceinline__ int map_bytes(int P) { return (P * 4 + 15) / 16 * 16; }

// Copies a plan blob [fac | spk | rinv | map] into LDS, eight 16-byte loads
// in flight per thread: small workgroups (a few systems of a short matrix)
// would otherwise wait for one round trip to L2 per 16 bytes.
__device__ __forceinline__ void stage_blob(unsigned char *lds, const unsigned char *blob, int bytes) {
    typedef unsigned int U4 __attribute__((ext_vector_type(4)));
    constexpr int U = 8;
    const U4 *src = reinterpret_cast<const U4 *>(blob);
    U4 *dst = reinterpret_cast<U4 *>(lds);
    const int total = bytes / 16, step = blockDim.x;
    int i = threadIdx.x;
    for (; i + (U - 1) * step < total; i += U * step) {
        U4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[i + u * step];
#pragma unroll
        for (int u = 0; u < U; ++u) dst[i + u * step] = v[u];
    }
    for (; i < total; i += step) dst[i] = src[i];
}

// CN: a Crank-Nicolson step (in == out) instead of a solve: after the
// correction each lane holds its block of u = A^{-1} c, swaps its first and
// last H values with the neighbouring blocks through LDS, and writes
// 2 u - A u with the band rows (CN 1: compact, NB = 2H + 1 per row, in LDS;
// CN 2: constant bands, the NB coefficients in `coef`).
// `periodic`: block 0 and block P-1 are neighbours (one more interface pair).
// ROWS: the systems are stored one after another (system j at j*n .. j*n+n-1,
// the rows of a row-major grid) instead of interleaved; each lane then reads
// and writes its block as one contiguous run.
template <int KIND, typename T, typename Tin, typename Tout, int LB, int MAXT, int CN = 0, bool ROWS = false>
__global__ __launch_bounds__(MAXT) void k_part(const unsigned char *__restrict__ blob, int fac_bytes, int spk_bytes,
                                               int rinv_bytes, int n, int P, int Nr, int S, int ngroups, int periodic,
                                               const BandRow *__restrict__ bands, BandCoef coef, const Tin *in,
                                               Tout *out, int64_t m) {
    using R = Rec<KIND, T>;
    using Row = typename R::Row;
    constexpr int H = KIND / 2;
    constexpr int NB = 2 * H + 1;
    extern __shared__ __align__(16) unsigned char lds[];
    const int blob_bytes = fac_bytes + spk_bytes + rinv_bytes + map_bytes(P);
    stage_blob(lds, blob, blob_bytes);
    const Row *lfac = reinterpret_cast<const Row *>(lds);
    const T *lspk = reinterpret_cast<const T *>(lds + fac_bytes);
    const T *lrinv = reinterpret_cast<const T *>(lds + fac_bytes + spk_bytes);
    const int *lmap = reinterpret_cast<const int *>(lds + fac_bytes + spk_bytes + rinv_bytes);
    T *lred = reinterpret_cast<T *>(lds + blob_bytes);
    const int ldr = Nr + 1;  // odd stride: the systems' rows fall in different banks
    const int npad = P * LB;
    // interface step on the matrix cores: FP64 pentadiagonal (4 unknowns per
    // lane from 4 (P - 1) values); the tridiagonal step is half as wide and
    // a quarter of the reads, and stays per lane
    constexpr bool MMA = std::is_same<T, double>::value && KIND == SBS_PENTA;
    const int red_bytes = (S * ldr * (int)sizeof(T) + 15) / 16 * 16;
    T *lz = reinterpret_cast<T *>(lds + blob_bytes + red_bytes);  // MMA: the interface unknowns
    unsigned char *after_red = lds + blob_bytes + red_bytes * (MMA ? 2 : 1);
    double *lband = reinterpret_cast<double *>(after_red);                                  // CN 1: [npad][NB]
    T *lend = reinterpret_cast<T *>(after_red + (CN == 1 ? (npad * NB * 8 + 15) / 16 * 16 : 0));  // CN: [S][P][2H]
    if constexpr (CN == 1) {
        for (int i = threadIdx.x; i < npad; i += blockDim.x)
#pragma unroll
            for (int k = 0; k < NB; ++k) lband[i * NB + k] = i < n ? bands[i].c[k] : 0.0;
    }
    __syncthreads();

    const int l = threadIdx.x, p = l / S, s = l - p * S;
    const int r0 = p * LB;
    const int q = lmap[p];  // stored copy of this block's factor and spikes
    const Row *fr = lfac + q * LB;
    const T *sp = lspk + q * LB * 2 * H;
    T *red = lred + s * ldr;
    const bool has_next = periodic || p <= P - 2, has_prev = periodic || p >= 1;
    const int pp = p == 0 ? P - 1 : p - 1, pn = p == P - 1 ? 0 : p + 1;
    const T *rt = lrinv + (2 * H * p + H) * Nr;  // rows of the next block's first H unknowns
    const T *rb = lrinv + (2 * H * pp) * Nr;     // rows of the previous block's last H
    const int64_t rs = ROWS ? 1 : m;  // distance between consecutive unknowns of a system
    for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t j = min((int64_t)g * S + s, m - 1);
        const int64_t base = ROWS ? j * n + r0 : (int64_t)r0 * rs + j;
        const Tin *src = in + base;
        T x[LB];
        // row layout with even n: every block starts on a 16-byte boundary,
        // so pairs of values move as one 16-byte access
        constexpr bool PAIRS = ROWS && sizeof(T) == 8 && sizeof(Tin) == 8 && sizeof(Tout) == 8;
        const bool paired = PAIRS && (n % 2 == 0) && r0 + LB <= n;
        if (paired) {
            typedef double D2 __attribute__((ext_vector_type(2)));
            const D2 *s2 = reinterpret_cast<const D2 *>(src);
#pragma unroll
            for (int t = 0; t < LB / 2; ++t) {
                const D2 v = s2[t];
                x[2 * t] = static_cast<T>(v.x);
                x[2 * t + 1] = static_cast<T>(v.y);
            }
        } else if (r0 + LB <= n) {
#pragma unroll
            for (int t = 0; t < LB; ++t) x[t] = static_cast<T>(src[(int64_t)t * rs]);
        } else {
#pragma unroll
            for (int t = 0; t < LB; ++t) x[t] = (r0 + t < n) ? static_cast<T>(src[(int64_t)t * rs]) : T(0);
        }
        typename R::Fwd st;
        fwd_chunk<KIND, T, LB>(fr, x, st);
        typename R::Bwd bs;
        bwd_regs<KIND, T, LB>(fr, x, bs);
        T xt[H], xb[H];
        // the matrix cores need whole waves: workgroups of fewer than 64
        // threads (small batches) keep the per-lane dot products
        if (MMA && blockDim.x % kWave == 0) {
            if constexpr (MMA)
                part_interface_mma<KIND, LB>(x, lred, lz, lrinv, s, p, pp, has_next, has_prev, Nr, S, ldr, xt, xb);
        } else {
            part_interface<KIND, T, LB>(x, red, rt, rb, p, pp, has_next, has_prev, Nr, xt, xb);
        }
        Tout *dst = out + base;
        if constexpr (PAIRS && !CN) {
            if (paired) {
                typedef double D2 __attribute__((ext_vector_type(2)));
                D2 *d2 = reinterpret_cast<D2 *>(dst);
#pragma unroll
                for (int t = 0; t < LB / 2; ++t) {
                    D2 v;
                    v.x = static_cast<double>(part_correct<KIND, T>(x[2 * t], sp + 2 * t * 2 * H, xt, xb));
                    v.y = static_cast<double>(part_correct<KIND, T>(x[2 * t + 1], sp + (2 * t + 1) * 2 * H, xt, xb));
                    __builtin_nontemporal_store(v, &d2[t]);
                }
                continue;
            }
        }
        if constexpr (!CN) {
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                const T v = part_correct<KIND, T>(x[t], sp + t * 2 * H, xt, xb);
                if (r0 + t < n) __builtin_nontemporal_store(static_cast<Tout>(v), &dst[(int64_t)t * rs]);
            }
        } else {
            // u = the corrected solution.  Only the block's first and last H
            // values are formed before the exchange; the rest are corrected
            // on the fly in a window of 2H + 1 rows, so that each solved value
            // is dropped as soon as it is used (as in the plain store loop).
            auto corr = [&](int i) -> T { return part_correct<KIND, T>(x[i], sp + i * 2 * H, xt, xb); };
            T *e = lend + (s * P + p) * 2 * H;
#pragma unroll
            for (int c = 0; c < H; ++c) {
                e[c] = corr(c);
                e[H + c] = corr(LB - H + c);
            }
            __syncthreads();
            T lft[H], rgt[H];  // u just before and just after the block (0 past the ends)
#pragma unroll
            for (int c = 0; c < H; ++c) {
                lft[c] = has_prev ? lend[(s * P + pp) * 2 * H + H + c] : T(0);
                rgt[c] = has_next ? lend[(s * P + pn) * 2 * H + c] : T(0);
            }
            __syncthreads();  // lend is rewritten next group
            T win[NB];        // win[k] = u at row t - H + k
#pragma unroll
            for (int k = 0; k < NB - 1; ++k) win[k] = k < H ? lft[k] : corr(k - H);
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                win[NB - 1] = t + H < LB ? corr(t + H) : rgt[t + H - LB];
                // constant bands: the coefficients are kernel arguments (the
                // values they meet outside the matrix are 0 in the window)
                const double *b = CN == 2 ? coef.c : lband + (r0 + t) * NB;
                T ax = T(b[0]) * win[0];
#pragma unroll
                for (int k = 1; k < NB; ++k) ax = fma(T(b[k]), win[k], ax);
                const T v = T(2) * win[H] - ax;
                // one store pointer stepped row by row (pinned, so that the
                // addresses of all rows are not formed up front and kept live)
                if (r0 + t < n) __builtin_nontemporal_store(static_cast<Tout>(v), dst);
                dst += rs;
                asm volatile("" : "+v"(dst));
#pragma unroll
                for (int k = 0; k < NB - 1; ++k) win[k] = win[k + 1];
                if (t % kGroup == kGroup - 1) pin(ax);  // band and spike reads stay with their rows
            }
        }
    }
}

// Mixed precision on the partition, fused: each lane keeps its block of the
// FP32 right-hand side b and of the FP64 solution x in registers through the
// FP32 solve, every residual r = b - A x (FP64, original bands, neighbouring
// blocks' values exchanged through LDS), the FP32 correction solves and the
// FP64 updates; b is read once and x written once (12 bytes per unknown).
template <int KIND, int LB, int MAXT>
__global__ __launch_bounds__(MAXT) void k_part_refine(const unsigned char *__restrict__ blob, int fac_bytes,
                                                      int spk_bytes, int rinv_bytes,
                                                      const BandRow *__restrict__ bands, int n, int P, int Nr, int S,
                                                      int ngroups, int sweeps, const float *b32, double *x64,
                                                      int64_t m) {
    using R = Rec<KIND, float>;
    using Row = typename R::Row;
    constexpr int H = KIND / 2;
    extern __shared__ __align__(16) unsigned char lds[];
    const int blob_bytes = fac_bytes + spk_bytes + rinv_bytes + map_bytes(P);
    const int npad = P * LB;
    stage_blob(lds, blob, blob_bytes);
    BandRow *lband = reinterpret_cast<BandRow *>(lds + blob_bytes);
    for (int i = threadIdx.x; i < npad; i += blockDim.x) lband[i] = bands[i];
    const Row *lfac = reinterpret_cast<const Row *>(lds);
    const float *lspk = reinterpret_cast<const float *>(lds + fac_bytes);
    const float *lrinv = reinterpret_cast<const float *>(lds + fac_bytes + spk_bytes);
    const int *lmap = reinterpret_cast<const int *>(lds + fac_bytes + spk_bytes + rinv_bytes);
    unsigned char *after = lds + blob_bytes + npad * sizeof(BandRow);
    const int ldr = Nr + 1;
    float *lred = reinterpret_cast<float *>(after);
    double *lnb = reinterpret_cast<double *>(after + ((S * ldr * 4 + 15) / 16) * 16);  // [S][P][2H]
    __syncthreads();

    const int l = threadIdx.x, p = l / S, s = l - p * S;
    const int r0 = p * LB;
    const int q = lmap[p];
    const Row *fr = lfac + q * LB;
    const float *sp = lspk + q * LB * 2 * H;
    float *red = lred + s * ldr;
    const float *rt = lrinv + (2 * H * p + H) * Nr;
    const float *rb = lrinv + (2 * H * (p - 1)) * Nr;
    double *nb = lnb + (int64_t)s * P * 2 * H;
    const BandRow *br = lband + r0;
    const int64_t rs = m;
    for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t j = min((int64_t)g * S + s, m - 1);
        const float *src = b32 + (int64_t)r0 * rs + j;
        float b[LB], w[LB];
        double x[LB];
#pragma unroll
        for (int t = 0; t < LB; ++t) b[t] = (r0 + t < n) ? src[(int64_t)t * rs] : 0.0f;
#pragma unroll
        for (int t = 0; t < LB; ++t) w[t] = b[t];
        {
            typename R::Fwd st;
            fwd_chunk<KIND, float, LB>(fr, w, st);
            typename R::Bwd bs;
            bwd_regs<KIND, float, LB>(fr, w, bs);
            float xt[H], xb[H];
            part_interface<KIND, float, LB>(w, red, rt, rb, p, p - 1, p <= P - 2, p >= 1, Nr, xt, xb);
#pragma unroll
            for (int t = 0; t < LB; ++t) x[t] = (double)part_correct<KIND, float>(w[t], sp + t * 2 * H, xt, xb);
        }
        for (int k = 0; k < sweeps; ++k) {
            // neighbours: the last H values of block p-1 and the first H of block p+1
#pragma unroll
            for (int c = 0; c < H; ++c) {
                nb[p * 2 * H + c] = x[c];
                nb[p * 2 * H + H + c] = x[LB - H + c];
            }
            __syncthreads();
            double win[LB + 2 * H];
#pragma unroll
            for (int c = 0; c < H; ++c) {
                win[c] = p >= 1 ? nb[(p - 1) * 2 * H + H + c] : 0.0;
                win[LB + H + c] = p <= P - 2 ? nb[(p + 1) * 2 * H + c] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < LB; ++t) win[H + t] = x[t];
            __syncthreads();  // nb is rewritten next sweep
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                const BandRow &rw = br[t];
                double ax = rw.c[0] * win[t];
#pragma unroll
                for (int q = 1; q < 2 * H + 1; ++q) ax = fma(rw.c[q], win[t + q], ax);
                w[t] = (float)((double)b[t] - ax);
            }
            typename R::Fwd st;
            fwd_chunk<KIND, float, LB>(fr, w, st);
            typename R::Bwd bs;
            bwd_regs<KIND, float, LB>(fr, w, bs);
            float xt[H], xb[H];
            part_interface<KIND, float, LB>(w, red, rt, rb, p, p - 1, p <= P - 2, p >= 1, Nr, xt, xb);
#pragma unroll
            for (int t = 0; t < LB; ++t) x[t] += (double)part_correct<KIND, float>(w[t], sp + t * 2 * H, xt, xb);
        }
        double *dst = x64 + (int64_t)r0 * rs + j;
#pragma unroll
        for (int t = 0; t < LB; ++t)
            if (r0 + t < n) __builtin_nontemporal_store(x[t], &dst[(int64_t)t * rs]);
    }
}

// ---------------------------------------------------------------------------
// Mixed-precision passes.  Lane per system again; a wave walks its 64
// columns in chunks of RL rows, with the next chunk's loads (x, delta, b and
// the band rows, staged through LDS) in flight while the current chunk is
// computed.
//  MODE 0: r_i = fl32(b_i - (A x)_i)
//  MODE 1: x_i += delta_i for every row, then r from the updated x
//  MODE 2: x is FP32 (the first solve's result x0) and delta the first
//          correction: r from x = fl64(x0 + delta), which is not stored
//          (the same values MODE 1 would store and use)
// (A x)_i is summed left to right over the row's coefficients, in FP64.
constexpr int kResRows = 16;  // RL: rows per residual chunk
constexpr size_t kResLds = 2 * kResRows * sizeof(BandRow);  // band rows of two chunks

// One residual chunk's inputs: x and delta of rows r0 .. r0+RL+H-1 (the
// last H rows are the next chunk's first, re-read from cache: row i's
// residual needs x_{i+H}), b of rows r0 .. r0+RL-1.  Rows at or beyond n read
// as 0.
template <int H, int MODE, typename XT = double>
struct ResChunk {
    static constexpr int RL = kResRows;
    XT x[RL + H];
    float d[RL + H], b[RL];
    __device__ __forceinline__ void load(const char *px, const char *pd, const char *pb, uint32_t lx, uint32_t l4,
                                         int r0, int n, int64_t rsx, int64_t rs4) {
#pragma unroll
        for (int t = 0; t < RL + H; ++t) {
            const bool in = r0 + t < n;
            x[t] = in ? ld<XT>(px + (int64_t)(r0 + t) * rsx, lx) : XT(0);
            if constexpr (MODE >= 1) d[t] = in ? ld<float>(pd + (int64_t)(r0 + t) * rs4, l4) : 0.0f;
            if (t < RL) b[t] = in ? ld<float>(pb + (int64_t)(r0 + t) * rs4, l4) : 0.0f;
        }
    }
};

template <int KIND, int MODE, typename XT = double>
__device__ __forceinline__ void residual_wave(const BandRow *__restrict__ bands, int64_t n64,
                                              const float *__restrict__ b, XT *__restrict__ x,
                                              const float *dl, float *r, int64_t m, int64_t j0,
                                              unsigned char *lds) {
    static_assert(MODE != 1 || sizeof(XT) == 8, "MODE 1 stores x in FP64");
    static_assert(MODE != 2 || sizeof(XT) == 4, "MODE 2 reads x0 in FP32");
    // dl and r may be the same buffer: a chunk's delta values are loaded
    // before any residual of that chunk is stored, and the H rows past the
    // chunk are loaded with the next chunk, before its residuals are stored.
    constexpr int H = KIND / 2, RL = kResRows, CBB = RL * (int)sizeof(BandRow);
    const int lane = threadIdx.x;
    bands = uni(bands);
    b = uni(b);
    x = uni(x);
    dl = uni(dl);
    r = uni(r);
    m = (int64_t)uni64((uint64_t)m);
    j0 = (int64_t)uni64((uint64_t)j0);
    const int n = __builtin_amdgcn_readfirstlane((int)n64);
    const int jl = (j0 + lane < m) ? lane : (int)(m - 1 - j0);
    const uint32_t l4 = (uint32_t)jl * 4, lx = (uint32_t)jl * (uint32_t)sizeof(XT);
    const char *pb = reinterpret_cast<const char *>(b + j0);
    char *px = reinterpret_cast<char *>(x + j0);
    const char *pd = reinterpret_cast<const char *>(dl + j0);
    char *pr = reinterpret_cast<char *>(r + j0);
    const int64_t rs4 = m * 4, rsx = m * (int64_t)sizeof(XT);
    const int K = (n + RL - 1) / RL;
    auto brow = [&](int k) { return reinterpret_cast<const BandRow *>(lds + (k & 1) * CBB); };
    FacRegs<CBB> bv;  // band rows of a chunk on their way to LDS

    // x_{r0-H} .. x_{r0-1} (updated), 0 above the matrix
    double prev[H];
#pragma unroll
    for (int q = 0; q < H; ++q) prev[q] = 0.0;
    ResChunk<H, MODE, XT> cur, nxt;
    bv.load(bands, lane);
    cur.load(px, pd, pb, lx, l4, 0, n, rsx, rs4);
    bv.stage(lds, lane);
    if (K > 1) bv.load(bands + RL, lane);
    for (int k = 0; k < K; ++k) {
        const int r0 = k * RL;
        const bool more = k + 1 < K;
        if (more) nxt.load(px, pd, pb, lx, l4, r0 + RL, n, rsx, rs4);
        // the chunk's x (and the H rows after it), updated by delta
        double xs[RL + H];
#pragma unroll
        for (int t = 0; t < RL + H; ++t) {
            xs[t] = (double)cur.x[t];
            if constexpr (MODE >= 1) xs[t] += (double)cur.d[t];
        }
        if constexpr (MODE == 1) {
#pragma unroll
            for (int t = 0; t < RL; ++t)
                if (r0 + t < n) st<double>(px + (int64_t)(r0 + t) * rsx, lx, xs[t]);
        }
        const BandRow *br = brow(k);
#pragma unroll
        for (int t = 0; t < RL; ++t) {
            // window x_{i-H} .. x_{i+H} of row i = r0 + t
            auto xw = [&](int q) -> double { return t + q - H < 0 ? prev[t + q] : xs[t + q - H]; };
            double ax = br[t].c[0] * xw(0);
#pragma unroll
            for (int q = 1; q < 2 * H + 1; ++q) ax = fma(br[t].c[q], xw(q), ax);
            if (r0 + t < n) st<float>(pr + (int64_t)(r0 + t) * rs4, l4, (float)((double)cur.b[t] - ax));
            if (t % kGroup == kGroup - 1) pin(ax);
        }
#pragma unroll
        for (int q = 0; q < H; ++q) prev[q] = xs[RL - H + q];
        if (more) {
            bv.stage(lds + ((k + 1) & 1) * CBB, lane);  // chunk k+1's band rows, loaded one chunk ago
            if (k + 2 < K) bv.load(bands + (k + 2) * RL, lane);
            cur = nxt;
        }
    }
}

template <int KIND, int MODE>
__global__ __launch_bounds__(kWave) void k_residual(const BandRow *__restrict__ bands, int64_t n,
                                                    const float *__restrict__ b, double *__restrict__ x,
                                                    const float *dl, float *r, int64_t m) {
    __shared__ __align__(16) unsigned char lds[kResLds];
    residual_wave<KIND, MODE>(bands, n, b, x, dl, r, m, (int64_t)blockIdx.x * kWave, lds);
}

// x = fl64(fl64(x0 + d1) + d2) over one wave's 64 systems: the refined
// tile's result from the first solve's FP32 values and the two FP32
// corrections (the same values as x += d1, then x += d2 in FP64), U rows per
// batch with the next batch's loads in flight.
__device__ __forceinline__ void finish_wave(double *x, const float *x0, const float *d1, const float *d2,
                                            int64_t n64, int64_t m, int64_t j0) {
    constexpr int U = 8;
    const int lane = threadIdx.x;
    x = uni(x);
    x0 = uni(x0);
    d1 = uni(d1);
    d2 = uni(d2);
    m = (int64_t)uni64((uint64_t)m);
    j0 = (int64_t)uni64((uint64_t)j0);
    const int n = __builtin_amdgcn_readfirstlane((int)n64);
    const int jl = (j0 + lane < m) ? lane : (int)(m - 1 - j0);
    char *px = reinterpret_cast<char *>(x + j0);
    const char *p0 = reinterpret_cast<const char *>(x0 + j0), *p1 = reinterpret_cast<const char *>(d1 + j0),
               *p2 = reinterpret_cast<const char *>(d2 + j0);
    const uint32_t l4 = (uint32_t)jl * 4, l8 = (uint32_t)jl * 8;
    const int64_t rs4 = m * 4, rs8 = m * 8;
    float c[3][U], nx[3][U];
    auto load = [&](float (&v)[3][U], int r0) {
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const bool in = r0 + t < n;
            const int64_t o = (int64_t)(r0 + t) * rs4;
            v[0][t] = in ? ld<float>(p0 + o, l4) : 0.0f;
            v[1][t] = in ? ld<float>(p1 + o, l4) : 0.0f;
            v[2][t] = in ? ld<float>(p2 + o, l4) : 0.0f;
        }
    };
    load(c, 0);
    for (int r0 = 0; r0 < n; r0 += U) {
        const bool more = r0 + U < n;
        if (more) load(nx, r0 + U);
#pragma unroll
        for (int t = 0; t < U; ++t)
            if (r0 + t < n)
                st<double>(px + (int64_t)(r0 + t) * rs8, l8, ((double)c[0][t] + (double)c[1][t]) + (double)c[2][t]);
        if (more) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int t = 0; t < U; ++t) c[q][t] = nx[q][t];
        }
    }
}

// x += delta, elementwise over the whole interleaved array (final correction).
__global__ __launch_bounds__(256) void k_update(double *__restrict__ x, const float *__restrict__ dl,
                                                int64_t total) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 2;
    for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; e < total; e += stride) {
        if (e + 1 < total) {
            double2 v = *reinterpret_cast<double2 *>(x + e);
            const float2 d = *reinterpret_cast<const float2 *>(dl + e);
            v.x += (double)d.x;
            v.y += (double)d.y;
            *reinterpret_cast<double2 *>(x + e) = v;
        } else {
            x[e] += (double)dl[e];
        }
    }
}

// ---------------------------------------------------------------------------
// Serving: one launch runs many requests (any matrix, n, m, precision).  The
// host cuts every request into tiles of 64 systems; each wave repeatedly
// takes the next tile from a counter and runs that tile's whole solve --
// for FP32 requests the FP32 solve, two residual/correction rounds and the
// final update, all on the tile's own columns -- with the same sweep and
// residual bodies as the plain entry points, so a request's result is
// bit-identical whether it runs alone or in a mix.  The loop ends when the
// counter passes the last tile, so every wave exits.
constexpr int kTileLds = 36 * 1024;  // LDS per tile wave: checkpoints + factor staging

template <int KIND, typename T>
__device__ __forceinline__ bool tile_fits_chunked(int n) {
    return wave_lds_bytes<KIND, T, 32, MODE_CHUNKED>((n + 31) / 32) <= (size_t)kTileLds;
}

template <int KIND>
__device__ __forceinline__ void run_tile_f64(const Tile &t, unsigned char *lds) {
    const int n = (int)t.n;
    using Row = typename Rec<KIND, double>::Row;
    const Row *fac = reinterpret_cast<const Row *>(t.fac);
    const double *in = reinterpret_cast<const double *>(t.in);
    if (tile_fits_chunked<KIND, double>(n))
        sweep_wave<KIND, double, double, double, 32, MODE_CHUNKED>(fac, n, in, t.x, t.m, t.col0, lds);
    else
        sweep_wave<KIND, double, double, double, 32, MODE_STREAM>(fac, n, in, t.x, t.m, t.col0, lds);
}

// The phases of an FP32 tile (solve, two residual / correction rounds, the
// final update) run one after another on the tile's 64 systems.
template <int KIND, typename Tout, int MODE>
__device__ __forceinline__ void tile_sweep_f32(const typename Rec<KIND, float>::Row *fac, int n, const float *in,
                                            Tout *out, int64_t m, int64_t j0, unsigned char *lds) {
    sweep_wave<KIND, float, float, Tout, 32, MODE>(fac, n, in, out, m, j0, lds);
}

// The refined tile keeps its intermediate values in FP32 in three n x m
// scratch arrays: x0 (the first solve), d1 (the first correction), r / d2
// (the second residual, then the second correction); x = fl64(x0 + d1) is
// formed where the second residual reads it and x = fl64(fl64(x0 + d1) + d2)
// at the end, the values an FP64 x updated in place would take (84 bytes per
// unknown with checkpointed sweeps, against 104 with x in FP64 throughout).
template <int KIND>
__device__ __forceinline__ void run_tile_f32(const Tile &t, unsigned char *lds) {
    const int n = (int)t.n;
    using Row = typename Rec<KIND, float>::Row;
    const Row *fac = reinterpret_cast<const Row *>(t.fac);
    const float *b = reinterpret_cast<const float *>(t.in);
    const int64_t nm = t.n * t.m;
    float *x0 = t.scratch, *d1 = t.scratch + nm, *d2 = t.scratch + 2 * nm;
    const bool chunk = tile_fits_chunked<KIND, float>(n);
    auto solve = [&](const float *in, float *out) {
        if (chunk)
            tile_sweep_f32<KIND, float, MODE_CHUNKED>(fac, n, in, out, t.m, t.col0, lds);
        else
            tile_sweep_f32<KIND, float, MODE_STREAM>(fac, n, in, out, t.m, t.col0, lds);
    };
    solve(b, x0);
    residual_wave<KIND, 0, float>(t.bands, n, b, x0, d1, d1, t.m, t.col0, lds);
    solve(d1, d1);
    residual_wave<KIND, 2, float>(t.bands, n, b, x0, d1, d2, t.m, t.col0, lds);
    solve(d2, d2);
    finish_wave(t.x, x0, d1, d2, n, t.m, t.col0);
}

// FP32 requests served as one FP64 sweep of their FP32 right-hand sides
// (the server's second mode for FP32 requests): the same result the
// mixed-precision solve converges to, the FP64 solve of the stored values,
// with 12 to 20 bytes per unknown instead of the correction rounds' passes.
template <int KIND>
__device__ __forceinline__ void run_tile_f32in(const Tile &t, unsigned char *lds) {
    const int n = (int)t.n;
    using Row = typename Rec<KIND, double>::Row;
    const Row *fac = reinterpret_cast<const Row *>(t.fac);
    const float *in = reinterpret_cast<const float *>(t.in);
    if (tile_fits_chunked<KIND, double>(n))
        sweep_wave<KIND, double, float, double, 32, MODE_CHUNKED>(fac, n, in, t.x, t.m, t.col0, lds);
    else
        sweep_wave<KIND, double, float, double, 32, MODE_STREAM>(fac, n, in, t.x, t.m, t.col0, lds);
}

// One kernel per (kind, precision) group of a launch's tiles (PREC 0: FP64
// requests, 1: FP32 requests refined, 2: FP32 requests as one FP64 sweep).
//
// Control flow in the persistent loop is wave-uniform throughout: every lane
// issues each atomic (lane 0 adds its amount, the others add 0) and the wave
// takes lane 0's result through readfirstlane, so every branch below is
// taken by the whole wave and no lane can reach the next ticket on a path of
// its own.  Completion of a request: after its tile each wave releases its
// results at system scope with its decrement of left[req]; the decrement that
// takes the count to zero also acquires every earlier one, and the flag store
// that follows releases them all to the host.
template <int KIND, int PREC>
__global__ __launch_bounds__(kWave) void k_tiles(const Tile *__restrict__ tiles, int ntiles, int *counter, int *left,
                                                 int *done) {
    __shared__ __align__(16) unsigned char lds[kTileLds];
    const int one = threadIdx.x == 0 ? 1 : 0;
    for (;;) {
        int t = atomicAdd(counter, one);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= ntiles) break;
        const Tile tl = tiles[t];
        if constexpr (PREC == 1)
            run_tile_f32<KIND>(tl, lds);
        else if constexpr (PREC == 2)
            run_tile_f32in<KIND>(tl, lds);
        else
            run_tile_f64<KIND>(tl, lds);
        const int req = __builtin_amdgcn_readfirstlane(tl.req);
        int before = __hip_atomic_fetch_add(&left[req], -one, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_SYSTEM);
        before = __builtin_amdgcn_readfirstlane(before);
        if (before == 1) __hip_atomic_store(&done[req], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// ---------------------------------------------------------------------------
// dst[c*rows + r] = src[r*cols + c] through a padded 64 x 64 LDS tile.
// Elements move as raw integers, so the copy is bit-exact.
template <typename E>
__global__ __launch_bounds__(256) void k_transpose(const E *__restrict__ src, E *__restrict__ dst,
                                                   int64_t rows, int64_t cols, int64_t tiles_c) {
    __shared__ E tile[64][65];
    const int64_t tr = blockIdx.x / tiles_c, tc = blockIdx.x % tiles_c;
    const int64_t r0 = tr * 64, c0 = tc * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int k = ty + 4 * q;
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) tile[k][tx] = src[r * cols + c];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int k = ty + 4 * q;
        const int64_t c = c0 + k, r = r0 + tx;
        if (c < cols && r < rows) dst[c * rows + r] = tile[tx][k];
    }
}

// ---------------------------------------------------------------------------
// Launch helpers.

template <int KIND, typename T, typename Tin, typename Tout, int L, int MODE>
hipError_t go(const sbs_lhs *h, const void *fac, const void *in, void *out, int64_t m,
              hipStream_t s) {
    using R = Rec<KIND, T>;
    const int64_t blocks = (m + kWave - 1) / kWave;
    const size_t lds = wave_lds_bytes<KIND, T, L, MODE>((int)((h->n + L - 1) / L));
    if (lds > kMaxLdsBytes) return hipErrorInvalidValue;
    // One wave may take up to the whole LDS of a CU: long systems keep their
    // chunk checkpoints on chip (24 bytes per unknown) instead of streaming
    // (32), at one or two waves per CU (pentadiagonal, 65536 systems: 2048
    // rows 671 us against 847 us, 3000 rows 1093 us against 1283 us).  Set
    // once per kernel (thread-safe static initialisation).
    static const hipError_t attr_small = hipFuncSetAttribute(
        reinterpret_cast<const void *>(k_sweep<KIND, T, Tin, Tout, L, MODE, false>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLdsBytes);
    static const hipError_t attr_big = hipFuncSetAttribute(
        reinterpret_cast<const void *>(k_sweep<KIND, T, Tin, Tout, L, MODE, true>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLdsBytes);
    if (attr_small != hipSuccess) return attr_small;
    if (attr_big != hipSuccess) return attr_big;
    // Row offsets inside a chunk must fit the 31-bit buffer offset, with room
    // for the lane offset; wider batches take one buffer resource per row.
    const int64_t span = (int64_t)L * m * (int64_t)(sizeof(Tin) > sizeof(Tout) ? sizeof(Tin) : sizeof(Tout));
    const auto *f = reinterpret_cast<const typename R::Row *>(fac);
    const auto *pi = reinterpret_cast<const Tin *>(in);
    auto *po = reinterpret_cast<Tout *>(out);
    if (span < (int64_t(1) << 31) - 4096)
        hipLaunchKernelGGL((k_sweep<KIND, T, Tin, Tout, L, MODE, false>), dim3((unsigned)blocks), dim3(kWave), lds, s,
                           f, (int)h->n, pi, po, m);
    else
        hipLaunchKernelGGL((k_sweep<KIND, T, Tin, Tout, L, MODE, true>), dim3((unsigned)blocks), dim3(kWave), lds, s,
                           f, (int)h->n, pi, po, m);
    return hipGetLastError();
}

template <int KIND, typename T, typename Tin, typename Tout>
hipError_t dispatch_mode(const sbs_lhs *h, int mode, const void *fac, const void *in, void *out,
                         int64_t m, hipStream_t s) {
    const int64_t n = h->n;
    if (mode == SBS_VARIANT_RESIDENT) {
        if (n <= 8) return go<KIND, T, Tin, Tout, 8, MODE_RESIDENT>(h, fac, in, out, m, s);
        if (n <= 16) return go<KIND, T, Tin, Tout, 16, MODE_RESIDENT>(h, fac, in, out, m, s);
        if (n <= 32) return go<KIND, T, Tin, Tout, 32, MODE_RESIDENT>(h, fac, in, out, m, s);
        if (n <= 64) return go<KIND, T, Tin, Tout, 64, MODE_RESIDENT>(h, fac, in, out, m, s);
        return hipErrorInvalidValue;
    }
    if (mode == SBS_VARIANT_CHUNKED) return go<KIND, T, Tin, Tout, 32, MODE_CHUNKED>(h, fac, in, out, m, s);
    return go<KIND, T, Tin, Tout, 32, MODE_STREAM>(h, fac, in, out, m, s);
}

// Crank-Nicolson step launches: the sweep variants with the output pass.
template <int KIND, typename T, int L, int MODE>
hipError_t go_cn(const sbs_lhs *h, const void *fac, void *c, int64_t m, hipStream_t s) {
    using R = Rec<KIND, T>;
    const int64_t blocks = (m + kWave - 1) / kWave;
    const size_t lds = wave_lds_bytes<KIND, T, L, MODE, true>((int)((h->n + L - 1) / L));
    if (lds > kMaxLdsBytes) return hipErrorInvalidValue;
    static const hipError_t attr_small = hipFuncSetAttribute(
        reinterpret_cast<const void *>(k_cn<KIND, T, L, MODE, false>), hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)kMaxLdsBytes);
    static const hipError_t attr_big = hipFuncSetAttribute(
        reinterpret_cast<const void *>(k_cn<KIND, T, L, MODE, true>), hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)kMaxLdsBytes);
    if (attr_small != hipSuccess) return attr_small;
    if (attr_big != hipSuccess) return attr_big;
    // the output pass stores up to two rows past the chunk
    const int64_t span = (int64_t)(L + 2) * m * (int64_t)sizeof(T);
    const auto *f = reinterpret_cast<const typename R::Row *>(fac);
    auto *pc = reinterpret_cast<T *>(c);
    if (span < (int64_t(1) << 31) - 4096)
        hipLaunchKernelGGL((k_cn<KIND, T, L, MODE, false>), dim3((unsigned)blocks), dim3(kWave), lds, s, f, h->bands,
                           (int)h->n, pc, m);
    else
        hipLaunchKernelGGL((k_cn<KIND, T, L, MODE, true>), dim3((unsigned)blocks), dim3(kWave), lds, s, f, h->bands,
                           (int)h->n, pc, m);
    return hipGetLastError();
}

template <int KIND, typename T>
hipError_t cn_mode(const sbs_lhs *h, const void *fac, void *c, int64_t m, hipStream_t s) {
    const int64_t n = h->n;
    if (n <= 8) return go_cn<KIND, T, 8, MODE_RESIDENT>(h, fac, c, m, s);
    if (n <= 16) return go_cn<KIND, T, 16, MODE_RESIDENT>(h, fac, c, m, s);
    if (n <= 32) return go_cn<KIND, T, 32, MODE_RESIDENT>(h, fac, c, m, s);
    if (n <= 64) return go_cn<KIND, T, 64, MODE_RESIDENT>(h, fac, c, m, s);
    if (wave_lds_bytes<KIND, T, 32, MODE_CHUNKED, true>((int)((n + 31) / 32)) <= kMaxLdsBytes)
        return go_cn<KIND, T, 32, MODE_CHUNKED>(h, fac, c, m, s);
    return go_cn<KIND, T, 32, MODE_STREAM>(h, fac, c, m, s);
}

template <typename T>
hipError_t cn_kind(const sbs_lhs *h, const void *fac, void *c, int64_t m, hipStream_t s) {
    if (h->kind == SBS_TRI) return cn_mode<SBS_TRI, T>(h, fac, c, m, s);
    if (h->kind == SBS_TRI_PERIODIC) return cn_mode<SBS_TRI_PERIODIC, T>(h, fac, c, m, s);
    return cn_mode<SBS_PENTA, T>(h, fac, c, m, s);
}

template <typename T, typename Tin, typename Tout>
hipError_t dispatch_kind(const sbs_lhs *h, int mode, const void *fac, const void *in, void *out,
                         int64_t m, hipStream_t s) {
    if (h->kind == SBS_TRI) return dispatch_mode<SBS_TRI, T, Tin, Tout>(h, mode, fac, in, out, m, s);
    if (h->kind == SBS_TRI_PERIODIC) return dispatch_mode<SBS_TRI_PERIODIC, T, Tin, Tout>(h, mode, fac, in, out, m, s);
    return dispatch_mode<SBS_PENTA, T, Tin, Tout>(h, mode, fac, in, out, m, s);
}

}  // namespace

size_t chunked_lds_bytes(const sbs_lhs *h, int tc) {
    const int K = (int)((h->n + 31) / 32);
    if (h->kind == SBS_TRI)
        return tc == 0 ? wave_lds_bytes<SBS_TRI, double, 32, MODE_CHUNKED>(K)
                       : wave_lds_bytes<SBS_TRI, float, 32, MODE_CHUNKED>(K);
    if (h->kind == SBS_TRI_PERIODIC)
        return tc == 0 ? wave_lds_bytes<SBS_TRI_PERIODIC, double, 32, MODE_CHUNKED>(K)
                       : wave_lds_bytes<SBS_TRI_PERIODIC, float, 32, MODE_CHUNKED>(K);
    return tc == 0 ? wave_lds_bytes<SBS_PENTA, double, 32, MODE_CHUNKED>(K)
                   : wave_lds_bytes<SBS_PENTA, float, 32, MODE_CHUNKED>(K);
}

hipError_t launch_cn(const sbs_lhs *h, int tc, void *c, int64_t m, hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    return tc == 0 ? cn_kind<double>(h, h->fac64, c, m, stream) : cn_kind<float>(h, h->fac32, c, m, stream);
}

int choose_variant(const sbs_lhs *h, int tc) {
    if (h->n <= 64) return SBS_VARIANT_RESIDENT;
    if (chunked_lds_bytes(h, tc) <= kMaxLdsBytes) return SBS_VARIANT_CHUNKED;
    return SBS_VARIANT_STREAM;
}

hipError_t launch_sweep(const sbs_lhs *h, int variant, int tc, int tin, int tout, const void *in,
                        void *out, int64_t m, hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    const int mode = variant == SBS_VARIANT_AUTO ? choose_variant(h, tc) : variant;
    if (tc == 0 && tin == 0 && tout == 0)
        return dispatch_kind<double, double, double>(h, mode, h->fac64, in, out, m, stream);
    if (tc == 1 && tin == 1 && tout == 1)
        return dispatch_kind<float, float, float>(h, mode, h->fac32, in, out, m, stream);
    if (tc == 1 && tin == 1 && tout == 0)
        return dispatch_kind<float, float, double>(h, mode, h->fac32, in, out, m, stream);
    return hipErrorInvalidValue;
}

namespace {
template <int KIND, typename T, int LB>
constexpr int part_maxt() {
    return (LB == 64 && sizeof(T) == 8) ? 512 : 1024;
}

// The partitioned kernel of (KIND, T, LB, CN), allowed the whole LDS of a CU.
template <int KIND, typename T, int LB, int CN>
hipError_t part_kernel(const void **fn) {
    auto kern = k_part<KIND, T, T, T, LB, part_maxt<KIND, T, LB>(), CN>;
    // once per instantiation; thread-safe static initialisation, so that
    // concurrent first launches from several host threads do not race
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kMaxPartLdsBytes);
    if (attr != hipSuccess) return attr;
    *fn = reinterpret_cast<const void *>(kern);
    return hipSuccess;
}

template <int KIND, typename T, int CN>
int part_wgs_lb(int lb, int threads, size_t lds) {
    const void *fn = nullptr;
    hipError_t e = lb == 16 ? part_kernel<KIND, T, 16, CN>(&fn)
                            : lb == 32 ? part_kernel<KIND, T, 32, CN>(&fn) : part_kernel<KIND, T, 64, CN>(&fn);
    return e != hipSuccess ? 0 : occupancy(fn, threads, lds);
}

// The blocks of a periodic tridiagonal matrix are plain tridiagonal.
int part_kind(int kind) { return kind == SBS_PENTA ? SBS_PENTA : SBS_TRI; }

// Workgroups of the partitioned kernel that one CU holds at once (registers,
// waves and LDS together).
template <int KIND, typename T>
int part_wgs_cn(int cn, int lb, int threads, size_t lds) {
    return cn == 2 ? part_wgs_lb<KIND, T, 2>(lb, threads, lds)
                   : cn == 1 ? part_wgs_lb<KIND, T, 1>(lb, threads, lds) : part_wgs_lb<KIND, T, 0>(lb, threads, lds);
}

int part_wgs_per_cu(int kind, int tc, int lb, int threads, size_t lds, int cn) {
    if (part_kind(kind) == SBS_TRI)
        return tc == 0 ? part_wgs_cn<SBS_TRI, double>(cn, lb, threads, lds)
                       : part_wgs_cn<SBS_TRI, float>(cn, lb, threads, lds);
    return tc == 0 ? part_wgs_cn<SBS_PENTA, double>(cn, lb, threads, lds)
                   : part_wgs_cn<SBS_PENTA, float>(cn, lb, threads, lds);
}

template <int KIND, typename T, int LB, int CN>
hipError_t go_part(const sbs_lhs *h, const PartChoice &c, const void *in, void *out, int64_t m, hipStream_t s) {
    constexpr int MAXT = part_maxt<KIND, T, LB>();
    const PartPlan &pp = h->part[c.plan];
    const bool f64 = sizeof(T) == 8;
    auto kern = k_part<KIND, T, T, T, LB, MAXT, CN>;
    const void *fn = nullptr;
    if (hipError_t e = part_kernel<KIND, T, LB, CN>(&fn); e != hipSuccess) return e;
    if (c.threads > MAXT) return hipErrorInvalidValue;
    const int ngroups = (int)((m + c.S - 1) / c.S);
    const int cus = device_cus(h->device);
    const int per_cu = std::max(1, c.wgs);
    const int grid = (int)std::min<int64_t>(ngroups, (int64_t)cus * per_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(c.threads), c.lds, s,
                       static_cast<const unsigned char *>(f64 ? pp.blob64 : pp.blob32),
                       (int)(f64 ? pp.fac_bytes64 : pp.fac_bytes32), (int)(f64 ? pp.spk_bytes64 : pp.spk_bytes32),
                       (int)(f64 ? pp.rinv_bytes64 : pp.rinv_bytes32), (int)h->n, pp.P, pp.Nr, c.S, ngroups,
                       (int)pp.periodic, h->bands, h->coef, static_cast<const T *>(in), static_cast<T *>(out), m);
    return hipGetLastError();
}

// Row layout (FP64 solves only): the same kernel reading each system as one
// contiguous run.
template <int KIND, int LB>
hipError_t go_part_rows(const sbs_lhs *h, const PartChoice &c, double *x, int64_t m, hipStream_t s) {
    constexpr int MAXT = part_maxt<KIND, double, LB>();
    const PartPlan &pp = h->part[c.plan];
    auto kern = k_part<KIND, double, double, double, LB, MAXT, 0, true>;
    // once per instantiation; thread-safe static initialisation, so that
    // concurrent first launches from several host threads do not race
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kMaxPartLdsBytes);
    if (attr != hipSuccess) return attr;
    if (c.threads > MAXT) return hipErrorInvalidValue;
    const int ngroups = (int)((m + c.S - 1) / c.S);
    const int cus = device_cus(h->device);
    const int grid = (int)std::min<int64_t>(ngroups, (int64_t)cus * std::max(1, c.wgs));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(c.threads), c.lds, s, static_cast<const unsigned char *>(pp.blob64),
                       (int)pp.fac_bytes64, (int)pp.spk_bytes64, (int)pp.rinv_bytes64, (int)h->n, pp.P, pp.Nr, c.S,
                       ngroups, (int)pp.periodic, h->bands, h->coef, x, x, m);
    return hipGetLastError();
}

template <int KIND, typename T, int CN>
hipError_t go_part_lb(const sbs_lhs *h, const PartChoice &c, const void *in, void *out, int64_t m, hipStream_t s) {
    switch (h->part[c.plan].lb) {
        case 16: return go_part<KIND, T, 16, CN>(h, c, in, out, m, s);
        case 32: return go_part<KIND, T, 32, CN>(h, c, in, out, m, s);
        default: return go_part<KIND, T, 64, CN>(h, c, in, out, m, s);
    }
}
}  // namespace

namespace {
// The fused refinement kernel of (KIND, LB), allowed the whole LDS of a CU.
template <int KIND, int LB>
hipError_t refine_kernel(const void **fn) {
    auto kern = k_part_refine<KIND, LB, 512>;
    // once per instantiation; thread-safe static initialisation, so that
    // concurrent first launches from several host threads do not race
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kMaxPartLdsBytes);
    if (attr != hipSuccess) return attr;
    *fn = reinterpret_cast<const void *>(kern);
    return hipSuccess;
}

int refine_wgs_per_cu(int kind, int lb, int threads, size_t lds) {
    const void *fn = nullptr;
    hipError_t e;
    if (kind == SBS_TRI)
        e = lb == 16 ? refine_kernel<SBS_TRI, 16>(&fn) : refine_kernel<SBS_TRI, 32>(&fn);
    else
        e = lb == 16 ? refine_kernel<SBS_PENTA, 16>(&fn) : refine_kernel<SBS_PENTA, 32>(&fn);
    return e != hipSuccess ? 0 : occupancy(fn, threads, lds);
}

template <int KIND, int LB>
hipError_t go_part_refine(const sbs_lhs *h, const PartChoice &c, const float *b, double *x, int64_t m, int sweeps,
                          hipStream_t s) {
    constexpr int MAXT = 512;
    const PartPlan &pp = h->part[c.plan];
    auto kern = k_part_refine<KIND, LB, MAXT>;
    const void *fn = nullptr;
    if (hipError_t e = refine_kernel<KIND, LB>(&fn); e != hipSuccess) return e;
    if (c.threads > MAXT) return hipErrorInvalidValue;
    const int ngroups = (int)((m + c.S - 1) / c.S);
    const int cus = device_cus(h->device);
    const int per_cu = std::max(1, c.wgs);
    const int grid = std::min(ngroups, cus * per_cu);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(c.threads), c.lds, s, static_cast<const unsigned char *>(pp.blob32),
                       (int)pp.fac_bytes32, (int)pp.spk_bytes32, (int)pp.rinv_bytes32, h->bands, (int)h->n, pp.P,
                       pp.Nr, c.S, ngroups, sweeps, b, x, m);
    return hipGetLastError();
}
}  // namespace

// Plan for the fused mixed-precision kernel: blocks of 16 or 32 rows (the
// lane keeps b, x and a work copy of its block in registers), at most 512
// threads, and LDS for the FP32 plan, the original bands, the interface
// values and the neighbour exchange.  Scored like the plain partition
// (concurrent waves, up to 8 per CU), but ties go first to more workgroups
// per CU: each group crosses several barriers, and two independent
// workgroups hide them (1M-system tridiagonal batch: 32-row blocks with 16
// systems per workgroup 2.77 ms, with 32 systems 3.03 ms, 16-row blocks
// 3.54 ms).
bool choose_partition_refine(const sbs_lhs *h, int64_t m, PartChoice *out) {
    const int H = h->kind / 2;
    const int cus = device_cus(h->device);
    PartChoice best;
    int64_t best_waves = -1;
    int best_wgs = 0;
    for (int q = 1; q >= 0; --q) {  // lb 32, then 16
        const PartPlan &pp = h->part[q];
        if (!pp.ok || m < 1) continue;
        for (int S = 64; S >= 16; S /= 2) {
            const int threads = S * pp.P;
            if (threads > 512) continue;
            const size_t npad = (size_t)pp.P * pp.lb;
            const size_t lds = pp.blob_bytes(1) + npad * sizeof(BandRow) +
                               ((size_t)S * (pp.Nr + 1) * 4 + 15) / 16 * 16 + (size_t)S * pp.P * 2 * H * 8;
            if (lds > kMaxPartLdsBytes) continue;
            const int wgs = refine_wgs_per_cu(h->kind, pp.lb, threads, lds);
            if (wgs < 1) continue;
            const int64_t groups = (m + S - 1) / S;
            const int64_t waves = std::min<int64_t>(
                std::min<int64_t>(groups, (int64_t)cus * wgs) * ((threads + kWave - 1) / kWave), (int64_t)cus * 8);
            if (waves > best_waves || (waves == best_waves && wgs > best_wgs)) {
                best_waves = waves;
                best_wgs = wgs;
                best.plan = q;
                best.S = S;
                best.threads = threads;
                best.lds = lds;
                best.wgs = wgs;
            }
        }
    }
    if (best.plan < 0) return false;
    *out = best;
    return true;
}

hipError_t launch_partition_refine(const sbs_lhs *h, const PartChoice &c, const float *b, double *x, int64_t m,
                                   int sweeps, hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    const int lb = h->part[c.plan].lb;
    if (h->kind == SBS_TRI)
        return lb == 16 ? go_part_refine<SBS_TRI, 16>(h, c, b, x, m, sweeps, stream)
                        : go_part_refine<SBS_TRI, 32>(h, c, b, x, m, sweeps, stream);
    return lb == 16 ? go_part_refine<SBS_PENTA, 16>(h, c, b, x, m, sweeps, stream)
                    : go_part_refine<SBS_PENTA, 32>(h, c, b, x, m, sweeps, stream);
}

// Block length and systems per workgroup S for the partitioned solve.  The
// score is the number of lanes that run at once over the whole batch and hold
// a system, counted up to 8 full waves per CU (enough to keep HBM busy: more
// buys nothing once the batch fills the chip, and a 1M-system tridiagonal
// batch ran 16% slower on the 32-row blocks that allow 16).  Lanes, not
// waves: a workgroup of 16 threads fills a quarter of its wave, and for small
// batches the shorter blocks that give each system more lanes win.  Ties go,
// in order, to row accesses that are whole 128-byte lines (S >= 16 in FP64,
// 32 in FP32), to more CUs engaged, to longer blocks (fewer interfaces) and
// to larger S (each row access of a block covers S consecutive systems, and
// wider runs stream better: on the 1024-row pentadiagonal batch S = 32 274
// us, S = 16 299 us, both with 8 waves per CU).  1024 tridiagonal systems of
// 256 rows, replayed from a graph: 16-row blocks with S = 16 (64 CUs) 5.1
// us, S = 8 5.5, S = 64 (16 CUs) 8.7; 64-row blocks with S = 4 13.5 us.
// Workgroups narrower than 16 systems are only tried when the batch is too
// small to give every CU a group.
// cn: 0 a solve; 1 a Crank-Nicolson step, which also holds the band rows
// (2h+1 doubles per row) and the exchange of block ends in LDS; 2 the same
// step for constant bands (no band rows).  In FP64 pentadiagonal plans the
// interface unknowns take a second array the size of the interface values
// (the matrix-core form).  rows: each lane reads its block as one contiguous
// run, so every S counts as whole lines and more CUs decide (2048 rows of a
// 2048 x 2048 grid: 8 systems per workgroup on 256 CUs 29.5 us, 16 on 128
// CUs 36.9 us; in the interleaved layout of its columns 16 systems, whole
// lines, 19.9 us against 26.3 us with 8).
bool choose_partition(const sbs_lhs *h, int tc, int64_t m, PartChoice *out, int cn, bool rows) {
    const size_t elem = tc == 0 ? 8 : 4;
    const int H = part_kind(h->kind) / 2;
    const int cus = device_cus(h->device);
    PartChoice best;
    int64_t best_lanes = -1, best_cus = -1;
    bool best_lines = false;
    for (int q = 2; q >= 0; --q) {  // largest block first: fewest interfaces
        const PartPlan &pp = h->part[q];
        if (!pp.ok || m < 1) continue;
        const int maxt = (pp.lb == 64 && elem == 8) ? 512 : 1024;
        const size_t blob = pp.blob_bytes(tc);
        for (int S = 64; S >= 4; S /= 2) {
            if (S < 16 && (m + 2 * S - 1) / (2 * S) >= cus) break;  // the wider S already fills the CUs
            const int threads = S * pp.P;
            if (threads > maxt) continue;
            // interface values, and for FP64 pentadiagonal the interface unknowns beside them
            const bool mma = tc == 0 && H == 2;
            size_t lds = blob + ((size_t)S * (pp.Nr + 1) * elem + 15) / 16 * 16 * (mma ? 2 : 1);
            if (cn == 1) lds += ((size_t)pp.P * pp.lb * (2 * H + 1) * 8 + 15) / 16 * 16;  // band rows
            if (cn) lds += ((size_t)S * pp.P * 2 * H * elem + 15) / 16 * 16;              // block ends
            if (lds > kMaxPartLdsBytes) continue;
            const int wgs = part_wgs_per_cu(h->kind, tc, pp.lb, threads, lds, cn);
            if (wgs < 1) continue;
            const int64_t groups = (m + S - 1) / S;
            // lanes that hold a system (a last group may be partly empty)
            const int64_t systems = std::min<int64_t>(m, std::min<int64_t>(groups, (int64_t)cus * wgs) * S);
            const int64_t lanes = std::min<int64_t>(systems * pp.P, (int64_t)cus * 8 * kWave);
            // the row layout reads each block as one run whatever S is
            const bool lines = rows || (size_t)S * elem >= 128;
            const int64_t engaged = std::min<int64_t>(groups, cus);
            // larger scores first; the loops visit longer blocks and then
            // larger S first, so a full tie keeps the earlier shape
            const bool better =
                lanes != best_lanes ? lanes > best_lanes
                                    : lines != best_lines ? lines : engaged > best_cus;
            if (better) {
                best_lanes = lanes;
                best_lines = lines;
                best_cus = engaged;
                best.plan = q;
                best.S = S;
                best.threads = threads;
                best.lds = lds;
                best.wgs = wgs;
            }
        }
    }
    if (best.plan < 0) return false;
    *out = best;
    return true;
}

bool part_shape(const sbs_lhs *h, int tc, int64_t m, int lb, int S, PartChoice *out) {
    const size_t elem = tc == 0 ? 8 : 4;
    const int H = part_kind(h->kind) / 2;
    for (int q = 0; q < 3; ++q) {
        const PartPlan &pp = h->part[q];
        if (!pp.ok || pp.lb != lb || m < 1 || S < 1 || S > 64) continue;
        const int maxt = (pp.lb == 64 && elem == 8) ? 512 : 1024;
        const int threads = S * pp.P;
        if (threads > maxt) return false;
        const bool mma = tc == 0 && H == 2;
        const size_t lds = pp.blob_bytes(tc) + ((size_t)S * (pp.Nr + 1) * elem + 15) / 16 * 16 * (mma ? 2 : 1);
        if (lds > kMaxPartLdsBytes) return false;
        const int wgs = part_wgs_per_cu(h->kind, tc, pp.lb, threads, lds, 0);
        if (wgs < 1) return false;
        out->plan = q;
        out->S = S;
        out->threads = threads;
        out->lds = lds;
        out->wgs = wgs;
        return true;
    }
    return false;
}

template <int KIND, typename T>
hipError_t go_part_cn(const sbs_lhs *h, const PartChoice &c, const void *in, void *out, int64_t m, hipStream_t s,
                      int cn) {
    return cn == 2 ? go_part_lb<KIND, T, 2>(h, c, in, out, m, s)
                   : cn == 1 ? go_part_lb<KIND, T, 1>(h, c, in, out, m, s) : go_part_lb<KIND, T, 0>(h, c, in, out, m, s);
}

hipError_t launch_partition(const sbs_lhs *h, const PartChoice &c, int tc, int tin, int tout, const void *in, void *out,
                            int64_t m, hipStream_t stream, int cn) {
    if (m <= 0) return hipSuccess;
    if (tc != tin || tc != tout || cn < 0 || cn > 2 || (cn == 2 && !h->constant_bands)) return hipErrorInvalidValue;
    if (part_kind(h->kind) == SBS_TRI)
        return tc == 0 ? go_part_cn<SBS_TRI, double>(h, c, in, out, m, stream, cn)
                       : go_part_cn<SBS_TRI, float>(h, c, in, out, m, stream, cn);
    return tc == 0 ? go_part_cn<SBS_PENTA, double>(h, c, in, out, m, stream, cn)
                   : go_part_cn<SBS_PENTA, float>(h, c, in, out, m, stream, cn);
}

hipError_t launch_partition_rows(const sbs_lhs *h, const PartChoice &c, double *x, int64_t m, hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    const int lb = h->part[c.plan].lb;
    if (part_kind(h->kind) == SBS_TRI)
        return lb == 16 ? go_part_rows<SBS_TRI, 16>(h, c, x, m, stream)
                        : lb == 32 ? go_part_rows<SBS_TRI, 32>(h, c, x, m, stream)
                                   : go_part_rows<SBS_TRI, 64>(h, c, x, m, stream);
    return lb == 16 ? go_part_rows<SBS_PENTA, 16>(h, c, x, m, stream)
                    : lb == 32 ? go_part_rows<SBS_PENTA, 32>(h, c, x, m, stream)
                               : go_part_rows<SBS_PENTA, 64>(h, c, x, m, stream);
}

hipError_t launch_refine_step(const sbs_lhs *h, int mode, const float *b, double *x,
                              const float *delta, float *r, int64_t m, hipStream_t stream) {
    if (m <= 0) return hipSuccess;
    if (mode == 2) {
        const int64_t total = h->n * m;
        int64_t blocks = (total / 2 + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(k_update, dim3((unsigned)blocks), dim3(256), 0, stream, x, delta, total);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((m + kWave - 1) / kWave));
    if (h->kind == SBS_TRI) {
        if (mode == 0)
            hipLaunchKernelGGL((k_residual<SBS_TRI, 0>), grid, dim3(kWave), 0, stream, h->bands, h->n, b, x, delta, r, m);
        else
            hipLaunchKernelGGL((k_residual<SBS_TRI, 1>), grid, dim3(kWave), 0, stream, h->bands, h->n, b, x, delta, r, m);
    } else {
        if (mode == 0)
            hipLaunchKernelGGL((k_residual<SBS_PENTA, 0>), grid, dim3(kWave), 0, stream, h->bands, h->n, b, x, delta, r, m);
        else
            hipLaunchKernelGGL((k_residual<SBS_PENTA, 1>), grid, dim3(kWave), 0, stream, h->bands, h->n, b, x, delta, r, m);
    }
    return hipGetLastError();
}

hipError_t launch_tiles(int kind, int prec, const Tile *dev_tiles, int ntiles, int *dev_counter, int *left,
                        int *done, int grid, hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    if (prec < 0 || prec > 2) return hipErrorInvalidValue;
    if (grid > ntiles) grid = ntiles;
    const dim3 g((unsigned)grid), b(kWave);
    const bool tri = kind == SBS_TRI;
    if (prec == 0) {
        if (tri)
            hipLaunchKernelGGL((k_tiles<SBS_TRI, 0>), g, b, 0, stream, dev_tiles, ntiles, dev_counter, left, done);
        else
            hipLaunchKernelGGL((k_tiles<SBS_PENTA, 0>), g, b, 0, stream, dev_tiles, ntiles, dev_counter, left, done);
    } else if (prec == 1) {
        if (tri)
            hipLaunchKernelGGL((k_tiles<SBS_TRI, 1>), g, b, 0, stream, dev_tiles, ntiles, dev_counter, left, done);
        else
            hipLaunchKernelGGL((k_tiles<SBS_PENTA, 1>), g, b, 0, stream, dev_tiles, ntiles, dev_counter, left, done);
    } else {
        if (tri)
            hipLaunchKernelGGL((k_tiles<SBS_TRI, 2>), g, b, 0, stream, dev_tiles, ntiles, dev_counter, left, done);
        else
            hipLaunchKernelGGL((k_tiles<SBS_PENTA, 2>), g, b, 0, stream, dev_tiles, ntiles, dev_counter, left, done);
    }
    return hipGetLastError();
}

hipError_t launch_transpose(const void *src, void *dst, int64_t rows, int64_t cols, int elem_bytes,
                            hipStream_t stream) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int64_t tiles_c = (cols + 63) / 64, tiles_r = (rows + 63) / 64;
    const int64_t blocks = tiles_c * tiles_r;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_transpose<unsigned long long>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           reinterpret_cast<const unsigned long long *>(src),
                           reinterpret_cast<unsigned long long *>(dst), rows, cols, tiles_c);
    else
        hipLaunchKernelGGL(k_transpose<unsigned int>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           reinterpret_cast<const unsigned int *>(src), reinterpret_cast<unsigned int *>(dst),
                           rows, cols, tiles_c);
    return hipGetLastError();
}

}  // namespace sbs
