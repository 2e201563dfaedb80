// Separator-partitioned solve (several lanes per system) for plain solves of
// interleaved right-hand sides.
//
// The rows of every system are cut into P blocks of LB rows.  The last H rows
// of each block (but the last, unless the matrix is periodic) are separator
// rows; the others are interior rows.  A workgroup holds S systems x P
// blocks: lane (p, s) loads rows [p*LB, (p+1)*LB) of VEC adjacent systems
// (VEC = 2: one 16-byte access per FP64 row), and then, per group of S
// systems:
//   1. runs the Section 3.1 / 4.1 recurrences over its block with the
//      block's interior factor (separator rows are identity rows, so they pass
//      through holding their right-hand sides);
//   2. writes to LDS its two parts of the separator right-hand sides
//      yhat = f_sep - (couplings of the separator rows to the interior rows
//      on either side) . g: its own separator's f_sep less the couplings to
//      the block's last interior rows (redL), and minus the previous
//      separator's couplings to the block's first rows (redR); one barrier;
//   3. the separators of all S systems follow as Z = S^{-1} Yhat, a dense
//      (Nr x Nr)(Nr x S) product on the matrix cores in FP64 (per-lane dot
//      products otherwise);
//   4. corrects its interior rows x = g - V z_own - W z_prev, takes its
//      separator rows from z, and stores every row once, non-temporally,
//      loading the next group's rows into the registers it frees.
// Each right-hand side crosses HBM once in and once out (16 bytes per FP64
// unknown).  The block factors, spikes V / W, separator band rows and S^{-1}
// depend only on the shared matrix; they are computed once on the host and
// copied into LDS once per persistent workgroup (where the whole plan does
// not fit, only S^{-1} is, and the rest is read from global memory).
#include <algorithm>

#include "internal.h"

namespace sbs {
namespace {

typedef double D2 __attribute__((ext_vector_type(2)));
typedef float F2 __attribute__((ext_vector_type(2)));
typedef double D4 __attribute__((ext_vector_type(4)));

template <int KIND, typename T>
struct RowOf;
template <typename T>
struct RowOf<SBS_TRI, T> {
    using type = TriRow<T>;
};
template <typename T>
struct RowOf<SBS_PENTA, T> {
    using type = PentaRow<T>;
};

template <typename T>
struct Pair;
template <>
struct Pair<double> {
    using type = D2;
};
template <>
struct Pair<float> {
    using type = F2;
};

// VEC adjacent values of one row (one 8/16-byte access for VEC = 2).
template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T *p, T (&v)[VEC]) {
    if constexpr (VEC == 1) {
        v[0] = *p;
    } else {
        const typename Pair<T>::type a = *reinterpret_cast<const typename Pair<T>::type *>(p);
        v[0] = a.x;
        v[1] = a.y;
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec_nt(T *p, const T (&v)[VEC]) {
    if constexpr (VEC == 1) {
        __builtin_nontemporal_store(v[0], p);
    } else {
        typename Pair<T>::type a;
        a.x = v[0];
        a.y = v[1];
        __builtin_nontemporal_store(a, reinterpret_cast<typename Pair<T>::type *>(p));
    }
}

__device__ __forceinline__ int align16(int b) { return (b + 15) / 16 * 16; }

// Copies the plan blob into LDS, eight 16-byte loads in flight per thread.
__device__ __forceinline__ void stage(unsigned char *lds, const unsigned char *blob, int bytes) {
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

struct SepArgs {
    int fac_bytes, spk_bytes, scf_bytes, sinv_bytes, map_bytes;
    int n, P, Nr, S, ngroups, periodic, flags;
    int kofs, kw;  // window of the S^{-1} product (kw = 0: every column)
    int64_t m;
    BandCoef coef;  // Crank-Nicolson steps: the matrix's constant band values
};

// Z = S^{-1} Yhat for the group on the matrix cores (Yhat = redl + redr, the
// two parts of the separator right-hand sides): 16 x 16 output tiles of
// v_mfma_f64_16x16x4f64 shared out over the waves (lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; item r of the result is
// D[4 r + l / 16][l % 16]).  Column s of Yhat / Z is at red / z + s * ldr.
//
// One 16 x 16 tile of Z: the lane's row i of S^{-1} and column j of Yhat
// over columns kb .. kb + kn - 1, four per matrix-core step.  Every operand
// is read at an index clamped inside the buffers, so that no read is
// conditional (as branches around each read the steps ran one after
// another), and the next step's operands are read before the current step's
// product.  Rows i >= Nr and columns j >= S of the tile hold other rows' and
// columns' values and are never stored; entries of S^{-1} past column Nr - 1
// are multiplied by 0 (finite values: the entries of S^{-1}), so the
// right-hand sides read there add nothing.
__device__ __forceinline__ D4 sep_tile(const double *sinv, const double *redl, const double *redr, int Nr, int S,
                                       int ldr, int i, int j, int lk, int kb, int kn) {
    const double *arow = sinv + (size_t)min(i, Nr - 1) * Nr;
    const double *bl = redl + min(j, S - 1) * ldr, *br = redr + min(j, S - 1) * ldr;
    auto opnd = [&](int k0, double &a, double &b) {
        const int k = k0 + lk, kc = min(k, Nr - 1);
        a = arow[kc] * (k < Nr ? 1.0 : 0.0);
        b = bl[kc] + br[kc];
    };
    D4 acc = {0.0, 0.0, 0.0, 0.0};
    double a, b;
    opnd(kb, a, b);
    for (int k0 = kb + 4; k0 < kb + kn; k0 += 4) {
        double an, bn;
        opnd(k0, an, bn);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        a = an;
        b = bn;
    }
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// The entries of S^{-1} outside a tile's window are 0 (the plan drops
// entries below 2^-60 / Nr of their row's largest), so the tile reads only
// columns k0 .. k0 + kw - 1, k0 = min(max(i0 + kofs, 0), max(Nr4 - kw, 0)),
// and the result is the product over every column bit for bit (the skipped
// terms are exact zeros); kw = 0 reads every column.
//
// ALIAS: z is redl's storage (the LDS holds no third buffer); each wave has
// at most one tile, and writes it only after every wave has read Yhat.
template <bool ALIAS>
__device__ __forceinline__ void sep_mma(const double *sinv, const double *redl, const double *redr, double *z, int Nr,
                                        int S, int ldr, int kofs, int kw) {
    // the thread's coordinates, made opaque at each call: the tile addresses
    // below are formed per call rather than kept live across the group loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid % kWave, wave = __builtin_amdgcn_readfirstlane(tid / kWave), nwaves = blockDim.x / kWave;
    const int mt = (Nr + 15) / 16, ntiles = mt * ((S + 15) / 16);
    const int lr = lane % 16, lk = lane / 16;
    const int Nr4 = (Nr + 3) / 4 * 4, kn = kw ? kw : Nr;
    auto kfirst = [&](int i0) { return kw ? min(max(i0 + kofs, 0), max(Nr4 - kw, 0)) : 0; };
    if constexpr (ALIAS) {
        const bool have = wave < ntiles;
        const int i0 = (wave % mt) * 16, j0 = (wave / mt) * 16;
        const int i = i0 + lr, j = j0 + lr;
        D4 acc = {0.0, 0.0, 0.0, 0.0};
        if (have) acc = sep_tile(sinv, redl, redr, Nr, S, ldr, i, j, lk, kfirst(i0), kn);
        __syncthreads();
        if (have) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + 4 * r + lk;
                if (row < Nr && j < S) z[j * ldr + row] = acc[r];
            }
        }
        return;
    }
    for (int tile = wave; tile < ntiles; tile += nwaves) {
        const int i0 = (tile % mt) * 16, j0 = (tile / mt) * 16;
        const int i = i0 + lr, j = j0 + lr;
        const D4 acc = sep_tile(sinv, redl, redr, Nr, S, ldr, i, j, lk, kfirst(i0), kn);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = i0 + 4 * r + lk;
            if (row < Nr && j < S) z[j * ldr + row] = acc[r];
        }
    }
}

// LDS layout after the blob: the two parts of the separator right-hand
// sides, redL and redR [S][ldr], and (FP64) the separators z [S][ldr].
template <typename T>
__host__ __device__ __forceinline__ int sep_red_bytes(int S, int Nr) {
    return (S * (Nr + 1) * (int)sizeof(T) + 15) / 16 * 16;
}

// Compiler-only fence: `v` must be computed here, and no memory access moves
// across (emits no instruction).  Keeps the coefficient reads of later rows
// from being hoisted to the start of a loop, where they would hold every
// row's coefficients in registers at once.
template <typename T>
__device__ __forceinline__ void pin(T &v) {
    asm volatile("" : "+v"(v) : : "memory");
}

constexpr int G = 4;  // rows per coefficient group (2 where registers are short)

// The block's forward and backward sweeps (Sections 3.1 / 4.1) over VEC
// systems in registers, with the block's factor rows from LDS.
// OPQ (rows in global memory): the row pointer is made opaque before each
// group of rows is read, so that the read-only loads are not all hoisted to
// the start (the fences below do not hold back loads of memory that nothing
// in the kernel writes).
template <int KIND, typename T, int LB, int VEC, bool OPQ>
__device__ __forceinline__ void block_sweeps(const typename RowOf<KIND, T>::type *fr, T (&x)[LB][VEC]) {
    // coefficient rows per group: fewer when the block's values fill the registers
    constexpr int NG = LB / G;
    if constexpr (KIND == SBS_TRI) {
        T cf[2][G][2];
        T y1[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) y1[v] = T(0);
        if constexpr (OPQ) asm volatile("" : "+v"(fr));
#pragma unroll
        for (int u = 0; u < G; ++u) cf[0][u][0] = fr[u].a_s, cf[0][u][1] = fr[u].inv;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (g + 1 < NG) {
                if constexpr (OPQ) asm volatile("" : "+v"(fr));
#pragma unroll
                for (int u = 0; u < G; ++u)
                    cf[(g + 1) & 1][u][0] = fr[(g + 1) * G + u].a_s, cf[(g + 1) & 1][u][1] = fr[(g + 1) * G + u].inv;
            }
#pragma unroll
            for (int u = 0; u < G; ++u)
#pragma unroll
                for (int v = 0; v < VEC; ++v)  // y_i = d_i / den_i - (a_i / den_i) y_{i-1}
                    y1[v] = x[g * G + u][v] = fma(-cf[g & 1][u][0], y1[v], x[g * G + u][v] * cf[g & 1][u][1]);
            pin(y1[0]);
        }
        T ch[2][G];
        T x1[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) x1[v] = T(0);
        if constexpr (OPQ) asm volatile("" : "+v"(fr));
#pragma unroll
        for (int u = 0; u < G; ++u) ch[(NG - 1) & 1][u] = fr[LB - 1 - u].chat;
#pragma unroll
        for (int g = NG - 1; g >= 0; --g) {
            if (g > 0) {
                if constexpr (OPQ) asm volatile("" : "+v"(fr));
#pragma unroll
                for (int u = 0; u < G; ++u) ch[(g - 1) & 1][u] = fr[g * G - 1 - u].chat;
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int t = g * G + G - 1 - u;
#pragma unroll
                for (int v = 0; v < VEC; ++v)  // x_i = y_i - chat_i x_{i+1}
                    x1[v] = x[t][v] = fma(-ch[g & 1][u], x1[v], x[t][v]);
            }
            pin(x1[0]);
        }
    } else {
        T cf[2][G][3];
        T g1[VEC], g2[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) g1[v] = g2[v] = T(0);
        if constexpr (OPQ) asm volatile("" : "+v"(fr));
#pragma unroll
        for (int u = 0; u < G; ++u) cf[0][u][0] = fr[u].eps_s, cf[0][u][1] = fr[u].beta_s, cf[0][u][2] = fr[u].inv;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (g + 1 < NG) {
                if constexpr (OPQ) asm volatile("" : "+v"(fr));
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const int t = (g + 1) * G + u;
                    cf[(g + 1) & 1][u][0] = fr[t].eps_s;
                    cf[(g + 1) & 1][u][1] = fr[t].beta_s;
                    cf[(g + 1) & 1][u][2] = fr[t].inv;
                }
            }
#pragma unroll
            for (int u = 0; u < G; ++u)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {  // g_i = (f_i - eps_i g_{i-2} - beta_i g_{i-1}) / alpha_i
                    const T *c = cf[g & 1][u];
                    const T gg = fma(-c[1], g1[v], fma(-c[0], g2[v], x[g * G + u][v] * c[2]));
                    g2[v] = g1[v];
                    g1[v] = gg;
                    x[g * G + u][v] = gg;
                }
            pin(g1[0]);
        }
        T cb[2][G][2];
        T x1[VEC], x2[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) x1[v] = x2[v] = T(0);
        if constexpr (OPQ) asm volatile("" : "+v"(fr));
#pragma unroll
        for (int u = 0; u < G; ++u) cb[(NG - 1) & 1][u][0] = fr[LB - 1 - u].gamma, cb[(NG - 1) & 1][u][1] = fr[LB - 1 - u].delta;
#pragma unroll
        for (int g = NG - 1; g >= 0; --g) {
            if (g > 0) {
                if constexpr (OPQ) asm volatile("" : "+v"(fr));
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const int t = g * G - 1 - u;
                    cb[(g - 1) & 1][u][0] = fr[t].gamma;
                    cb[(g - 1) & 1][u][1] = fr[t].delta;
                }
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int t = g * G + G - 1 - u;
#pragma unroll
                for (int v = 0; v < VEC; ++v) {  // x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2}
                    const T xx = fma(-cb[g & 1][u][0], x1[v], fma(-cb[g & 1][u][1], x2[v], x[t][v]));
                    x2[v] = x1[v];
                    x1[v] = xx;
                    x[t][v] = xx;
                }
            }
            pin(x1[0]);
        }
    }
}

// flags: bit 0 XCD-grouped order of the groups (the workgroups a chiplet
// runs at once take adjacent groups); bit 2 workgroups start out of step (see
// below); bit 6 the S^{-1} product over every column instead of the plan's
// window (same result).  (Issuing the next group's loads into registers while the current
// group is stored was measured slower: each wave's loads then queue behind
// its stores.)
//
// GF: the plan does not fit the LDS with the group's buffers; only S^{-1}
// is copied there, and the factor rows, spikes, separator rows and block map
// are read from global memory (the caches hold them: every group reads the
// same plan).  The separators then overwrite redL, and the corrected rows
// are stored after all of them are computed (a spike load issued after a
// store would wait for that store).
//
// CN: one Crank-Nicolson step c <- A^{-1} (2I - A) c (Sections 3.2, 4.2) of a
// matrix whose bands are constant (the values in a.coef): with u = A^{-1} c in
// registers, row t of the output is 2 u_t - sum_e coef_e u_{t-H+e}.  The rows
// above the block are the previous block's separators (known to the lane);
// the first H rows of the next block come through LDS, one more barrier.
// Values outside the matrix are 0, so the constant coefficients also give
// the truncated rows at its ends.
template <int KIND, typename T, int LB, int VEC, int MAXT, bool GF, bool CN = false>
__global__ __launch_bounds__(MAXT) void k_sep(const unsigned char *__restrict__ blob, SepArgs a, const T *in,
                                              T *out) {
    using Row = typename RowOf<KIND, T>::type;
    constexpr int H = KIND / 2, NB = 2 * H + 1, NI = LB - H;
    constexpr bool MMA = sizeof(T) == 8;
    extern __shared__ __align__(16) unsigned char lds[];
    const int P = a.P, Nr = a.Nr, S = a.S, n = a.n;
    const int blob_bytes = a.fac_bytes + a.spk_bytes + a.scf_bytes + a.sinv_bytes + a.map_bytes;
    const int sinv_at = a.fac_bytes + a.spk_bytes + a.scf_bytes;
    const Row *lfac;
    const T *lspk, *lscf, *lsinv;
    const int *lmap;
    if constexpr (GF) {
        lfac = reinterpret_cast<const Row *>(blob);
        lspk = reinterpret_cast<const T *>(blob + a.fac_bytes);
        lscf = reinterpret_cast<const T *>(blob + a.fac_bytes + a.spk_bytes);
        lmap = reinterpret_cast<const int *>(blob + sinv_at + a.sinv_bytes);
        lsinv = reinterpret_cast<const T *>(lds);
    } else {
        lfac = reinterpret_cast<const Row *>(lds);
        lspk = reinterpret_cast<const T *>(lds + a.fac_bytes);
        lscf = reinterpret_cast<const T *>(lds + a.fac_bytes + a.spk_bytes);
        lsinv = reinterpret_cast<const T *>(lds + sinv_at);
        lmap = reinterpret_cast<const int *>(lds + sinv_at + a.sinv_bytes);
    }
    const int plan_lds = GF ? a.sinv_bytes : blob_bytes;
    const int ldr = Nr + 1;  // odd stride: the systems' columns fall in different banks
    T *lredl = reinterpret_cast<T *>(lds + plan_lds);
    T *lredr = reinterpret_cast<T *>(lds + plan_lds + sep_red_bytes<T>(S, Nr));
    // flags bit 5 (GF only, set by the launch when the LDS has no room for a
    // third buffer): the separators overwrite redL
    const bool alias = GF && (a.flags & 32);
    T *lz = alias ? lredl : reinterpret_cast<T *>(lds + plan_lds + 2 * sep_red_bytes<T>(S, Nr));
    // CN: the first H rows of every block of the group, [S][P][H]
    T *ltop = reinterpret_cast<T *>(lds + plan_lds + (alias ? 2 : 3) * sep_red_bytes<T>(S, Nr));


    const int Ls = S / VEC;  // lanes per block row
    const int l = threadIdx.x, p = l / Ls, sl = l - p * Ls;
    const int r0 = p * LB;
    const bool has_sep = a.periodic || p < P - 1, has_prev = a.periodic || p > 0;
    const int pp = p == 0 ? P - 1 : p - 1;
    const int s0 = sl * VEC;  // the lane's first system within the group
    const int64_t m = a.m;
    const bool full = r0 + LB <= n;
    const int grid = gridDim.x;
    int b = blockIdx.x;
    if ((a.flags & 1) && grid % 8 == 0) b = (b % 8) * (grid / 8) + b / 8;

    T x[LB][VEC];
    // lanes past the last system take the last VEC systems: same values, same
    // addresses, so their duplicate stores are harmless
    auto col = [&](int g) { return min((int64_t)g * S + s0, m - VEC); };
    auto load_group = [&](int g) {
        const T *src = in + (int64_t)r0 * m + col(g);
        if (full) {
#pragma unroll
            for (int t = 0; t < LB; ++t) load_vec<T, VEC>(src + (int64_t)t * m, x[t]);
        } else {
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                if (r0 + t < n) {
                    load_vec<T, VEC>(src + (int64_t)t * m, x[t]);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) x[t][v] = T(0);
                }
            }
        }
    };

    int g = b;
    if constexpr (GF)
        stage(lds, blob + sinv_at, a.sinv_bytes);
    else
        stage(lds, blob, blob_bytes);
    // flags bit 2: workgroups start out of step (b % 4 quarter steps of
    // `stagger` sleeps of 4096 cycles each), so that while some compute their
    // separators others stream, instead of every CU reaching its compute
    // phase at the same time
    if (a.flags & 4) {
        const int steps = (b % 4) * (a.flags >> 8);
        for (int i = 0; i < steps; ++i) __builtin_amdgcn_s_sleep(64);
    }
    __syncthreads();
    if (g < a.ngroups) load_group(g);
    const int q = lmap[p];  // stored copy of this block's factor, spikes and separator rows
    const Row *fr0 = lfac + q * LB;
    const T *sp0 = lspk + q * LB * 2 * H;
    const T *cf = lscf + q * H * NB;
    const T *cfp = lscf + lmap[pp] * H * NB;  // the previous block's separator rows
    // the separator rows' couplings to interior rows, the same for every
    // group: the own separator's to this block's last rows (c + d < H) and
    // the previous separator's to this block's first rows (c + d >= 2H)
    T cl[H][H], cr[H][H];
#pragma unroll
    for (int c = 0; c < H; ++c)
#pragma unroll
        for (int d = 0; d < H; ++d) {
            cl[c][d] = (c + d < H) ? cf[c * NB + d] : T(0);
            cr[c][d] = (2 * H - c + d < NB) ? cfp[c * NB + 2 * H - c + d] : T(0);
        }
    for (; g < a.ngroups; g += grid) {
        // the lane's offsets into the separator buffers, made opaque each
        // group so that the addresses derived from them are formed where they
        // are used instead of being kept live (and spilled) across the loop
        int o_own = s0 * ldr + H * p, o_prev = s0 * ldr + H * pp, o_col = s0 * ldr;
        asm volatile("" : "+v"(o_own), "+v"(o_prev), "+v"(o_col));
        // GF: the plan is read-only global memory, and its loads would be
        // hoisted out of the loop (every row's coefficients live at once)
        // unless its addresses are opaque here too
        const Row *fr = fr0;
        const T *sp = sp0;
        if constexpr (GF) asm volatile("" : "+v"(fr), "+v"(sp));

        // 1. block sweeps (Section 3.1 / 4.1 recurrences, block factor);
        // each group of G rows reads its coefficients while the previous
        // group computes
        block_sweeps<KIND, T, LB, VEC, GF>(fr, x);
        // 2. the separator right-hand sides in two parts: the previous
        // separator takes minus its couplings to this block's first rows
        // (redr), the block's own separator takes f_sep minus its couplings to
        // this block's last interior rows (redl); one barrier.  (In this order
        // the first rows' values are dropped before the last rows' are used,
        // which keeps the FP64 pentadiagonal kernel within its registers.)
        if (has_prev) {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
#pragma unroll
                for (int c = 0; c < H; ++c) {
                    // band d = 2H - c + e of separator row c meets this block's row e
                    T yh = T(0);
#pragma unroll
                    for (int e = 0; e + 2 * H - c < NB; ++e) yh = fma(-cr[c][e], x[e][v], yh);
                    lredr[o_prev + v * ldr + c] = yh;
                }
        }
        if (has_sep) {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
#pragma unroll
                for (int c = 0; c < H; ++c) {
                    // separator rows are identity rows of the block factor: the
                    // sweeps leave their right-hand sides in place
                    T yh = x[NI + c][v];
                    // band d < H - c of separator row c meets row NI + c + d - H
#pragma unroll
                    for (int d = 0; d + c < H; ++d) yh = fma(-cl[c][d], x[NI + c + d - H][v], yh);
                    lredl[o_own + v * ldr + c] = yh;
                }
        }
        __syncthreads();
        // 3. separators
        T zr[H][VEC], zl[H][VEC];
        if (Nr == 0) {
#pragma unroll
            for (int c = 0; c < H; ++c)
#pragma unroll
                for (int v = 0; v < VEC; ++v) zr[c][v] = zl[c][v] = T(0);
        } else if (MMA && blockDim.x % kWave == 0 &&
                   (!alias || ((Nr + 15) / 16) * ((S + 15) / 16) <= (int)(blockDim.x / kWave))) {
            if constexpr (MMA) {
                // flags bit 6: every column of S^{-1}
                const int kw = (a.flags & 64) ? 0 : a.kw;
                if (alias)
                    sep_mma<true>(lsinv, lredl, lredr, lz, Nr, S, ldr, a.kofs, kw);
                else
                    sep_mma<false>(lsinv, lredl, lredr, lz, Nr, S, ldr, a.kofs, kw);
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < H; ++c)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    // indices stay inside the separators even where unused
                    const T zo = lz[(has_sep ? o_own : o_col) + v * ldr + c];
                    const T zp = lz[(has_prev ? o_prev : o_col) + v * ldr + c];
                    zr[c][v] = has_sep ? zo : T(0);
                    zl[c][v] = has_prev ? zp : T(0);
                }
            // the separators are redL's storage: the next group writes redL
            // only after every lane has read them
            if (alias) __syncthreads();
        } else {
            // rows of S^{-1} for the own and the previous separator (a block
            // without one reads the other's rows and discards the result)
            const T *rr = lsinv + (size_t)H * (has_sep ? p : pp) * Nr;
            const T *rl = lsinv + (size_t)H * (has_prev ? pp : p) * Nr;
            T ar[H][VEC], al[H][VEC];
#pragma unroll
            for (int c = 0; c < H; ++c)
#pragma unroll
                for (int v = 0; v < VEC; ++v) ar[c][v] = al[c][v] = T(0);
            for (int k = 0; k < Nr; ++k) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const T y = lredl[o_col + v * ldr + k] + lredr[o_col + v * ldr + k];
#pragma unroll
                    for (int c = 0; c < H; ++c) {
                        ar[c][v] = fma(rr[c * Nr + k], y, ar[c][v]);
                        al[c][v] = fma(rl[c * Nr + k], y, al[c][v]);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < H; ++c)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    zr[c][v] = has_sep ? ar[c][v] : T(0);
                    zl[c][v] = has_prev ? al[c][v] : T(0);
                }
            // every lane has read redL / redR before the next group writes them
            __syncthreads();
        }
        // 4. correction and stores
        T *dst = out + (int64_t)r0 * m + col(g);
        // the spikes of GC rows per round trip; from global memory (GF) the
        // next rows' spikes are loaded before the current rows are stored,
        // since a load issued after a store waits for that store
        constexpr int GC = GF ? 2 : G, NS = GF ? 2 : 1;
        T spt[NS][GC][2 * H];
        auto spikes = [&](int gr, T(&dstk)[GC][2 * H]) {
            if constexpr (GF) asm volatile("" : "+v"(sp));
#pragma unroll
            for (int u = 0; u < GC; ++u)
#pragma unroll
                for (int k = 0; k < 2 * H; ++k) dstk[u][k] = sp[(gr * GC + u) * 2 * H + k];
        };
        if constexpr (GF) spikes(0, spt[0]);
#pragma unroll
        for (int gr = 0; gr < LB / GC; ++gr) {
            T(&cur)[GC][2 * H] = spt[GF ? gr & 1 : 0];
            if constexpr (GF) {
                if (gr + 1 < LB / GC) spikes(gr + 1, spt[(gr + 1) & 1]);
            } else {
                spikes(gr, cur);
            }
#pragma unroll
            for (int u = 0; u < GC; ++u) {
                const int t = gr * GC + u;
                T v2[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    T val = x[t][v];
#pragma unroll
                    for (int c = 0; c < H; ++c) {
                        val = fma(-cur[u][c], zr[c][v], val);
                        val = fma(-cur[u][H + c], zl[c][v], val);
                    }
                    if (t >= NI) val = has_sep ? zr[t >= NI ? t - NI : 0][v] : val;
                    v2[v] = val;
                }
                if constexpr (CN) {
                    // computed here, not sunk past the barrier below (which
                    // would keep every row's spikes live until then)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        x[t][v] = v2[v];
                        asm volatile("" : "+v"(x[t][v]));
                    }
                } else if (full || r0 + t < n) {
                    store_vec_nt<T, VEC>(dst + (int64_t)t * m, v2);
                }
            }
            pin(zr[0][0]);
        }
        if constexpr (CN) {
            // 5. Crank-Nicolson output rows from the block's solution
#pragma unroll
            for (int v = 0; v < VEC; ++v)
#pragma unroll
                for (int c = 0; c < H; ++c) ltop[((s0 + v) * P + p) * H + c] = x[c][v];
            __syncthreads();
            const bool has_next = a.periodic || p < P - 1;
            const int pn = p == P - 1 ? 0 : p + 1;
            T dn[H][VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v)
#pragma unroll
                for (int c = 0; c < H; ++c) {
                    const T t0 = ltop[((s0 + v) * P + pn) * H + c];
                    dn[c][v] = has_next ? t0 : T(0);
                }
            // rows above the block: the previous block's separators (0 above
            // the first block of a matrix that does not wrap round)
            const T c0 = (T)a.coef.c[0];
            // one store pointer stepped row by row (opaque, so that the
            // rows' addresses are not all formed up front and kept live)
            T *q = dst;
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                T v2[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    T ax = T(0);
#pragma unroll
                    for (int e = 0; e < NB; ++e) {
                        const int i = t - H + e;
                        const T u = i < 0 ? zl[i + H][v] : (i >= LB ? dn[i - LB][v] : x[i][v]);
                        ax = e == 0 ? c0 * u : fma((T)a.coef.c[e], u, ax);
                    }
                    v2[v] = T(2) * x[t][v] - ax;
                }
                if (full || r0 + t < n) store_vec_nt<T, VEC>(q, v2);
                q += m;
                asm volatile("" : "+v"(q));
                if (t % G == G - 1) pin(v2[0]);
            }
        }
        if (g + grid < a.ngroups) load_group(g + grid);
    }
}

// ---------------------------------------------------------------------------
// Launch side.

// Threads a workgroup may have: the lane's LB * VEC values take
// LB * VEC * sizeof(T) / 4 registers, and a CU's register file holds 512 per
// lane of one wave per SIMD.
template <typename T, int LB, int VEC>
constexpr int sep_maxt() {
    return LB * VEC * (int)sizeof(T) / 4 <= 64 ? 1024 : 512;
}

template <int KIND, typename T, int LB, int VEC, bool GF, bool CN = false>
hipError_t sep_kernel(const void **fn) {
    auto kern = k_sep<KIND, T, LB, VEC, sep_maxt<T, LB, VEC>(), GF, CN>;
    // once per instantiation; thread-safe static initialisation, so that
    // concurrent first launches from several host threads do not race
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)kMaxPartLdsBytes);
    if (attr != hipSuccess) return attr;
    *fn = reinterpret_cast<const void *>(kern);
    return hipSuccess;
}

// The shapes built: (LB, VEC) with at most 128 registers of values per lane;
// with the plan in global memory (GF) the two longest, (32, 2) and (64, 1);
// Crank-Nicolson steps of pentadiagonal matrices (plan in LDS) (32, 1),
// (32, 2) and (64, 1).
template <int KIND, typename T>
hipError_t sep_kernel_of(int lb, int vec, bool gf, bool cn, const void **fn, int *maxt) {
    if (cn) {
        if constexpr (KIND == SBS_PENTA) {
            if (gf) return hipErrorInvalidValue;
            if (lb == 32 && vec == 1) return *maxt = sep_maxt<T, 32, 1>(), sep_kernel<KIND, T, 32, 1, false, true>(fn);
            if (lb == 32 && vec == 2) return *maxt = sep_maxt<T, 32, 2>(), sep_kernel<KIND, T, 32, 2, false, true>(fn);
            if (lb == 64 && vec == 1) return *maxt = sep_maxt<T, 64, 1>(), sep_kernel<KIND, T, 64, 1, false, true>(fn);
        }
        return hipErrorInvalidValue;
    }
    if (gf) {
        if (lb == 32 && vec == 2) return *maxt = sep_maxt<T, 32, 2>(), sep_kernel<KIND, T, 32, 2, true>(fn);
        if (lb == 64 && vec == 1) return *maxt = sep_maxt<T, 64, 1>(), sep_kernel<KIND, T, 64, 1, true>(fn);
        return hipErrorInvalidValue;
    }
    if (lb == 16 && vec == 1) return *maxt = sep_maxt<T, 16, 1>(), sep_kernel<KIND, T, 16, 1, false>(fn);
    if (lb == 16 && vec == 2) return *maxt = sep_maxt<T, 16, 2>(), sep_kernel<KIND, T, 16, 2, false>(fn);
    if (lb == 32 && vec == 1) return *maxt = sep_maxt<T, 32, 1>(), sep_kernel<KIND, T, 32, 1, false>(fn);
    if (lb == 32 && vec == 2) return *maxt = sep_maxt<T, 32, 2>(), sep_kernel<KIND, T, 32, 2, false>(fn);
    if (lb == 64 && vec == 1) return *maxt = sep_maxt<T, 64, 1>(), sep_kernel<KIND, T, 64, 1, false>(fn);
    if constexpr (sizeof(T) == 4)
        if (lb == 64 && vec == 2) return *maxt = sep_maxt<T, 64, 2>(), sep_kernel<KIND, T, 64, 2, false>(fn);
    return hipErrorInvalidValue;
}

hipError_t sep_fn(int kind, int tc, int lb, int vec, bool gf, bool cn, const void **fn, int *maxt) {
    const int k = kind == SBS_PENTA ? SBS_PENTA : SBS_TRI;  // periodic blocks are plain tridiagonal
    if (k == SBS_TRI)
        return tc == 0 ? sep_kernel_of<SBS_TRI, double>(lb, vec, gf, cn, fn, maxt)
                       : sep_kernel_of<SBS_TRI, float>(lb, vec, gf, cn, fn, maxt);
    return tc == 0 ? sep_kernel_of<SBS_PENTA, double>(lb, vec, gf, cn, fn, maxt)
                   : sep_kernel_of<SBS_PENTA, float>(lb, vec, gf, cn, fn, maxt);
}

// LDS of one workgroup: the plan (GF: S^{-1} only), the two parts of the
// separator right-hand sides and (FP64: the matrix-core product's output)
// the separators, unless `alias` puts them in redL's storage; Crank-Nicolson
// steps add the blocks' first rows after a third buffer.
// (cn_h: the half band width H of a Crank-Nicolson step, 0 for a solve)
size_t sep_lds(const SepPlan &sp, int tc, int S, bool gf, bool alias, int cn_h = 0) {
    const size_t elem = tc == 0 ? 8 : 4;
    const size_t red = tc == 0 ? sep_red_bytes<double>(S, sp.Nr) : sep_red_bytes<float>(S, sp.Nr);
    const size_t plan = gf ? (tc == 0 ? sp.sinv_bytes64 : sp.sinv_bytes32) : sp.blob_bytes(tc);
    if (cn_h) return plan + 3 * red + ((size_t)S * sp.P * cn_h * elem + 15) / 16 * 16;
    return plan + red * (tc == 0 && !alias ? 3 : 2);
}

int cu_count(int device) { return device_cus(device); }

// Checks one shape and fills in its launch figures; false if it cannot run.
// The plan goes to LDS whole where it fits with the group's buffers, else
// (or with flags bit 4) only S^{-1} does (GF), and where even that leaves no
// room for a third FP64 buffer the separators overwrite redL (flags bit 5,
// which only this function sets).
//
// cn: a Crank-Nicolson step of a matrix with constant bands (plan in LDS only).
bool sep_fit(const sbs_lhs *h, int tc, int64_t m, const void *x, int q, int vec, int S, int flags, SepChoice *c,
             bool cn = false) {
    const SepPlan &sp = h->sep[q];
    const size_t elem = tc == 0 ? 8 : 4;
    if (!sp.ok || m < vec || S < vec || S % vec) return false;
    if (vec == 2 && (m % 2 || reinterpret_cast<uintptr_t>(x) % (2 * elem))) return false;
    flags &= ~32;
    bool gf = (flags & 16) != 0, alias = false;
    if (cn && gf) return false;
    if (!cn && !gf && sep_lds(sp, tc, S, false, false) > kMaxPartLdsBytes) gf = true;
    if (!cn && gf && sep_lds(sp, tc, S, true, false) > kMaxPartLdsBytes) alias = tc == 0;
    const size_t lds = sep_lds(sp, tc, S, gf, alias, cn ? h->kind / 2 : 0);
    if (lds > kMaxPartLdsBytes) return false;
    const void *fn = nullptr;
    int maxt = 0;
    if (sep_fn(h->kind, tc, sp.lb, vec, gf, cn, &fn, &maxt) != hipSuccess) return false;
    const int threads = (S / vec) * sp.P;
    if (threads > maxt) return false;
    // the separators in redL: one matrix-core tile per wave
    if (alias && (threads % kWave || ((sp.Nr + 15) / 16) * ((S + 15) / 16) > threads / kWave)) return false;
    int wgs = 0;
    if ((wgs = occupancy(fn, threads, lds)) < 1) return false;
    c->plan = q;
    c->vec = vec;
    c->S = S;
    c->threads = threads;
    c->lds = lds;
    c->wgs = wgs;
    c->flags = flags | (gf ? 16 : 0) | (alias ? 32 : 0);
    c->gf = gf;
    c->cn = cn;
    return true;
}

}  // namespace

// Default launch options: groups in launch order.
constexpr int kSepDefaultFlags = 0;

bool choose_sep(const sbs_lhs *h, int tc, int64_t m, const void *x, SepChoice *out, bool cn) {
    const size_t elem = tc == 0 ? 8 : 4;
    const int cus = cu_count(h->device);
    SepChoice best;
    int64_t best_key[5] = {-1, -1, -1, -1, -1};
    for (int q = 2; q >= 0; --q)
        for (int vec = 2; vec >= 1; --vec)
            for (int S = 64; S >= 1; S /= 2) {
                SepChoice c;
                if (!sep_fit(h, tc, m, x, q, vec, S, kSepDefaultFlags, &c, cn)) continue;
                const int64_t groups = (m + S - 1) / S;
                const int64_t engaged = std::min<int64_t>(groups, (int64_t)cus * c.wgs);
                // CUs engaged, the plan held in LDS, rows read in whole
                // 256-byte runs, 16-byte accesses, then lanes at work (up to
                // 8 waves per CU)
                const int64_t run = std::min<int64_t>((int64_t)S * elem, 256);
                const int64_t acc = (int64_t)vec * elem;
                const int64_t lanes = std::min<int64_t>(engaged * c.threads, (int64_t)cus * 8 * kWave);
                const int64_t key[5] = {std::min<int64_t>(engaged, cus), c.gf ? 0 : 1, run, acc, lanes};
                if (std::lexicographical_compare(best_key, best_key + 5, key, key + 5)) {
                    std::copy(key, key + 5, best_key);
                    best = c;
                }
            }
    if (best.plan < 0) return false;
    *out = best;
    return true;
}

bool sep_fills(const sbs_lhs *h, int tc, int64_t m, const SepChoice &c) {
    const size_t elem = tc == 0 ? 8 : 4;
    const int64_t groups = (m + c.S - 1) / c.S;
    return (size_t)c.S * elem >= 256 && groups >= cu_count(h->device);
}

bool sep_shape(const sbs_lhs *h, int tc, int64_t m, const void *x, int lb, int vec, int S, int flags, SepChoice *out) {
    for (int q = 0; q < 3; ++q)
        if (kPartLbs[q] == lb) return sep_fit(h, tc, m, x, q, vec, S, flags, out);
    return false;
}

hipError_t launch_sep(const sbs_lhs *h, const SepChoice &c, int tc, void *x, int64_t m, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const SepPlan &sp = h->sep[c.plan];
    const void *fn = nullptr;
    int maxt = 0;
    if (hipError_t e = sep_fn(h->kind, tc, sp.lb, c.vec, c.gf, c.cn, &fn, &maxt); e != hipSuccess) return e;
    if (c.threads > maxt) return hipErrorInvalidValue;
    const int64_t ngroups = (m + c.S - 1) / c.S;
    if (ngroups > 0x7fffffff) return hipErrorInvalidValue;
    SepArgs a;
    const bool f64 = tc == 0;
    a.fac_bytes = (int)(f64 ? sp.fac_bytes64 : sp.fac_bytes32);
    a.spk_bytes = (int)(f64 ? sp.spk_bytes64 : sp.spk_bytes32);
    a.scf_bytes = (int)(f64 ? sp.scf_bytes64 : sp.scf_bytes32);
    a.sinv_bytes = (int)(f64 ? sp.sinv_bytes64 : sp.sinv_bytes32);
    a.map_bytes = (int)sp.map_bytes;
    a.n = (int)h->n;
    a.P = sp.P;
    a.Nr = sp.Nr;
    a.S = c.S;
    a.ngroups = (int)ngroups;
    a.periodic = sp.periodic ? 1 : 0;
    a.flags = c.flags;
    a.kofs = sp.kofs;
    a.kw = sp.kw;
    a.m = m;
    a.coef = h->coef;
    const int grid = (int)std::min<int64_t>(ngroups, (int64_t)cu_count(h->device) * std::max(1, c.wgs));
    const unsigned char *blob = static_cast<const unsigned char *>(f64 ? sp.blob64 : sp.blob32);
    void *args[] = {&blob, &a, &x, &x};
    return hipLaunchKernel(fn, dim3(grid), dim3(c.threads), args, c.lds, s);
}

}  // namespace sbs
