// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sbs.h"

namespace sbs {

// Factor rows, one per matrix row (32 B tri / 64 B penta in FP64).  The
// sweeps stage chunks of them through LDS and broadcast each row to the
// wave; the partitioned kernels copy a plan's rows into LDS once.
//
// Tridiagonal (Section 3.1): with den_i = b_i - a_i chat_{i-1},
//   forward   y_i = d_i / den_i - (a_i / den_i) y_{i-1}
//   backward  x_i = y_i - chat_i x_{i+1}
// so a row stores { a_i / den_i, chat_i, 1 / den_i }.
template <typename T>
struct alignas(4 * sizeof(T)) TriRow {
    T a_s, chat, inv, pad;
};

// Pentadiagonal (Section 4.1), A = L R:
//   forward   g_i = f_i / alpha_i - (eps_i / alpha_i) g_{i-2} - (beta_i / alpha_i) g_{i-1}
//   backward  x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2}
// so a row stores { eps_i / alpha_i, beta_i / alpha_i, 1 / alpha_i, gamma_i, delta_i }.
template <typename T>
struct alignas(8 * sizeof(T)) PentaRow {
    T eps_s, beta_s, inv, gamma, delta, p0, p1, p2;
};

// Periodic tridiagonal (Section 3.3), A = A' + u v^T with A' tridiagonal:
//   forward   y_i = d_i / den_i - (a_i / den_i) y_{i-1},  acc += wt_i d_i
//   backward  y_i = yhat_i - chat_i y_{i+1},  x_i = y_i - acc z_i
// where den / chat factor A', z = A'^{-1} u and wt = A'^{-T} v / (1 + v.z),
// so acc ends the forward sweep equal to (v.y) / (1 + v.z).
template <typename T>
struct alignas(8 * sizeof(T)) PeriodicRow {
    T a_s, chat, inv, wt, z, p0, p1, p2;
};

// Original coefficients of row i, for the FP64 residual b - A x:
// tri {a_i, b_i, c_i, 0}; penta {a_i, b_i, c_i, d_i, e_i, 0, 0, 0}.
// Coefficients outside the matrix are stored as 0.
struct alignas(64) BandRow {
    double c[8];
};

// The 2h+1 coefficients of a matrix whose bands are constant, passed to
// kernels by value.
struct BandCoef {
    double c[5];
};

constexpr int kWave = 64;       // lanes per wavefront on gfx950
constexpr int kRowPad = 64;     // factor rows are padded with zero rows to a multiple of this
                                // (every chunk length divides it, so chunks never read past the end)

}  // namespace sbs

namespace sbs {

// Block partition of the shared matrix (several lanes per system).
// Rows are cut into P blocks of lb rows (the last block padded with identity
// rows).  For block p: its own factor A_p, and the spikes V_p = A_p^{-1} B_p,
// W_p = A_p^{-1} C_p, where B_p / C_p hold the coefficients that couple the
// block to the first h unknowns of block p+1 / the last h unknowns of block
// p-1 (h = 1 tri, 2 penta).  With g_p = A_p^{-1} f_p every block's solution is
//   x_p = g_p - V_p x_{p+1}[0:h] - W_p x_{p-1}[lb-h:lb],
// and the 2h(P-1) interface unknowns (x_p bottom, x_{p+1} top for p < P-1)
// solve a small system R z = (g interface values) whose inverse is stored.
// Everything depends on the matrix only, so it is computed once, in FP64.
struct PartPlan {
    int lb = 0, P = 0, Nr = 0;
    int D = 0;  // distinct blocks stored (bit-identical blocks share one copy)
    bool ok = false;
    bool periodic = false;  // blocks wrap round: P interface pairs, not P-1
    // Device arrays, each [fac | spk | rinv | map] contiguous and 16-byte aligned:
    //   fac: D*lb factor rows of the distinct blocks (TriRow/PentaRow)
    //   spk: D*lb rows of {V[0..h), W[0..h)}
    //   rinv: Nr*Nr, row-major
    //   map: P ints, block p uses stored block map[p]
    void *blob64 = nullptr, *blob32 = nullptr;
    size_t fac_bytes64 = 0, spk_bytes64 = 0, rinv_bytes64 = 0;
    size_t fac_bytes32 = 0, spk_bytes32 = 0, rinv_bytes32 = 0;
    size_t map_bytes = 0;
    size_t blob_bytes(int tc) const {
        return (tc == 0 ? fac_bytes64 + spk_bytes64 + rinv_bytes64 : fac_bytes32 + spk_bytes32 + rinv_bytes32) +
               map_bytes;
    }
};
constexpr int kPartLbs[3] = {16, 32, 64};

// Separator partition of the shared matrix (several lanes per system, the
// form the plain partitioned solve runs).  Rows are cut into P blocks of lb
// rows; the last h rows of every block but the last (of every block when the
// matrix is periodic) are separator rows, the others interior rows.  With
// the separators z known, the interior rows of block p decouple:
//   x_I(p) = g_p - V_p z_p - W_p z_{p-1},   g_p = A_II(p)^{-1} f_I(p),
// V_p / W_p = A_II(p)^{-1} times the columns of its own / the previous
// separator.  Substituting into the separator rows gives the Schur
// complement system S z = yhat, yhat_p = f_sep(p) - (separator rows' couplings
// to the neighbouring interior rows) . g, with h(P-1) unknowns (hP periodic),
// half the interface of the pair form above.  Everything but g and yhat
// depends on the matrix only and is computed once, in FP64.
// The separator plan rearranged for the one-wave-per-block mixed-precision
// kernel (non-periodic plans of 32- and 64-row blocks): byte offsets from
// `base` of the forward coefficients, backward coefficients and spikes
// ([D][lb][..] FP32), of the original band rows ([P][lb][2h+1] FP64) and of
// S^{-1} ([Nr][ldsinv] FP32, rows padded with zeros to a multiple of 8).
struct RefinePlan {
    void *base = nullptr;
    size_t fwd = 0, bwd = 0, spk = 0, band = 0, sinv = 0;
    int ldsinv = 0;
};

struct SepPlan {
    int lb = 0, P = 0, Nr = 0;
    int D = 0;  // distinct blocks stored
    bool ok = false;
    bool periodic = false;
    // Device arrays, each [fac | spk | scf | sinv | map] contiguous, 16-byte aligned:
    //   fac: D*lb factor rows (interior factor; identity on separator rows)
    //   spk: D*lb rows of {V[0..h), W[0..h)} (0 on separator rows)
    //   scf: D*h rows of 2h+1 coefficients: band row of each separator row,
    //        0 on separator columns and outside the matrix
    //   sinv: Nr*Nr, row-major (inverse of S; entries that cannot matter
    //         are 0, and the product reads only the window kofs / kw)
    //   map: P ints
    void *blob64 = nullptr, *blob32 = nullptr;
    size_t fac_bytes64 = 0, spk_bytes64 = 0, scf_bytes64 = 0, sinv_bytes64 = 0;
    size_t fac_bytes32 = 0, spk_bytes32 = 0, scf_bytes32 = 0, sinv_bytes32 = 0;
    size_t map_bytes = 0;
    // 16-row tile t of S^{-1} has its nonzero entries in columns k0 .. k0 + kw - 1,
    // k0 = min(max(16t + kofs, 0), max(Nr4 - kw, 0)), Nr4 = Nr rounded up to 4;
    // kw = 0: every column
    int kofs = 0, kw = 0;
    RefinePlan refine;
    size_t blob_bytes(int tc) const {
        return (tc == 0 ? fac_bytes64 + spk_bytes64 + scf_bytes64 + sinv_bytes64
                        : fac_bytes32 + spk_bytes32 + scf_bytes32 + sinv_bytes32) +
               map_bytes;
    }
};

}  // namespace sbs

struct sbs_lhs {
    int32_t kind = 0;
    int64_t n = 0;
    int64_t rows = 0;           // n rounded up to kRowPad
    void *dev = nullptr;        // one allocation holding the three arrays below
    void *fac64 = nullptr;      // TriRow<double>[rows] or PentaRow<double>[rows]
    void *fac32 = nullptr;      // TriRow<float>[rows]  or PentaRow<float>[rows]
    sbs::BandRow *bands = nullptr;  // BandRow[rows]
    void *pdev = nullptr;       // partition data (one allocation for all plans)
    sbs::PartPlan part[3];      // block lengths 16, 32, 64
    sbs::SepPlan sep[3];        // block lengths 16, 32, 64
    // every band constant over the rows where it lies inside the matrix
    // (every row for a periodic matrix): the coefficients themselves
    bool constant_bands = false;
    sbs::BandCoef coef{};
    int64_t device_bytes = 0;
    int device = 0;
    uint64_t id = 0;  // unique per handle in the process (keys the host's cached launch choices)
};

namespace sbs {

// Host-side launch figures, queried from the runtime once and then kept
// (every solve chooses its shape, and the queries cost microseconds each):
// compute units of a device, and workgroups of kernel `fn` resident per CU
// at `threads` threads and `lds` bytes of dynamic LDS on the current device
// (0 if the runtime reports an error).
int device_cus(int device);
int occupancy(const void *fn, int threads, size_t lds);

struct SweepArgs {
    const sbs_lhs *h;
    const void *in;
    void *out;
    int64_t m;
    hipStream_t stream;
};

// Plain solve (in == out allowed).  tin/tout/tc: 0 = f64, 1 = f32.
hipError_t launch_sweep(const sbs_lhs *h, int variant, int tc, int tin, int tout,
                        const void *in, void *out, int64_t m, hipStream_t stream);

// Residual / update kernels of the mixed-precision driver.
//  mode 0: r = fl32(b - A x)
//  mode 1: x += delta; r = fl32(b - A x)
//  mode 2: x += delta
hipError_t launch_refine_step(const sbs_lhs *h, int mode, const float *b, double *x,
                              const float *delta, float *r, int64_t m, hipStream_t stream);

hipError_t launch_transpose(const void *src, void *dst, int64_t rows, int64_t cols,
                            int elem_bytes, hipStream_t stream);

// One Crank-Nicolson step in place: c <- A^{-1} (2I - A) c (tc: 0 f64, 1 f32).
hipError_t launch_cn(const sbs_lhs *h, int tc, void *c, int64_t m, hipStream_t stream);

// Which variant AUTO picks, and the LDS bytes per wave the chunked variant
// needs (tc: 0 = f64, 1 = f32).
int choose_variant(const sbs_lhs *h, int tc);
size_t chunked_lds_bytes(const sbs_lhs *h, int tc);
constexpr size_t kMaxLdsBytes = 160 * 1024;       // LDS budget of the chunked variant (one wave)
constexpr size_t kMaxPartLdsBytes = 160 * 1024;   // LDS one workgroup may allocate on gfx950

// Partitioned solve (SBS_VARIANT_PARTITION): choose a plan and systems per
// workgroup for m systems; returns false if no plan fits.
struct PartChoice {
    int plan = -1, S = 0, threads = 0;
    size_t lds = 0;
    int wgs = 1;  // workgroups resident per CU at this size
};
// cn: 0 a solve; 1 a Crank-Nicolson step c <- A^{-1} (2I - A) c (in == out)
// with the band rows staged in LDS; 2 the same for a matrix with constant
// bands (coefficients passed by value, nothing staged).
// rows: the systems are rows of a row-major grid (launch_partition_rows).
bool choose_partition(const sbs_lhs *h, int tc, int64_t m, PartChoice *out, int cn = 0, bool rows = false);
// A given pair-partition shape for a plain solve (block length lb, S).
bool part_shape(const sbs_lhs *h, int tc, int64_t m, int lb, int S, PartChoice *out);
hipError_t launch_partition(const sbs_lhs *h, const PartChoice &c, int tc, int tin, int tout, const void *in,
                            void *out, int64_t m, hipStream_t stream, int cn = 0);
// FP64 solve of m systems stored one after another (system j at x + j*n),
// in place, on the partition chosen for them.
hipError_t launch_partition_rows(const sbs_lhs *h, const PartChoice &c, double *x, int64_t m, hipStream_t stream);
sbs_status build_partitions(sbs_lhs *h, const double *bands);
bool choose_partition_refine(const sbs_lhs *h, int64_t m, PartChoice *out);
hipError_t launch_partition_refine(const sbs_lhs *h, const PartChoice &c, const float *b, double *x, int64_t m,
                                   int sweeps, hipStream_t stream);

// Mixed-precision solve on a separator plan, one wave per block and 64
// systems per group (coefficients wave-uniform, through scalar loads).
struct RefwChoice {
    int plan = -1;
    size_t lds = 0;
};
bool choose_refine_wave(const sbs_lhs *h, int64_t m, RefwChoice *out);
hipError_t launch_refine_wave(const sbs_lhs *h, const RefwChoice &c, const float *b, double *x, int64_t m,
                              int sweeps, hipStream_t stream);

// Separator-partitioned solve (plain solves of interleaved right-hand sides):
// plan, values per lane (VEC adjacent systems, one access per row), systems
// per workgroup, launch options (bit 0: XCD-grouped group order, bit 2:
// workgroups start out of step by bits 8.. sleeps of 4096 cycles per quarter,
// bit 4: plan in global memory, bit 5: separators overwrite redL).
struct SepChoice {
    int plan = -1, vec = 1, S = 0, threads = 0, flags = 0;
    bool gf = false;  // plan read from global memory, S^{-1} alone in LDS
    bool cn = false;  // a Crank-Nicolson step (constant bands) instead of a solve
    size_t lds = 0;
    int wgs = 1;  // workgroups resident per CU at this size
};
// The shape AUTO runs for m systems at x (the alignment of x decides whether
// pairs of systems can move as one access); false if no plan fits.
// cn: shapes for a Crank-Nicolson step of a matrix with constant bands.
bool choose_sep(const sbs_lhs *h, int tc, int64_t m, const void *x, SepChoice *out, bool cn = false);
// A given shape (block length lb, VEC, S, flags); false if it cannot run.
bool sep_shape(const sbs_lhs *h, int tc, int64_t m, const void *x, int lb, int vec, int S, int flags, SepChoice *out);
// In place on the interleaved (n, m) array x (tc: 0 f64, 1 f32).
hipError_t launch_sep(const sbs_lhs *h, const SepChoice &c, int tc, void *x, int64_t m, hipStream_t stream);
// Whether the separator shape fills the GPU with whole 256-byte row runs.
bool sep_fills(const sbs_lhs *h, int tc, int64_t m, const SepChoice &c);

// Mixed-precision solve (sbs_solve_batch_refined): argument checks, whether
// the fused kernel serves m systems (then no scratch is used), and the run
// itself with r, the FP32 residual scratch of n*m floats (unused when fused).
sbs_status refined_check(const sbs_lhs *h, const float *b, const double *x, int64_t m, int32_t sweeps);
bool refined_fused(const sbs_lhs *h, int64_t m);
sbs_status refined_run(const sbs_lhs *h, const float *b, double *x, int64_t m, int32_t sweeps, float *r,
                       hipStream_t s);

// Serving: heterogeneous tile launches (see server.cpp).
struct Tile {
    const void *fac;            // factor rows of this tile's matrix (FP32 for prec 1, else FP64)
    const BandRow *bands;       // original bands (mixed precision only)
    const void *in;             // rhs of the request
    double *x;                  // FP64 result of the request
    float *scratch;             // FP32 residual scratch (mixed precision only)
    int64_t n, m, col0;         // system range [col0, col0 + 64) of the request
    // prec 0: FP64 request; 1: FP32 request, mixed precision with two
    // corrections; 2: FP32 request, one FP64 sweep of its stored values
    int32_t kind, prec;
    int32_t req;                // the request's slot in the launch's completion arrays
    int32_t pad;
};

// Runs tiles [0, ntiles), all of one kind and prec, with `grid`
// persistent waves; *dev_counter must be 0 when the kernel starts.
// Per-request completion: left[r] holds the number of tiles of request r
// (device memory); the wave that finishes the last of them sets done[r] = 1
// (host-visible memory), after every result of the request is visible to the
// host and to other work on the device.
hipError_t launch_tiles(int kind, int prec, const Tile *dev_tiles, int ntiles, int *dev_counter, int *left,
                        int *done, int grid, hipStream_t stream);

}  // namespace sbs
