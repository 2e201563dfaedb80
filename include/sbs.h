/*
 * sbs.h -- batched solves of many right-hand sides against ONE shared
 * tridiagonal or pentadiagonal matrix, on an AMD Instinct MI355X (gfx950).
 *
 * Method: Gloster, Carroll, Bustamante, O Naraigh, "Efficient Interleaved
 * Batch Matrix Solvers for CUDA" (arXiv:1909.04539).  One copy of the
 * factored left-hand side is shared by every system (Section 2); the
 * right-hand sides are interleaved so that unknown i of system j lives at
 * element i*m + j (Section 2, and the storage paragraphs closing Sections
 * 3.1 and 4.1); each GPU lane runs one system's forward sweep and backward
 * sweep (Section 2): the Thomas recurrences of Section 3.1 for tridiagonal
 * matrices and the L R recurrences of Section 4.1 for pentadiagonal ones.
 *
 * Conventions for every call:
 *  - Every function returns an sbs_status; no exception or abort crosses the
 *    ABI.  Argument errors are detected before any device work is queued.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device memory of the current device.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Solves are queued asynchronously on it; a failed launch returns
 *    SBS_ERR_DEVICE, faults inside kernels surface at the next synchronisation.
 *  - A handle is immutable after it is created, so any number of solves may
 *    use it concurrently on any streams.  It must outlive every solve queued
 *    with it (release it after synchronising).
 *  - Every call is thread-safe except that a handle must not be released
 *    while another thread still uses it.
 */
#ifndef SBS_H
#define SBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sbs_status {
    SBS_OK = 0,
    SBS_ERR_INVALID_ARG = 1, /* bad kind/dtype/size, null pointer, unknown id  */
    SBS_ERR_ZERO_PIVOT = 2,  /* a factor pivot is zero or not finite          */
    SBS_ERR_NONFINITE = 3,   /* a matrix coefficient is NaN or infinite        */
    SBS_ERR_DEVICE = 4,      /* a HIP call failed (no device, launch failure)  */
    SBS_ERR_NO_MEMORY = 5,   /* device or host allocation failed               */
    SBS_ERR_BUDGET = 6,      /* request larger than the server's whole budget  */
    SBS_ERR_NOT_FOUND = 7,   /* unknown ticket                                 */
    SBS_ERR_TIMEOUT = 8,     /* wait timed out; the request is still pending   */
    SBS_ERR_SHUTDOWN = 9     /* server is shutting down                        */
} sbs_status;

typedef enum sbs_kind {
    SBS_TRI = 3,           /* tridiagonal                                   */
    SBS_PENTA = 5,         /* pentadiagonal                                 */
    SBS_TRI_PERIODIC = 13  /* tridiagonal with periodic wrap (three bands)  */
} sbs_kind;
typedef enum sbs_dtype { SBS_F64 = 0, SBS_F32 = 1 } sbs_dtype;

/* Sweep variants (all compute the same recurrences; they differ only in how
 * a lane keeps its column between the forward and the backward sweep). */
typedef enum sbs_variant {
    SBS_VARIANT_AUTO = 0,     /* chosen from n and dtype                      */
    SBS_VARIANT_RESIDENT = 1, /* whole column in registers (n <= 64)          */
    SBS_VARIANT_CHUNKED = 2,  /* checkpoint every chunk, recompute backwards  */
    SBS_VARIANT_STREAM = 3,   /* forward result written over the rhs, re-read */
    SBS_VARIANT_PARTITION = 4 /* each system's rows split over several lanes:  */
                              /* block solves, shared spikes, interface solve */
} sbs_variant;

typedef struct sbs_lhs *sbs_handle;

/* Human-readable name of a status code (static storage, never NULL). */
const char *sbs_status_str(sbs_status s);

/* Library version string (static storage). */
const char *sbs_version(void);

/*
 * Factor the shared matrix once, in FP64, on the host, and upload the factor.
 * Sections 3.1 (tridiagonal pre-factorisation: chat_i and the denominators
 * b_i - a_i chat_{i-1}) and 4.1 (pentadiagonal A = L R: alpha, beta, gamma,
 * delta, epsilon).  The paper performs this step on the CPU (Section 2).
 *
 *  kind     SBS_TRI, SBS_PENTA or SBS_TRI_PERIODIC.
 *  n        number of unknowns per system, 1 <= n <= INT32_MAX (n >= 3 for
 *           SBS_TRI_PERIODIC).
 *  bands    host, kind*n doubles, band-major and row-aligned: band k, entry i
 *           is the coefficient in row i.  Tridiagonal row i reads
 *           a_i x_{i-1} + b_i x_i + c_i x_{i+1}  (bands a, b, c);
 *           pentadiagonal row i reads a_i x_{i-2} + b_i x_{i-1} + c_i x_i
 *           + d_i x_{i+1} + e_i x_{i+2}  (bands a, b, c, d, e).
 *           Entries outside the matrix (tri a_0, c_{n-1}; penta a_0, a_1, b_0,
 *           d_{n-1}, e_{n-2}, e_{n-1}) are ignored.  The array is copied; the
 *           caller keeps ownership.
 *           SBS_TRI_PERIODIC (Section 3.3) takes the three tridiagonal bands
 *           with the wrap: row i reads a_i x_{(i-1) mod n} + b_i x_i
 *           + c_i x_{(i+1) mod n}, so a_0 and c_{n-1} are the corner
 *           entries.  It is factored by Sherman-Morrison: A = A' + u v^T with
 *           u = (-b_0, 0, .., 0, c_{n-1}), v = (1, 0, .., 0, -a_0/b_0) and A'
 *           tridiagonal (A'_00 = 2 b_0, A'_{n-1,n-1} = b_{n-1}
 *           + a_0 c_{n-1} / b_0, no corners).  z = A'^{-1} u and
 *           w = A'^{-T} v / (1 + v.z) are computed here, so that each solve
 *           is x = y - (w.d) z with y = A'^{-1} d, in the same two sweeps.
 *           Periodic handles take the plain solves (every variant, FP64
 *           or FP32; the partitioned variant solves the periodic system
 *           directly when n is a whole number of blocks), Crank-Nicolson
 *           steps and the ADI step; the refined solve and the serving loop
 *           reject them with SBS_ERR_INVALID_ARG.
 *  out      receives the new handle (owned by the caller; free with
 *           sbs_release).  Set to NULL on every error.
 *  bad_row  optional (may be NULL): on SBS_ERR_ZERO_PIVOT or
 *           SBS_ERR_NONFINITE the 0-based offending row, else -1.  For
 *           SBS_TRI_PERIODIC, bad_row == n means 1 + v.z is zero or not
 *           finite (the rank-one correction fails).
 * There is no pivoting (the paper has none): a zero or non-finite pivot is
 * reported as SBS_ERR_ZERO_PIVOT.  Diagonally dominant and symmetric
 * positive definite matrices never produce one.
 * Errors: SBS_ERR_INVALID_ARG (kind, n < 1, n > INT32_MAX or periodic
 *         n < 3, NULL bands/out),
 *         SBS_ERR_NONFINITE, SBS_ERR_ZERO_PIVOT, SBS_ERR_NO_MEMORY,
 *         SBS_ERR_DEVICE.
 */
sbs_status sbs_factor_shared_lhs(int32_t kind, int64_t n, const double *bands,
                                 sbs_handle *out, int64_t *bad_row);

/*
 * As sbs_factor_shared_lhs for a matrix with constant bands (the uniform
 * variant described at the close of Section 4.1 and measured in Section
 * 4.3): coeffs holds one value per band, in band order
 * (tri a, b, c; penta a, b, c, d, e).  The ends are truncated as for banded
 * kinds; SBS_TRI_PERIODIC wraps round.  The result is the handle the general
 * call gives for the expanded bands (same solutions bit for bit); with
 * constant bands every interior block of the partitioned variant is the
 * same, so its plan keeps three blocks whatever n is.
 * Errors: as sbs_factor_shared_lhs (NULL coeffs is SBS_ERR_INVALID_ARG).
 */
sbs_status sbs_factor_uniform(int32_t kind, int64_t n, const double *coeffs,
                              sbs_handle *out, int64_t *bad_row);

/*
 * Solve m systems in place: forward sweep then backward sweep per system
 * (Section 3.1 for SBS_TRI, Section 4.1 for SBS_PENTA), one GPU lane per
 * system, the shared factor read by all lanes (Section 2).
 *
 *  rhs    device, n*m elements of `dtype`, interleaved: element i*m + j is
 *         unknown i of system j.  Overwritten with the solution.
 *  m      number of systems, m >= 0 (m == 0 queues nothing and returns OK).
 *  dtype  SBS_F64 (FP64 throughout) or SBS_F32 (FP32 storage and FP32
 *         arithmetic with the FP32 rounding of the FP64 factor).
 * Errors: SBS_ERR_INVALID_ARG (NULL handle/rhs with m > 0, m < 0, dtype),
 *         SBS_ERR_DEVICE.
 */
sbs_status sbs_solve_batch(sbs_handle h, void *rhs, int64_t m, int32_t dtype,
                           void *stream);

/* As sbs_solve_batch with an explicit sweep variant (SBS_VARIANT_*).  The
 * resident variant needs n <= 64, the partitioned variant a matrix whose
 * blocks and interface system factor without a zero pivot and fit in LDS
 * (n up to a few thousand); otherwise SBS_ERR_INVALID_ARG.
 * The partitioned variant is not in the paper: it cuts every system's rows
 * into blocks solved by different lanes and couples them through the
 * partition ("spike") form of the same banded system; the couplings depend on
 * the matrix only, so they are computed once with the factor. */
sbs_status sbs_solve_batch_variant(sbs_handle h, void *rhs, int64_t m,
                                   int32_t dtype, int32_t variant, void *stream);

/*
 * The partitioned variant with an explicit shape (tests check every shape
 * against the oracle; benchmarks compare shapes).  Two forms:
 *  form 0  pair form: each block's first and last h unknowns are the
 *          interface (2h per block boundary); lb in {16, 32, 64}, S systems
 *          per workgroup, vec = 1, flags = 0.
 *  form 1  separator form: the last h rows of each block are separator rows,
 *          solved through the Schur complement of the interior rows (h per
 *          block boundary); lb in {16, 32, 64}, vec 1 or 2 adjacent systems
 *          per lane (2: one 16-byte FP64 access per row; needs m even and
 *          rhs aligned to 2 elements), S systems per workgroup (a multiple
 *          of vec), flags bit 0: workgroups of one chiplet take adjacent
 *          groups, bit 2: workgroups start out of step, workgroup b waiting
 *          (b % 4) * k * 4096 cycles first, with k in bits 8..15, bit 4:
 *          read the plan's factor rows, spikes and separator rows from
 *          global memory with only S^{-1} in LDS (taken anyway where the
 *          whole plan does not fit the LDS; shapes (lb, vec) = (32, 2) and
 *          (64, 1) only).  Bit 5 is ignored.  Bit 6: the FP64 product
 *          with S^{-1} over every column; by default each 16-row tile of
 *          S^{-1} reads only the columns that hold its nonzero entries (the
 *          plan sets entries of at most 2^-60 / Nr of their row's largest to
 *          0), which gives the same result bit for bit.
 * Same arguments and results as sbs_solve_batch otherwise.  A shape that has
 * no plan, exceeds 1024 threads, the register budget or the LDS returns
 * SBS_ERR_INVALID_ARG.
 */
sbs_status sbs_solve_batch_partition(sbs_handle h, void *rhs, int64_t m,
                                     int32_t dtype, int32_t form, int32_t lb,
                                     int32_t vec, int32_t S, int32_t flags,
                                     void *stream);

/* The partitioned shape AUTO runs for m systems of this dtype at rhs (host
 * only, rhs is not read: its alignment decides vec).  Returns
 * SBS_ERR_NOT_FOUND (outputs 0) if AUTO runs the sweeps. */
sbs_status sbs_partition_shape(sbs_handle h, int64_t m, int32_t dtype,
                               const void *rhs, int32_t *form, int32_t *lb,
                               int32_t *vec, int32_t *S);

/* The variant SBS_VARIANT_AUTO runs for m systems of this dtype: the
 * partitioned variant when a plan exists and fits, otherwise resident
 * (n <= 64), chunked (checkpoints fit 160 KiB of LDS) or stream.  Host only,
 * no device work.  Errors: SBS_ERR_INVALID_ARG (NULL handle or output,
 * m < 1, dtype). */
sbs_status sbs_auto_variant(sbs_handle h, int64_t m, int32_t dtype,
                            int32_t *variant);

/*
 * Mixed precision: FP32 right-hand sides, FP64 solution.
 * x0 = FP32 solve of b; then `sweeps` times: r = b - A x in FP64 with the
 * original FP64 bands, delta = FP32 solve of fl32(r), x += delta in FP64.
 * The FP32 solves use the FP32 rounding of the FP64 factor.  When the
 * matrix has a partition plan (see SBS_VARIANT_PARTITION) all passes run in
 * one kernel that keeps each system's b and x on chip, so b is read once and
 * x written once; `work` is then not touched.  That kernel holds 64 systems
 * per workgroup with one wave per block of rows where the separator plan
 * allows (at most 16 blocks of 32 rows or 8 of 64, and b of the 64 systems
 * within the LDS: n up to about 560), else the pair-form plan's kernel.
 *
 *  b          device, n*m floats, interleaved, read only.
 *  x          device, n*m doubles, interleaved, written (may not alias b).
 *  sweeps     number of corrections, 0..8 (2 is the usual choice).
 *  work       device scratch of at least sbs_refined_workspace_bytes(h, m)
 *             bytes (caller-owned; contents on return are unspecified).
 * Errors: SBS_ERR_INVALID_ARG (also for an SBS_TRI_PERIODIC handle),
 *         SBS_ERR_DEVICE.
 */
sbs_status sbs_solve_batch_refined(sbs_handle h, const float *b, double *x,
                                   int64_t m, int32_t sweeps, void *work,
                                   size_t work_bytes, void *stream);

/* Bytes of device scratch sbs_solve_batch_refined needs for m systems
 * (0 for an invalid handle). */
size_t sbs_refined_workspace_bytes(sbs_handle h, int64_t m);

/*
 * sbs_solve_batch_refined without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * sbs_solve_batch_refined, except that the FP32 residual scratch is a
 * library-owned device array of sbs_refined_static_scratch_bytes() bytes
 * (64 MiB) per GPU, held from the library's load until the process ends.
 * Its device address is looked up on the first call on each device (that
 * device must be current); the call itself allocates nothing.
 *  - Systems that the fused kernel serves (a partition plan exists) use no
 *    scratch and have no size limit.
 *  - Otherwise sbs_refined_workspace_bytes(h, m) must not exceed the array:
 *    larger requests return SBS_ERR_INVALID_ARG before any work is queued.
 *  - Every call on one GPU shares that GPU's array.  Calls that overlap on
 *    one GPU (different streams or host threads without ordering between
 *    them) race on it and give wrong results; calls queued on one stream are
 *    ordered and safe.  The array keeps the last call's contents; each call
 *    writes all of the scratch it reads before reading it.
 * Errors: as sbs_solve_batch_refined, plus SBS_ERR_INVALID_ARG for a
 *         request beyond the scratch size and SBS_ERR_DEVICE if the array's
 *         address cannot be found.
 */
sbs_status sbs_solve_batch_refined_noalloc(sbs_handle h, const float *b,
                                           double *x, int64_t m,
                                           int32_t sweeps, void *stream);

/* Bytes of the library's static scratch array (per GPU). */
size_t sbs_refined_static_scratch_bytes(void);

/*
 * Crank-Nicolson time steps in place (Sections 3.2 and 4.2): `steps` times
 *   A c' = (2I - A) c,
 * the scheme of both benchmark problems (the explicit half of diffusion,
 * s C_{i-1} + (1 - 2s) C_i + s C_{i+1}, and of hyperdiffusion, is 2I - A for
 * their matrices A), with the explicit half taken from the handle's own rows,
 * periodic rows wrapping round.  The explicit half is fused into the solve:
 * each step reads and writes every unknown as one solve does.
 *  c      device, interleaved (n, m), dtype SBS_F64 or SBS_F32; overwritten.
 *  steps  >= 0 (0 and m == 0 do nothing).
 * Any kind of handle.  Asynchronous on `stream`.
 * Errors: SBS_ERR_INVALID_ARG, SBS_ERR_DEVICE.
 */
sbs_status sbs_cn_step(sbs_handle h, void *c, int64_t m, int32_t dtype,
                       int32_t steps, void *stream);

/*
 * Out-of-place transpose: dst[c*rows + r] = src[r*cols + c].  Bit-exact
 * copy of 8-byte (SBS_F64) or 4-byte (SBS_F32) elements.  Converts a
 * row-major grid into the interleaved layout of its other direction.
 * src and dst are device buffers of rows*cols elements and must not overlap.
 */
sbs_status sbs_transpose(const void *src, void *dst, int64_t rows,
                         int64_t cols, int32_t dtype, void *stream);

/*
 * One alternating-direction step on a row-major FP64 grid g[y*nx + x]:
 * solve along y with hy (n == ny; the columns are already interleaved with
 * m = nx), then along x with hx (n == nx, m = ny).  The x systems are the
 * grid's rows: when hx has a partition plan they are solved in place, each
 * lane reading its block of a row as one contiguous run, and `work` is not
 * touched; otherwise the grid is transposed into `work`, solved there and
 * transposed back (the route of the paper's layout).  Either handle may be
 * of any kind (periodic handles give periodic directions).
 *  grid  device, ny*nx doubles, overwritten.
 *  work  device scratch, ny*nx doubles (caller-owned; required even when
 *        the in-place route leaves it untouched).
 */
sbs_status sbs_adi_step(sbs_handle hy, sbs_handle hx, double *grid,
                        double *work, int64_t ny, int64_t nx, void *stream);

/* Release a handle and its device memory.  NULL is accepted (no-op). */
sbs_status sbs_release(sbs_handle h);

/*
 * Query a handle.  Any output pointer may be NULL.  device_bytes is the
 * device memory the handle owns: O(kind * n), independent of how many
 * systems are later solved with it (the storage argument of Sections 3.1
 * and 4.1).
 */
sbs_status sbs_handle_info(sbs_handle h, int32_t *kind, int64_t *n,
                           int64_t *device_bytes);

/* ---------------------------------------------------------------------------
 * Serving: a request loop over registered shared matrices.
 *
 * The server owns a device arena of `budget_bytes`.  Each request reserves
 * its result buffer (n*m doubles) plus its scratch in the arena when it is
 * admitted, in arrival order, as soon as the bytes are free; a request
 * larger than the whole budget is rejected with SBS_ERR_BUDGET.  Admitted
 * requests are coalesced into shared launches (many requests, any n and m,
 * one kernel) that run on several streams at once, so requests that arrive
 * while others run are admitted and overlap them on the device.
 * FP64 requests get the plain FP64 solve; FP32 requests get the mixed
 * precision solve with 2 corrections (or, after sbs_server_set_fp32_mode,
 * one FP64 sweep of their stored values).  Either way the result is FP64.
 */
typedef struct sbs_server sbs_server;

typedef struct sbs_server_stats {
    uint64_t submitted, completed, rejected, launches;
    uint64_t queued;           /* waiting for admission now                 */
    uint64_t in_flight;        /* admitted, not yet complete                */
    uint64_t bytes_reserved;   /* arena bytes held by admitted requests     */
    uint64_t budget_bytes;
    double p50_us, p99_us, max_us; /* submit -> completion latency so far   */
    double unknowns;           /* sum of n*m over completed requests        */
} sbs_server_stats;

/* max_streams: concurrent launch streams (1..16; 0 = default 4).
 * max_batch_requests: cap on requests coalesced into one launch (0 = 4096). */
sbs_status sbs_server_create(size_t budget_bytes, int32_t max_streams,
                             int32_t max_batch_requests, sbs_server **out);

/* Register a factored matrix; the server keeps a reference, the caller still
 * owns the handle and must keep it alive until sbs_server_destroy.
 * SBS_TRI and SBS_PENTA handles only (SBS_ERR_INVALID_ARG otherwise). */
sbs_status sbs_server_register(sbs_server *srv, sbs_handle h, int32_t *lhs_id);

/* How FP32 requests submitted after this call are solved (requests already
 * submitted keep theirs):
 *  SBS_SERVE_F32_REFINED     (default) the mixed-precision form of
 *                            sbs_solve_batch_refined with 2 corrections:
 *                            FP32 sweeps, FP64 residuals and accumulation;
 *                            each tile's passes go through HBM (about 84
 *                            bytes per unknown, more for systems too long
 *                            for checkpoints) and the arena holds three
 *                            FP32 scratch arrays (12 bytes per unknown)
 *                            besides x.
 *  SBS_SERVE_F32_FP64_SWEEP  one FP64 sweep of the FP32 values (read and
 *                            promoted as they are loaded): the FP64 solve of
 *                            the stored right-hand sides, which is what the
 *                            refined form converges to, at 16 bytes per
 *                            unknown (28 for systems too long for
 *                            checkpoints) and with no scratch.
 * Errors: SBS_ERR_INVALID_ARG for any other mode. */
#define SBS_SERVE_F32_REFINED 0
#define SBS_SERVE_F32_FP64_SWEEP 1
sbs_status sbs_server_set_fp32_mode(sbs_server *srv, int32_t mode);

/* Queue a request.  rhs: device, n*m elements of dtype (interleaved),
 * read-only, must stay valid until the request completes.  Returns at once
 * with a ticket.  Errors: SBS_ERR_INVALID_ARG, SBS_ERR_BUDGET,
 * SBS_ERR_SHUTDOWN. */
sbs_status sbs_server_submit(sbs_server *srv, int32_t lhs_id, const void *rhs,
                             int64_t m, int32_t dtype, uint64_t *ticket);

/* Wait up to timeout_us (< 0: forever) for a request.  On completion
 * *x_device points at its FP64 solution (n*m doubles, interleaved) inside
 * the arena; it stays valid until sbs_server_release(ticket).  *latency_us
 * (optional) is submit -> completion.  Returns SBS_ERR_TIMEOUT if still
 * pending, SBS_ERR_NOT_FOUND for an unknown ticket. */
sbs_status sbs_server_wait(sbs_server *srv, uint64_t ticket, int64_t timeout_us,
                           const double **x_device, double *latency_us);

/* Copy a completed request's FP64 solution (n*m doubles) to the device
 * buffer dst, asynchronously on `stream`; the request must not be released
 * before that copy has finished. */
sbs_status sbs_server_fetch(sbs_server *srv, uint64_t ticket, double *dst, void *stream);

/* Give a completed request's arena bytes back (admits waiting requests). */
sbs_status sbs_server_release(sbs_server *srv, uint64_t ticket);

sbs_status sbs_server_stats_get(sbs_server *srv, sbs_server_stats *out);

/* Replay a trace of requests against the server from native threads (a
 * load generator with no interpreter in the loop).  Request k (matrix
 * lhs_ids[k], right-hand sides rhs[k] of m[k] systems in dtype[k], as for
 * sbs_server_submit) is submitted arrival_us[k] microseconds after the call
 * starts (arrival_us NULL: all at once, a closed loop); a second thread
 * waits for each request in order and releases it at once (the results are
 * not kept).  latency_us (optional, count doubles) receives each request's
 * submit -> completion latency, -1 for a request that was not accepted;
 * *elapsed_s (optional) the time from the start to the last release.
 * Returns the first error of any submission, wait or release (the other
 * requests still run), else SBS_OK.  All arrays are host memory owned by
 * the caller; the right-hand sides must stay valid until the call returns. */
sbs_status sbs_server_replay(sbs_server *srv, int64_t count, const int32_t *lhs_ids,
                             const void *const *rhs, const int64_t *m,
                             const int32_t *dtype, const double *arrival_us,
                             double *latency_us, double *elapsed_s);

/* Drain all work, then free the arena and the server. */
sbs_status sbs_server_destroy(sbs_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SBS_H */
