// Runs the partitioned solve on the host from the FP64 plan that
// build_partitions serialises (the CPU stand-in for the device keeps the
// uploaded blob in host memory), step for step as the kernel does: per block
// p the factor and spikes of stored block map[p], the block solve, the
// interface unknowns from rows of the stored inverse, the correction.
//   part_emulate in.bin out.bin
// in:  int32 kind, int64 n, int64 m, bands (3 or 5 x n doubles), rhs (n x m)
// out: per block length 16, 32, 64: int32 lb (0 if no plan), P, D, Nr, then
//      the n x m solution (only when the plan exists); first for the pair
//      plans, then for the separator plans (whose header is followed, when
//      the plan exists, by int32 kofs, kw: the window of the S^{-1}
//      product); then, for block lengths 32 and
//      64, the mixed-precision form run from the separator plan's copy for
//      the one-wave-per-block kernel (the right-hand sides rounded to FP32,
//      two correction rounds): int32 lb (0 if there is no copy), then x
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "factor_rows.h"
#include "internal.h"

using namespace sbs;

template <typename Row, typename Solve>
void emulate(const sbs_lhs &h, const PartPlan &pp, const double *rhs, int64_t m, double *x, Solve solve) {
    const int H = h.kind == SBS_PENTA ? 2 : 1, lb = pp.lb, P = pp.P, Nr = pp.Nr;
    const unsigned char *blob = static_cast<const unsigned char *>(pp.blob64);
    const Row *fac = reinterpret_cast<const Row *>(blob);
    const double *spk = reinterpret_cast<const double *>(blob + pp.fac_bytes64);
    const double *rinv = reinterpret_cast<const double *>(blob + pp.fac_bytes64 + pp.spk_bytes64);
    const int *map = reinterpret_cast<const int *>(blob + pp.fac_bytes64 + pp.spk_bytes64 + pp.rinv_bytes64);
    const int64_t n = h.n;
    std::vector<double> g((size_t)P * lb), red(Nr > 0 ? Nr : 1);
    for (int64_t j = 0; j < m; ++j) {
        for (int64_t i = 0; i < (int64_t)P * lb; ++i) g[i] = i < n ? rhs[i * m + j] : 0.0;
        for (int p = 0; p < P; ++p) solve(lb, fac + (int64_t)map[p] * lb, g.data() + (int64_t)p * lb);
        // pair q: (bottom of block q, top of the next block); a periodic plan
        // also pairs block P-1 with block 0
        auto has_next = [&](int p) { return pp.periodic || p <= P - 2; };
        auto has_prev = [&](int p) { return pp.periodic || p >= 1; };
        auto prev = [&](int p) { return p == 0 ? P - 1 : p - 1; };
        for (int p = 0; p < P; ++p) {
            if (has_next(p))
                for (int c = 0; c < H; ++c) red[2 * H * p + c] = g[(int64_t)p * lb + lb - H + c];
            if (has_prev(p))
                for (int c = 0; c < H; ++c) red[2 * H * prev(p) + H + c] = g[(int64_t)p * lb + c];
        }
        for (int p = 0; p < P; ++p) {
            double xt[2] = {0, 0}, xb[2] = {0, 0};
            for (int c = 0; c < H; ++c)
                for (int k = 0; k < Nr; ++k) {
                    if (has_next(p)) xt[c] += rinv[(size_t)(2 * H * p + H + c) * Nr + k] * red[k];
                    if (has_prev(p)) xb[c] += rinv[(size_t)(2 * H * prev(p) + c) * Nr + k] * red[k];
                }
            const double *sp = spk + (size_t)map[p] * lb * 2 * H;
            for (int t = 0; t < lb; ++t) {
                const int64_t i = (int64_t)p * lb + t;
                if (i >= n) continue;
                double v = g[i];
                for (int c = 0; c < H; ++c) v -= sp[t * 2 * H + c] * xt[c];
                for (int c = 0; c < H; ++c) v -= sp[t * 2 * H + H + c] * xb[c];
                x[i * m + j] = v;
            }
        }
    }
}

// The separator plan, step for step as its kernel runs it: block sweeps
// (separator rows pass through), separator right-hand sides from the
// separator rows' couplings, separators from the stored inverse of S,
// interior correction with the spikes.
template <typename Row, typename Solve>
void emulate_sep(const sbs_lhs &h, const SepPlan &pp, const double *rhs, int64_t m, double *x, Solve solve) {
    const int H = h.kind == SBS_PENTA ? 2 : 1, NB = 2 * H + 1, lb = pp.lb, P = pp.P, Nr = pp.Nr;
    const unsigned char *blob = static_cast<const unsigned char *>(pp.blob64);
    const Row *fac = reinterpret_cast<const Row *>(blob);
    const double *spk = reinterpret_cast<const double *>(blob + pp.fac_bytes64);
    const double *scf = reinterpret_cast<const double *>(blob + pp.fac_bytes64 + pp.spk_bytes64);
    const double *sinv = reinterpret_cast<const double *>(blob + pp.fac_bytes64 + pp.spk_bytes64 + pp.scf_bytes64);
    const int *map = reinterpret_cast<const int *>(blob + pp.fac_bytes64 + pp.spk_bytes64 + pp.scf_bytes64 +
                                                   pp.sinv_bytes64);
    const int64_t n = h.n;
    auto has_sep = [&](int p) { return pp.periodic || p < P - 1; };
    auto has_prev = [&](int p) { return pp.periodic || p >= 1; };
    auto prev = [&](int p) { return p == 0 ? P - 1 : p - 1; };
    auto next = [&](int p) { return p == P - 1 ? 0 : p + 1; };
    std::vector<double> g((size_t)P * lb), f((size_t)P * lb), yh(Nr > 0 ? Nr : 1), z(Nr > 0 ? Nr : 1);
    for (int64_t j = 0; j < m; ++j) {
        for (int64_t i = 0; i < (int64_t)P * lb; ++i) f[i] = g[i] = i < n ? rhs[i * m + j] : 0.0;
        for (int p = 0; p < P; ++p) solve(lb, fac + (int64_t)map[p] * lb, g.data() + (int64_t)p * lb);
        for (int p = 0; p < P; ++p) {
            if (!has_sep(p)) continue;
            for (int c = 0; c < H; ++c) {
                double v = f[(int64_t)p * lb + lb - H + c];
                for (int d = 0; d < NB; ++d) {
                    const int t = lb - H + c + d - H;
                    const double cf = scf[((size_t)map[p] * H + c) * NB + d];
                    if (t < lb - H) v -= cf * g[(int64_t)p * lb + t];
                    else if (t >= lb) v -= cf * g[(int64_t)next(p) * lb + t - lb];
                }
                yh[H * p + c] = v;
            }
        }
        // the product over the window of the row's 16-row tile; an entry
        // outside the window must be 0
        const int Nr4 = (Nr + 3) / 4 * 4;
        for (int r = 0; r < Nr; ++r) {
            const int k0 = pp.kw ? std::min(std::max(r / 16 * 16 + pp.kofs, 0), std::max(Nr4 - pp.kw, 0)) : 0;
            const int k1 = pp.kw ? std::min(k0 + pp.kw, Nr) : Nr;
            double v = 0.0;
            for (int k = k0; k < k1; ++k) v += sinv[(size_t)r * Nr + k] * yh[k];
            for (int k = 0; k < Nr; ++k)
                if ((k < k0 || k >= k1) && sinv[(size_t)r * Nr + k] != 0.0) v = NAN;
            z[r] = v;
        }
        for (int p = 0; p < P; ++p) {
            const double *sp = spk + (size_t)map[p] * lb * 2 * H;
            for (int t = 0; t < lb; ++t) {
                const int64_t i = (int64_t)p * lb + t;
                if (i >= n) continue;
                double v;
                if (has_sep(p) && t >= lb - H) {
                    v = z[H * p + t - (lb - H)];
                } else {
                    v = g[i];
                    for (int c = 0; c < H; ++c) {
                        if (has_sep(p)) v -= sp[t * 2 * H + c] * z[H * p + c];
                        if (has_prev(p)) v -= sp[t * 2 * H + H + c] * z[H * prev(p) + c];
                    }
                }
                x[i * m + j] = v;
            }
        }
    }
}

// The one-wave-per-block mixed-precision kernel's steps, from its copy of
// the separator plan (FP32 coefficients pass by pass, FP64 band rows) and
// the FP32 plan's separator rows, S^{-1} and map: x = fl64(solve32(b)), then
// twice r = fl32(b - A x) (FP64), x += fl64(solve32(r)).
void emulate_refine(const sbs_lhs &h, const SepPlan &pp, const double *rhs, int64_t m, double *x) {
    const int H = h.kind == SBS_PENTA ? 2 : 1, NB = 2 * H + 1, lb = pp.lb, P = pp.P, Nr = pp.Nr;
    const int F = H == 1 ? 2 : 3, Bk = H == 1 ? 1 : 2;
    const unsigned char *blob = static_cast<const unsigned char *>(pp.blob32);
    const float *scf = reinterpret_cast<const float *>(blob + pp.fac_bytes32 + pp.spk_bytes32);
    const int *map = reinterpret_cast<const int *>(blob + pp.fac_bytes32 + pp.spk_bytes32 + pp.scf_bytes32 +
                                                   pp.sinv_bytes32);
    const unsigned char *rec = static_cast<const unsigned char *>(pp.refine.base);
    const float *fwd = reinterpret_cast<const float *>(rec + pp.refine.fwd);
    const float *bwd = reinterpret_cast<const float *>(rec + pp.refine.bwd);
    const float *spk = reinterpret_cast<const float *>(rec + pp.refine.spk);
    const double *band = reinterpret_cast<const double *>(rec + pp.refine.band);
    const float *sinv = reinterpret_cast<const float *>(rec + pp.refine.sinv);
    const int lds = pp.refine.ldsinv;
    const int64_t n = h.n, np = (int64_t)P * lb;
    auto solve32 = [&](std::vector<float> &w) {
        for (int p = 0; p < P; ++p) {
            const int q = map[p];
            float *v = w.data() + (int64_t)p * lb;
            const float *fr = fwd + (size_t)q * lb * F, *br = bwd + (size_t)q * lb * Bk;
            if (H == 1) {
                float y = 0.0f;
                for (int t = 0; t < lb; ++t) y = v[t] = std::fma(-fr[2 * t], y, v[t] * fr[2 * t + 1]);
                float x1 = 0.0f;
                for (int t = lb - 1; t >= 0; --t) x1 = v[t] = std::fma(-br[t], x1, v[t]);
            } else {
                float g1 = 0.0f, g2 = 0.0f;
                for (int t = 0; t < lb; ++t) {
                    const float gg = std::fma(-fr[3 * t + 1], g1, std::fma(-fr[3 * t], g2, v[t] * fr[3 * t + 2]));
                    g2 = g1;
                    g1 = v[t] = gg;
                }
                float x1 = 0.0f, x2 = 0.0f;
                for (int t = lb - 1; t >= 0; --t) {
                    const float xx = std::fma(-br[2 * t], x1, std::fma(-br[2 * t + 1], x2, v[t]));
                    x2 = x1;
                    x1 = v[t] = xx;
                }
            }
        }
        std::vector<float> yh(Nr > 0 ? Nr : 1, 0.0f), z(Nr > 0 ? Nr : 1, 0.0f);
        for (int p = 0; p + 1 < P; ++p) {
            const float *cl = scf + (size_t)map[p] * H * NB, *cr = cl;  // separator p's band rows
            for (int c = 0; c < H; ++c) {
                // own block's last interior rows, then the next block's first rows
                float v = w[(int64_t)p * lb + lb - H + c];
                for (int d = 0; d + c < H; ++d) v = std::fma(-cl[c * NB + d], w[(int64_t)p * lb + lb - 2 * H + c + d], v);
                float r = 0.0f;
                for (int e = 0; e + 2 * H - c < NB; ++e) r = std::fma(-cr[c * NB + 2 * H - c + e], w[(int64_t)(p + 1) * lb + e], r);
                yh[H * p + c] = v + r;
            }
        }
        for (int r = 0; r < Nr; ++r) {
            float v = 0.0f;
            for (int k = 0; k < Nr; ++k) v = std::fma(sinv[(size_t)r * lds + k], yh[k], v);
            for (int k = Nr; k < lds; ++k)
                if (sinv[(size_t)r * lds + k] != 0.0f) v = NAN;  // the padding is zero
            z[r] = v;
        }
        for (int p = 0; p < P; ++p) {
            const float *sp = spk + (size_t)map[p] * lb * 2 * H;
            for (int t = 0; t < lb; ++t) {
                float &v = w[(int64_t)p * lb + t];
                if (p < P - 1 && t >= lb - H) {
                    v = z[H * p + t - (lb - H)];
                    continue;
                }
                for (int c = 0; c < H; ++c) {
                    if (p < P - 1) v = std::fma(-sp[t * 2 * H + c], z[H * p + c], v);
                    if (p > 0) v = std::fma(-sp[t * 2 * H + H + c], z[H * (p - 1) + c], v);
                }
            }
        }
    };
    std::vector<float> b(np), w(np);
    std::vector<double> xc(np);
    for (int64_t j = 0; j < m; ++j) {
        for (int64_t i = 0; i < np; ++i) w[i] = b[i] = i < n ? (float)rhs[i * m + j] : 0.0f;
        solve32(w);
        for (int64_t i = 0; i < np; ++i) xc[i] = (double)w[i];
        for (int k = 0; k < 2; ++k) {
            for (int64_t i = 0; i < np; ++i) {
                double ax = 0.0;
                for (int e = 0; e < NB; ++e) {
                    const int64_t c = i - H + e;
                    const double xv = (c >= 0 && c < np) ? xc[c] : 0.0;
                    ax = e == 0 ? band[i * NB] * xv : std::fma(band[i * NB + e], xv, ax);
                }
                w[i] = (float)((double)b[i] - ax);
            }
            solve32(w);
            for (int64_t i = 0; i < np; ++i) xc[i] += (double)w[i];
        }
        for (int64_t i = 0; i < n; ++i) x[i * m + j] = xc[i];
    }
}

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t kind;
    int64_t n, m;
    if (std::fread(&kind, 4, 1, f) != 1 || std::fread(&n, 8, 1, f) != 1 || std::fread(&m, 8, 1, f) != 1) return 2;
    const int nb = kind == SBS_TRI_PERIODIC ? 3 : kind;
    std::vector<double> bands((size_t)nb * n), rhs((size_t)n * m), x((size_t)n * m);
    if (std::fread(bands.data(), 8, bands.size(), f) != bands.size()) return 2;
    if (std::fread(rhs.data(), 8, rhs.size(), f) != rhs.size()) return 2;
    std::fclose(f);
    sbs_lhs h;
    h.kind = kind;
    h.n = n;
    if (build_partitions(&h, bands.data()) != SBS_OK) return 3;
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 2;
    for (int q = 0; q < 3; ++q) {
        const PartPlan &pp = h.part[q];
        int32_t hdr[4] = {pp.ok ? pp.lb : 0, pp.P, pp.D, pp.Nr};
        std::fwrite(hdr, 4, 4, o);
        if (!pp.ok) continue;
        if (kind != SBS_PENTA)  // periodic plans have plain tridiagonal blocks
            emulate<TriRow<double>>(h, pp, rhs.data(), m, x.data(), solve_tri_rows);
        else
            emulate<PentaRow<double>>(h, pp, rhs.data(), m, x.data(), solve_penta_rows);
        std::fwrite(x.data(), 8, x.size(), o);
    }
    for (int q = 0; q < 3; ++q) {
        const SepPlan &pp = h.sep[q];
        int32_t hdr[4] = {pp.ok ? pp.lb : 0, pp.P, pp.D, pp.Nr};
        std::fwrite(hdr, 4, 4, o);
        if (!pp.ok) continue;
        const int32_t win[2] = {pp.kofs, pp.kw};
        std::fwrite(win, 4, 2, o);
        if (kind != SBS_PENTA)
            emulate_sep<TriRow<double>>(h, pp, rhs.data(), m, x.data(), solve_tri_rows);
        else
            emulate_sep<PentaRow<double>>(h, pp, rhs.data(), m, x.data(), solve_penta_rows);
        std::fwrite(x.data(), 8, x.size(), o);
    }
    for (int q = 1; q < 3; ++q) {
        const SepPlan &pp = h.sep[q];
        const int32_t lb = pp.ok && pp.refine.base ? pp.lb : 0;
        std::fwrite(&lb, 4, 1, o);
        if (!lb) continue;
        emulate_refine(h, pp, rhs.data(), m, x.data());
        std::fwrite(x.data(), 8, x.size(), o);
    }
    std::fclose(o);
    if (h.pdev) std::free(h.pdev);
    return 0;
}
