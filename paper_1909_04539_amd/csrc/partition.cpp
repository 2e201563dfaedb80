// Host side of the partitioned solve: block factors, spikes and the inverse
// of the interface system, all in FP64, computed once per shared matrix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <vector>

#include "factor_rows.h"
#include "internal.h"

namespace sbs {
namespace {

constexpr int kMaxBlocks = 64;
constexpr int kMaxInterface = 90;  // interface unknowns: the FP64 inverse stays under 64 KB of LDS

size_t align16(size_t v) { return (v + 15) / 16 * 16; }
size_t align256(size_t v) { return (v + 255) / 256 * 256; }  // each blob starts as a device allocation would

// Gauss-Jordan inverse with partial pivoting, in place (row-major n x n).
bool invert(std::vector<double> &a, int n) {
    std::vector<double> inv((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
        const double pv = a[(size_t)piv * n + c];
        if (!std::isfinite(pv) || std::fabs(pv) < 1e-300) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)piv * n + k], a[(size_t)c * n + k]);
                std::swap(inv[(size_t)piv * n + k], inv[(size_t)c * n + k]);
            }
        const double s = 1.0 / pv;
        for (int k = 0; k < n; ++k) {
            a[(size_t)c * n + k] *= s;
            inv[(size_t)c * n + k] *= s;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = a[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    for (double v : inv)
        if (!std::isfinite(v)) return false;
    a.swap(inv);
    return true;
}

struct HostPlan {
    int lb = 0, P = 0, Nr = 0, D = 0;
    std::vector<unsigned char> fac;  // D*lb FP64 rows (distinct blocks only)
    std::vector<double> spk;         // D*lb*2h
    std::vector<double> rinv;        // Nr*Nr
    std::vector<int> map;            // block p -> stored block map[p]
};

// Accuracy gate of a plan.  The partition reaches the same solution as the
// sweeps in exact arithmetic, but it rounds differently: through the block
// pivots and the interface inverse.  A block whose own pivots are tiny, or an
// ill-conditioned matrix whose interface system amplifies rounding, can move
// the partitioned result far from the recurrences of Sections 3.1 / 4.1 even
// when every pivot is nonzero.  So the plan is run on the host, in FP64, on a
// few seeded right-hand sides and compared with the sweep recurrences on the
// whole matrix; a plan whose result differs by more than kPlanTolerance
// (relative, per column, infinity norm) is dropped and the sweeps serve that
// matrix.
constexpr double kPlanTolerance = 1e-13;
constexpr int kPlanChecks = 4;  // seeded right-hand sides

// Reference: the whole matrix through its factor rows, the recurrences the
// sweep kernels run.  Periodic matrices (Section 3.3): y = A'^{-1} d, then
// x = y - (wt.d) z.
void reference_solve(int kind, bool periodic, int64_t n, const double *bands, std::vector<double> &x) {
    auto cf = [&](int k, int64_t i) -> double {
        if (periodic) return bands[(int64_t)k * n + i];
        const int64_t col = i + k - kind / 2;
        return (col < 0 || col >= n) ? 0.0 : bands[(int64_t)k * n + i];
    };
    int64_t bad = -1;
    if (periodic) {
        std::vector<PeriodicRow<double>> r(n);
        std::vector<TriRow<double>> t(n);
        if (!factor_periodic_rows(n, cf, r.data(), &bad)) return;
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            t[i] = {r[i].a_s, r[i].chat, r[i].inv, 0.0};
            acc += r[i].wt * x[i];
        }
        solve_tri_rows(n, t.data(), x.data());
        for (int64_t i = 0; i < n; ++i) x[i] -= acc * r[i].z;
    } else if (kind == SBS_TRI) {
        std::vector<TriRow<double>> r(n);
        if (factor_tri_rows(n, cf, r.data(), &bad)) solve_tri_rows(n, r.data(), x.data());
    } else {
        std::vector<PentaRow<double>> r(n);
        if (factor_penta_rows(n, cf, r.data(), &bad)) solve_penta_rows(n, r.data(), x.data());
    }
}

// The plan's own solve of one column, as the kernel runs it: block solves,
// interface unknowns from the stored inverse, correction.
template <typename Row, typename SolveFn>
void plan_solve(const HostPlan &hp, int h, bool periodic, int64_t n, SolveFn solve, std::vector<double> &x) {
    const int lb = hp.lb, P = hp.P, Nr = hp.Nr;
    const Row *fac = reinterpret_cast<const Row *>(hp.fac.data());
    std::vector<double> g((size_t)P * lb, 0.0), y(Nr > 0 ? Nr : 1, 0.0);
    for (int64_t i = 0; i < n; ++i) g[i] = x[i];
    for (int p = 0; p < P; ++p) solve(lb, fac + (int64_t)hp.map[p] * lb, g.data() + (int64_t)p * lb);
    auto has_next = [&](int p) { return periodic || p <= P - 2; };
    auto has_prev = [&](int p) { return periodic || p >= 1; };
    auto prev = [&](int p) { return p == 0 ? P - 1 : p - 1; };
    for (int p = 0; p < P; ++p) {
        if (has_next(p))
            for (int c = 0; c < h; ++c) y[2 * h * p + c] = g[(int64_t)p * lb + lb - h + c];
        if (has_prev(p))
            for (int c = 0; c < h; ++c) y[2 * h * prev(p) + h + c] = g[(int64_t)p * lb + c];
    }
    for (int p = 0; p < P; ++p) {
        double xt[2] = {0.0, 0.0}, xb[2] = {0.0, 0.0};
        for (int c = 0; c < h; ++c)
            for (int k = 0; k < Nr; ++k) {
                if (has_next(p)) xt[c] += hp.rinv[(size_t)(2 * h * p + h + c) * Nr + k] * y[k];
                if (has_prev(p)) xb[c] += hp.rinv[(size_t)(2 * h * prev(p) + c) * Nr + k] * y[k];
            }
        const double *sp = hp.spk.data() + (size_t)hp.map[p] * lb * 2 * h;
        for (int t = 0; t < lb; ++t) {
            const int64_t i = (int64_t)p * lb + t;
            if (i >= n) break;
            double v = g[i];
            for (int c = 0; c < h; ++c) v -= sp[t * 2 * h + c] * xt[c];
            for (int c = 0; c < h; ++c) v -= sp[t * 2 * h + h + c] * xb[c];
            x[i] = v;
        }
    }
}

template <typename Row, typename SolveFn>
double plan_deviation(const HostPlan &hp, int kind, bool periodic, int64_t n, const double *bands, SolveFn solve) {
    const int h = kind / 2;
    uint64_t st = 0x9e3779b97f4a7c15ull;  // xorshift64, fixed seed
    double worst = 0.0;
    std::vector<double> d(n), a, b;
    for (int q = 0; q < kPlanChecks; ++q) {
        for (int64_t i = 0; i < n; ++i) {
            st ^= st << 13;
            st ^= st >> 7;
            st ^= st << 17;
            d[i] = (double)(st >> 11) * 0x1.0p-52 - 1.0;  // U[-1, 1)
        }
        a = d;
        b = d;
        reference_solve(kind, periodic, n, bands, a);
        plan_solve<Row>(hp, h, periodic, n, solve, b);
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            num = std::max(num, std::fabs(b[i] - a[i]));
            den = std::max(den, std::fabs(a[i]));
        }
        const double e = den > 0.0 ? num / den : num;
        if (!(e <= worst)) worst = e;  // a NaN stays
    }
    return worst;
}

// kind is 3 or 5 (the bandwidth); `periodic` wraps a tridiagonal matrix
// round (row 0 couples to row n-1 and back), which needs n to be a whole
// number of blocks: then block 0's left neighbour is block P-1 and block
// P-1's right neighbour is block 0, and the interface system gains that pair.
template <typename Row, typename FactorFn, typename SolveFn>
bool build_plan(int kind, bool periodic, int64_t n, const double *bands, int lb, FactorFn factor, SolveFn solve,
                HostPlan &hp) {
    const int h = kind / 2;
    const int P = (int)((n + lb - 1) / lb);
    const int pairs = periodic ? P : P - 1;
    if (P > kMaxBlocks || lb < 2 * h || 2 * h * pairs > kMaxInterface) return false;
    if (periodic && (n % lb != 0 || P < 2)) return false;
    const int64_t npad = (int64_t)P * lb;
    std::vector<Row> rows(npad);
    std::vector<double> spk((size_t)npad * 2 * h, 0.0);
    // Coefficient k of global row i restricted to block p (identity past n).
    auto local = [&](int p, int k, int64_t i) -> double {
        if (i >= n) return k == h ? 1.0 : 0.0;
        const int64_t col = i + k - h;
        if (col < (int64_t)p * lb || col >= (int64_t)(p + 1) * lb || col >= n) return 0.0;
        return bands[(int64_t)k * n + i];
    };
    // Entry of row i < n in column col (any index; wrapped when periodic).
    auto entry = [&](int64_t i, int64_t col) -> double {
        if (i >= n) return 0.0;
        int64_t d = col - i;
        if (periodic) {
            d = ((d % n) + n) % n;
            if (d > n / 2) d -= n;
        } else if (col < 0 || col >= n) {
            return 0.0;
        }
        return (d >= -h && d <= h) ? bands[(int64_t)(d + h) * n + i] : 0.0;
    };
    std::vector<double> v(lb);
    for (int p = 0; p < P; ++p) {
        const int64_t r0 = (int64_t)p * lb;
        int64_t bad = -1;
        if (!factor(lb, [&](int k, int64_t t) { return local(p, k, r0 + t); }, rows.data() + r0, &bad)) return false;
        // Right spike columns: coupling of row r0+t to column r0+lb+c
        // (block p+1's first unknowns; none past the last block unless periodic).
        for (int c = 0; c < h; ++c) {
            for (int t = 0; t < lb; ++t)
                v[t] = (p < P - 1 || periodic) ? entry(r0 + t, r0 + lb + c) : 0.0;
            solve(lb, rows.data() + r0, v.data());
            for (int t = 0; t < lb; ++t) spk[(size_t)(r0 + t) * 2 * h + c] = v[t];
        }
        // Left spike columns: coupling of row r0+t to column r0-h+c.
        for (int c = 0; c < h; ++c) {
            for (int t = 0; t < lb; ++t) v[t] = (p > 0 || periodic) ? entry(r0 + t, r0 - h + c) : 0.0;
            solve(lb, rows.data() + r0, v.data());
            for (int t = 0; t < lb; ++t) spk[(size_t)(r0 + t) * 2 * h + h + c] = v[t];
        }
    }
    // Interface system.  Unknown order: pair q holds (bottom h of block q,
    // top h of block q+1), q = 0..P-2, and q = P-1 (block P-1, block 0) when
    // periodic.
    const int Nr = 2 * h * pairs;
    std::vector<double> R((size_t)Nr * Nr, 0.0);
    const auto next = [&](int p) { return p == P - 1 ? 0 : p + 1; };
    const auto prev = [&](int p) { return p == 0 ? P - 1 : p - 1; };
    const auto has_next = [&](int p) { return periodic || p <= P - 2; };
    const auto has_prev = [&](int p) { return periodic || p >= 1; };
    auto ibot = [&](int p, int c) { return 2 * h * p + c; };              // bottom of block p
    auto itop = [&](int p, int c) { return 2 * h * prev(p) + h + c; };    // top of block p
    auto V = [&](int p, int t, int c) { return spk[(size_t)((int64_t)p * lb + t) * 2 * h + c]; };
    auto Wt = [&](int p, int t, int c) { return spk[(size_t)((int64_t)p * lb + t) * 2 * h + h + c]; };
    for (int p = 0; p < P; ++p) {
        for (int c = 0; c < h; ++c) {
            // equation of block p's local row t, for its interface rows
            for (int side = 0; side < 2; ++side) {
                int row, t;
                if (side == 0) {  // bottom rows
                    if (!has_next(p)) continue;
                    row = ibot(p, c);
                    t = lb - h + c;
                } else {  // top rows
                    if (!has_prev(p)) continue;
                    row = itop(p, c);
                    t = c;
                }
                R[(size_t)row * Nr + row] += 1.0;
                for (int c2 = 0; c2 < h; ++c2) {
                    if (has_next(p)) R[(size_t)row * Nr + itop(next(p), c2)] += V(p, t, c2);
                    if (has_prev(p)) R[(size_t)row * Nr + ibot(prev(p), c2)] += Wt(p, t, c2);
                }
            }
        }
    }
    if (Nr > 0 && !invert(R, Nr)) return false;
    hp.lb = lb;
    hp.P = P;
    hp.Nr = Nr;
    // Blocks whose factor rows and spikes are bit-identical (every interior
    // block of a matrix with constant bands) are stored once.
    const size_t rb = sizeof(Row) * lb, sb = sizeof(double) * lb * 2 * h;
    hp.map.assign(P, -1);
    hp.fac.clear();
    hp.spk.clear();
    for (int p = 0; p < P; ++p) {
        const unsigned char *rp = reinterpret_cast<const unsigned char *>(rows.data() + (int64_t)p * lb);
        const double *sp = spk.data() + (size_t)p * lb * 2 * h;
        for (int q = 0; q < hp.D && hp.map[p] < 0; ++q)
            if (!std::memcmp(hp.fac.data() + q * rb, rp, rb) && !std::memcmp(hp.spk.data() + q * lb * 2 * h, sp, sb))
                hp.map[p] = q;
        if (hp.map[p] < 0) {
            hp.map[p] = hp.D++;
            hp.fac.insert(hp.fac.end(), rp, rp + rb);
            hp.spk.insert(hp.spk.end(), sp, sp + (size_t)lb * 2 * h);
        }
    }
    hp.rinv.swap(R);
    const double dev = plan_deviation<Row>(hp, kind, periodic, n, bands, solve);
    return dev <= kPlanTolerance;
}

// ---------------------------------------------------------------------------
// Separator partition (SepPlan).

constexpr int kMaxSepInterface = 128;  // separator unknowns: the FP64 inverse stays within 128 KB of LDS

struct SepHostPlan {
    int lb = 0, P = 0, Nr = 0, D = 0;
    std::vector<unsigned char> fac;  // D*lb FP64 rows
    std::vector<double> spk;         // D*lb*2h: V (own separator), W (previous separator)
    std::vector<double> scf;         // D*h*(2h+1)
    std::vector<double> sinv;        // Nr*Nr
    std::vector<int> map;
    int kofs = 0, kw = 0;            // window of the S^{-1} product (sep_window)
};

// Entries of S^{-1} that cannot matter, and the window of columns the
// kernel's product then reads.  The separators of blocks far apart are
// coupled only through the spikes, which decay row by row for a diagonally
// dominant or positive definite matrix, so most of S^{-1} is far below its
// row's largest entry (for the 1024-row hyperdiffusion matrix in 32-row
// blocks, entries two separators apart are below 1e-24 of it).  An entry
// whose magnitude is at most 2^-60 / Nr of its row's largest is set to 0:
// the dropped part of any z_i = sum_j S^{-1}_ij yhat_j is then at most
// 2^-60 max_j |S^{-1}_ij| max |yhat|, below 1 / (128 Nr) of the rounding
// error bound of the product itself.  The product is done in 16-row tiles of
// S^{-1}; tile t (rows 16t .. 16t + 15) reads columns k0 .. k0 + kw - 1 with
// k0 = min(max(16t + kofs, 0), max(Nr4 - kw, 0)), Nr4 = Nr rounded up to 4,
// which holds every nonzero entry of the tile's rows.  kw = 0: every column.
void sep_window(std::vector<double> &S, int Nr, int &kofs, int &kw) {
    kofs = kw = 0;
    if (Nr <= 0) return;
    for (int i = 0; i < Nr; ++i) {
        double mx = 0.0;
        for (int j = 0; j < Nr; ++j) mx = std::max(mx, std::fabs(S[(size_t)i * Nr + j]));
        const double thr = std::ldexp(mx, -60) / Nr;
        for (int j = 0; j < Nr; ++j)
            if (std::fabs(S[(size_t)i * Nr + j]) <= thr) S[(size_t)i * Nr + j] = 0.0;
    }
    const int mt = (Nr + 15) / 16, Nr4 = (Nr + 3) / 4 * 4;
    std::vector<int> lo(mt, Nr), hi(mt, -1);
    for (int i = 0; i < Nr; ++i)
        for (int j = 0; j < Nr; ++j)
            if (S[(size_t)i * Nr + j] != 0.0) {
                lo[i / 16] = std::min(lo[i / 16], j);
                hi[i / 16] = std::max(hi[i / 16], j);
            }
    int ofs = 0;
    for (int t = 0; t < mt; ++t) ofs = std::min(ofs, lo[t] - 16 * t);
    ofs = -((-ofs + 3) / 4 * 4);
    for (int w = 4; w < Nr4; w += 4) {
        bool holds = true;
        for (int t = 0; t < mt && holds; ++t) {
            const int k0 = std::min(std::max(16 * t + ofs, 0), std::max(Nr4 - w, 0));
            holds = lo[t] >= k0 && hi[t] < k0 + w;
        }
        if (holds) {
            kofs = ofs;
            kw = w;
            return;
        }
    }
}

// The separator plan's own solve of one column, as the kernel runs it:
// block sweeps (separator rows pass through unchanged), separator
// right-hand sides yhat, separators z = S^{-1} yhat, interior correction.
template <typename Row, typename SolveFn>
void sep_plan_solve(const SepHostPlan &hp, int h, bool periodic, int64_t n, SolveFn solve, std::vector<double> &x) {
    const int lb = hp.lb, P = hp.P, Nr = hp.Nr, nb = 2 * h + 1;
    const Row *fac = reinterpret_cast<const Row *>(hp.fac.data());
    auto has_sep = [&](int p) { return periodic || p < P - 1; };
    auto has_prev = [&](int p) { return periodic || p >= 1; };
    auto prev = [&](int p) { return p == 0 ? P - 1 : p - 1; };
    auto next = [&](int p) { return p == P - 1 ? 0 : p + 1; };
    std::vector<double> g((size_t)P * lb, 0.0), f = g, yh(Nr > 0 ? Nr : 1, 0.0), z = yh;
    for (int64_t i = 0; i < n; ++i) f[i] = g[i] = x[i];
    for (int p = 0; p < P; ++p) solve(lb, fac + (int64_t)hp.map[p] * lb, g.data() + (int64_t)p * lb);
    for (int p = 0; p < P; ++p) {
        if (!has_sep(p)) continue;
        const double *cf = hp.scf.data() + (size_t)hp.map[p] * h * nb;
        for (int c = 0; c < h; ++c) {
            double v = f[(int64_t)p * lb + lb - h + c];
            for (int d = 0; d < nb; ++d) {
                const int t = lb - h + c + d - h;  // column, relative to the block's first row
                double val = 0.0;
                if (t < lb - h) val = g[(int64_t)p * lb + t];
                else if (t >= lb) val = g[(int64_t)next(p) * lb + t - lb];
                v -= cf[c * nb + d] * val;
            }
            yh[h * p + c] = v;
        }
    }
    for (int r = 0; r < Nr; ++r) {
        double v = 0.0;
        for (int k = 0; k < Nr; ++k) v += hp.sinv[(size_t)r * Nr + k] * yh[k];
        z[r] = v;
    }
    for (int p = 0; p < P; ++p) {
        const double *sp = hp.spk.data() + (size_t)hp.map[p] * lb * 2 * h;
        for (int t = 0; t < lb; ++t) {
            const int64_t i = (int64_t)p * lb + t;
            if (i >= n) break;
            double v;
            if (has_sep(p) && t >= lb - h) {
                v = z[h * p + t - (lb - h)];
            } else {
                v = g[i];
                for (int c = 0; c < h; ++c) {
                    if (has_sep(p)) v -= sp[t * 2 * h + c] * z[h * p + c];
                    if (has_prev(p)) v -= sp[t * 2 * h + h + c] * z[h * prev(p) + c];
                }
            }
            x[i] = v;
        }
    }
}

template <typename Row, typename SolveFn>
double sep_plan_deviation(const SepHostPlan &hp, int kind, bool periodic, int64_t n, const double *bands,
                          SolveFn solve) {
    const int h = kind / 2;
    uint64_t st = 0x9e3779b97f4a7c15ull;  // xorshift64, fixed seed
    double worst = 0.0;
    std::vector<double> d(n), a, b;
    for (int q = 0; q < kPlanChecks; ++q) {
        for (int64_t i = 0; i < n; ++i) {
            st ^= st << 13;
            st ^= st >> 7;
            st ^= st << 17;
            d[i] = (double)(st >> 11) * 0x1.0p-52 - 1.0;  // U[-1, 1)
        }
        a = d;
        b = d;
        reference_solve(kind, periodic, n, bands, a);
        sep_plan_solve<Row>(hp, h, periodic, n, solve, b);
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            num = std::max(num, std::fabs(b[i] - a[i]));
            den = std::max(den, std::fabs(a[i]));
        }
        const double e = den > 0.0 ? num / den : num;
        if (!(e <= worst)) worst = e;  // a NaN stays
    }
    return worst;
}

// kind 3 or 5; `periodic` wraps a tridiagonal matrix round (needs n a whole
// number P >= 2 of blocks; every block then has a separator).
template <typename Row, typename FactorFn, typename SolveFn>
bool build_sep_plan(int kind, bool periodic, int64_t n, const double *bands, int lb, FactorFn factor, SolveFn solve,
                    SepHostPlan &hp) {
    const int h = kind / 2, nb = 2 * h + 1;
    const int P = (int)((n + lb - 1) / lb);
    if (periodic && (n % lb != 0 || P < 2)) return false;
    const int nsep = periodic ? P : P - 1;
    if (P > kMaxBlocks || lb < 2 * h + 1 || h * nsep > kMaxSepInterface) return false;
    const int64_t npad = (int64_t)P * lb;
    auto has_sep = [&](int p) { return periodic || p < P - 1; };
    auto has_prev = [&](int p) { return periodic || p >= 1; };
    auto prev = [&](int p) { return p == 0 ? P - 1 : p - 1; };
    auto next = [&](int p) { return p == P - 1 ? 0 : p + 1; };
    auto interior = [&](int p) { return has_sep(p) ? lb - h : lb; };
    // Entry of row i < n in column col (any index; wrapped when periodic).
    auto entry = [&](int64_t i, int64_t col) -> double {
        if (i >= n) return 0.0;
        int64_t d = col - i;
        if (periodic) {
            d = ((d % n) + n) % n;
            if (d > n / 2) d -= n;
        } else if (col < 0 || col >= n) {
            return 0.0;
        }
        return (d >= -h && d <= h) ? bands[(int64_t)(d + h) * n + i] : 0.0;
    };
    std::vector<Row> rows(npad);
    std::vector<double> spk((size_t)npad * 2 * h, 0.0), scf((size_t)P * h * nb, 0.0);
    std::vector<double> v(lb);
    for (int p = 0; p < P; ++p) {
        const int64_t r0 = (int64_t)p * lb;
        const int ni = interior(p);
        // the interior block: coefficients among its own interior columns,
        // identity on separator rows and past the end
        auto local = [&](int k, int64_t t) -> double {
            const int64_t i = r0 + t;
            if (i >= n || t >= ni) return k == h ? 1.0 : 0.0;
            const int64_t ct = t + k - h;
            if (ct < 0 || ct >= ni || r0 + ct >= n) return 0.0;
            return bands[(int64_t)k * n + i];
        };
        int64_t bad = -1;
        if (!factor(lb, local, rows.data() + r0, &bad)) return false;
        for (int c = 0; c < h; ++c) {
            // V: the block's own separator rows r0 + ni + c
            for (int t = 0; t < lb; ++t) v[t] = (has_sep(p) && t < ni) ? entry(r0 + t, r0 + ni + c) : 0.0;
            solve(lb, rows.data() + r0, v.data());
            for (int t = 0; t < lb; ++t) spk[(size_t)(r0 + t) * 2 * h + c] = t < ni ? v[t] : 0.0;
            // W: the previous separator, rows r0 - h + c (wrapped for block 0)
            const int64_t pc = p == 0 ? n - h + c : r0 - h + c;
            for (int t = 0; t < lb; ++t) v[t] = (has_prev(p) && t < ni) ? entry(r0 + t, pc) : 0.0;
            solve(lb, rows.data() + r0, v.data());
            for (int t = 0; t < lb; ++t) spk[(size_t)(r0 + t) * 2 * h + h + c] = t < ni ? v[t] : 0.0;
        }
        if (!has_sep(p)) continue;
        // band rows of the separator rows, without the separator columns
        for (int c = 0; c < h; ++c)
            for (int d = 0; d < nb; ++d) {
                const int t = ni + c + d - h;
                if (t >= ni && t < lb) continue;
                scf[((size_t)p * h + c) * nb + d] = entry(r0 + ni + c, r0 + t);
            }
    }
    // S: separator s (of block s), row c.  Unknown order h * s + c.
    const int Nr = h * nsep;
    std::vector<double> S((size_t)Nr * Nr, 0.0);
    auto V = [&](int p, int t, int c) { return spk[(size_t)((int64_t)p * lb + t) * 2 * h + c]; };
    auto W = [&](int p, int t, int c) { return spk[(size_t)((int64_t)p * lb + t) * 2 * h + h + c]; };
    for (int s = 0; s < nsep; ++s) {
        const int64_t r0 = (int64_t)s * lb;
        const int ni = lb - h, nx = next(s);
        for (int c = 0; c < h; ++c) {
            const int row = h * s + c;
            for (int c2 = 0; c2 < h; ++c2) S[(size_t)row * Nr + h * s + c2] += entry(r0 + ni + c, r0 + ni + c2);
            for (int d = 0; d < nb; ++d) {
                const int t = ni + c + d - h;
                const double cf = scf[((size_t)s * h + c) * nb + d];
                if (cf == 0.0) continue;
                if (t < ni) {  // interior row t of block s
                    for (int c2 = 0; c2 < h; ++c2) {
                        S[(size_t)row * Nr + h * s + c2] -= cf * V(s, t, c2);
                        if (has_prev(s)) S[(size_t)row * Nr + h * prev(s) + c2] -= cf * W(s, t, c2);
                    }
                } else {  // interior row t - lb of the next block
                    const int u = t - lb;
                    for (int c2 = 0; c2 < h; ++c2) {
                        S[(size_t)row * Nr + h * s + c2] -= cf * W(nx, u, c2);
                        if (has_sep(nx)) S[(size_t)row * Nr + h * nx + c2] -= cf * V(nx, u, c2);
                    }
                }
            }
        }
    }
    if (Nr > 0 && !invert(S, Nr)) return false;
    sep_window(S, Nr, hp.kofs, hp.kw);
    hp.lb = lb;
    hp.P = P;
    hp.Nr = Nr;
    hp.D = 0;
    const size_t rb = sizeof(Row) * lb, sb = sizeof(double) * lb * 2 * h, cb = sizeof(double) * h * nb;
    hp.map.assign(P, -1);
    hp.fac.clear();
    hp.spk.clear();
    hp.scf.clear();
    for (int p = 0; p < P; ++p) {
        const unsigned char *rp = reinterpret_cast<const unsigned char *>(rows.data() + (int64_t)p * lb);
        const double *sp = spk.data() + (size_t)p * lb * 2 * h;
        const double *cp = scf.data() + (size_t)p * h * nb;
        for (int q = 0; q < hp.D && hp.map[p] < 0; ++q)
            if (!std::memcmp(hp.fac.data() + q * rb, rp, rb) && !std::memcmp(hp.spk.data() + q * lb * 2 * h, sp, sb) &&
                !std::memcmp(hp.scf.data() + (size_t)q * h * nb, cp, cb))
                hp.map[p] = q;
        if (hp.map[p] < 0) {
            hp.map[p] = hp.D++;
            hp.fac.insert(hp.fac.end(), rp, rp + rb);
            hp.spk.insert(hp.spk.end(), sp, sp + (size_t)lb * 2 * h);
            hp.scf.insert(hp.scf.end(), cp, cp + (size_t)h * nb);
        }
    }
    hp.sinv.swap(S);
    return sep_plan_deviation<Row>(hp, kind, periodic, n, bands, solve) <= kPlanTolerance;
}

template <typename Row32, typename Row64>
Row32 narrow_row(const Row64 &r);
template <>
TriRow<float> narrow_row(const TriRow<double> &r) {
    return {(float)r.a_s, (float)r.chat, (float)r.inv, 0.0f};
}
template <>
PentaRow<float> narrow_row(const PentaRow<double> &r) {
    return {(float)r.eps_s, (float)r.beta_s, (float)r.inv, (float)r.gamma, (float)r.delta, 0.f, 0.f, 0.f};
}

// memcpy that accepts an empty source (an empty vector's data() may be null).
void copy_bytes(void *dst, const void *src, size_t bytes) {
    if (bytes) std::memcpy(dst, src, bytes);
}

// Serialise one plan as [fac | spk | rinv | map] in FP64 and in FP32.
template <typename Row64, typename Row32>
void serialise(const HostPlan &hp, std::vector<unsigned char> &b64, std::vector<unsigned char> &b32, PartPlan &pp) {
    const size_t nrow = hp.fac.size() / sizeof(Row64);
    const size_t map_bytes = align16(hp.map.size() * sizeof(int));
    pp.fac_bytes64 = align16(hp.fac.size());
    pp.spk_bytes64 = align16(hp.spk.size() * 8);
    pp.rinv_bytes64 = align16(hp.rinv.size() * 8);
    b64.assign(pp.fac_bytes64 + pp.spk_bytes64 + pp.rinv_bytes64 + map_bytes, 0);
    copy_bytes(b64.data(), hp.fac.data(), hp.fac.size());
    copy_bytes(b64.data() + pp.fac_bytes64, hp.spk.data(), hp.spk.size() * 8);
    copy_bytes(b64.data() + pp.fac_bytes64 + pp.spk_bytes64, hp.rinv.data(), hp.rinv.size() * 8);
    copy_bytes(b64.data() + pp.fac_bytes64 + pp.spk_bytes64 + pp.rinv_bytes64, hp.map.data(),
                hp.map.size() * sizeof(int));
    pp.fac_bytes32 = align16(nrow * sizeof(Row32));
    pp.spk_bytes32 = align16(hp.spk.size() * 4);
    pp.rinv_bytes32 = align16(hp.rinv.size() * 4);
    b32.assign(pp.fac_bytes32 + pp.spk_bytes32 + pp.rinv_bytes32 + map_bytes, 0);
    const Row64 *r64 = reinterpret_cast<const Row64 *>(hp.fac.data());
    Row32 *r32 = reinterpret_cast<Row32 *>(b32.data());
    for (size_t i = 0; i < nrow; ++i) r32[i] = narrow_row<Row32>(r64[i]);
    float *s32 = reinterpret_cast<float *>(b32.data() + pp.fac_bytes32);
    for (size_t i = 0; i < hp.spk.size(); ++i) s32[i] = (float)hp.spk[i];
    float *q32 = reinterpret_cast<float *>(b32.data() + pp.fac_bytes32 + pp.spk_bytes32);
    for (size_t i = 0; i < hp.rinv.size(); ++i) q32[i] = (float)hp.rinv[i];
    copy_bytes(b32.data() + pp.fac_bytes32 + pp.spk_bytes32 + pp.rinv_bytes32, hp.map.data(),
                hp.map.size() * sizeof(int));
    pp.map_bytes = map_bytes;
    pp.D = hp.D;
}

// Serialise one separator plan as [fac | spk | scf | sinv | map] in FP64 and FP32.
template <typename Row64, typename Row32>
void serialise_sep(const SepHostPlan &hp, std::vector<unsigned char> &b64, std::vector<unsigned char> &b32,
                   SepPlan &pp) {
    const size_t nrow = hp.fac.size() / sizeof(Row64);
    const size_t map_bytes = align16(hp.map.size() * sizeof(int));
    pp.fac_bytes64 = align16(hp.fac.size());
    pp.spk_bytes64 = align16(hp.spk.size() * 8);
    pp.scf_bytes64 = align16(hp.scf.size() * 8);
    pp.sinv_bytes64 = align16(hp.sinv.size() * 8);
    b64.assign(pp.fac_bytes64 + pp.spk_bytes64 + pp.scf_bytes64 + pp.sinv_bytes64 + map_bytes, 0);
    unsigned char *at = b64.data();
    copy_bytes(at, hp.fac.data(), hp.fac.size());
    copy_bytes(at += pp.fac_bytes64, hp.spk.data(), hp.spk.size() * 8);
    copy_bytes(at += pp.spk_bytes64, hp.scf.data(), hp.scf.size() * 8);
    copy_bytes(at += pp.scf_bytes64, hp.sinv.data(), hp.sinv.size() * 8);
    copy_bytes(at += pp.sinv_bytes64, hp.map.data(), hp.map.size() * sizeof(int));
    pp.fac_bytes32 = align16(nrow * sizeof(Row32));
    pp.spk_bytes32 = align16(hp.spk.size() * 4);
    pp.scf_bytes32 = align16(hp.scf.size() * 4);
    pp.sinv_bytes32 = align16(hp.sinv.size() * 4);
    b32.assign(pp.fac_bytes32 + pp.spk_bytes32 + pp.scf_bytes32 + pp.sinv_bytes32 + map_bytes, 0);
    const Row64 *r64 = reinterpret_cast<const Row64 *>(hp.fac.data());
    Row32 *r32 = reinterpret_cast<Row32 *>(b32.data());
    for (size_t i = 0; i < nrow; ++i) r32[i] = narrow_row<Row32>(r64[i]);
    auto put = [](unsigned char *dst, const std::vector<double> &src) {
        float *f = reinterpret_cast<float *>(dst);
        for (size_t i = 0; i < src.size(); ++i) f[i] = (float)src[i];
    };
    unsigned char *q = b32.data() + pp.fac_bytes32;
    put(q, hp.spk);
    put(q += pp.spk_bytes32, hp.scf);
    put(q += pp.scf_bytes32, hp.sinv);
    copy_bytes(q += pp.sinv_bytes32, hp.map.data(), hp.map.size() * sizeof(int));
    pp.map_bytes = map_bytes;
    pp.D = hp.D;
    pp.lb = hp.lb;
    pp.P = hp.P;
    pp.Nr = hp.Nr;
    pp.kofs = hp.kofs;
    pp.kw = hp.kw;
}

// The one-wave-per-block mixed-precision kernel's copy of a separator plan:
// each pass's coefficients contiguous, so that a wave reads a run of rows
// with a few wide scalar loads.  Per distinct block (FP32, from the plan):
// forward coefficients (tri a/den, 1/den; penta eps/alpha, beta/alpha,
// 1/alpha), backward coefficients (tri chat; penta gamma, delta), spikes;
// per block (FP64): the original band rows, 0 outside the matrix; and S^{-1}
// (FP32) with its rows padded with zeros to a multiple of 8 entries.
template <typename Row32>
void serialise_refine(const SepHostPlan &hp, const std::vector<unsigned char> &b32, const SepPlan &sp, int kind,
                      int64_t n, const double *bands, std::vector<unsigned char> &out, RefinePlan &rp) {
    const int h = kind / 2, nb = 2 * h + 1, lb = hp.lb, D = hp.D, P = hp.P;
    const int F = kind == SBS_TRI ? 2 : 3, Bk = kind == SBS_TRI ? 1 : 2;
    rp.fwd = 0;
    rp.bwd = align256(rp.fwd + (size_t)D * lb * F * 4);
    rp.spk = align256(rp.bwd + (size_t)D * lb * Bk * 4);
    rp.band = align256(rp.spk + (size_t)D * lb * 2 * h * 4);
    rp.ldsinv = (hp.Nr + 7) / 8 * 8;
    rp.sinv = align256(rp.band + (size_t)P * lb * nb * 8);
    const size_t total = align256(rp.sinv + (size_t)hp.Nr * rp.ldsinv * 4);
    out.assign(total, 0);
    const Row32 *rows = reinterpret_cast<const Row32 *>(b32.data());
    float *fwd = reinterpret_cast<float *>(out.data() + rp.fwd);
    float *bwd = reinterpret_cast<float *>(out.data() + rp.bwd);
    for (size_t i = 0; i < (size_t)D * lb; ++i) {
        if constexpr (sizeof(Row32) == sizeof(TriRow<float>)) {
            fwd[2 * i] = rows[i].a_s;
            fwd[2 * i + 1] = rows[i].inv;
            bwd[i] = rows[i].chat;
        } else {
            fwd[3 * i] = rows[i].eps_s;
            fwd[3 * i + 1] = rows[i].beta_s;
            fwd[3 * i + 2] = rows[i].inv;
            bwd[2 * i] = rows[i].gamma;
            bwd[2 * i + 1] = rows[i].delta;
        }
    }
    copy_bytes(out.data() + rp.spk, b32.data() + sp.fac_bytes32, (size_t)D * lb * 2 * h * 4);
    double *band = reinterpret_cast<double *>(out.data() + rp.band);
    for (int64_t i = 0; i < std::min<int64_t>(n, (int64_t)P * lb); ++i)
        for (int k = 0; k < nb; ++k) {
            const int64_t col = i + k - h;
            band[i * nb + k] = (col >= 0 && col < n) ? bands[(int64_t)k * n + i] : 0.0;
        }
    float *sinv = reinterpret_cast<float *>(out.data() + rp.sinv);
    for (int r = 0; r < hp.Nr; ++r)
        for (int k = 0; k < hp.Nr; ++k) sinv[(size_t)r * rp.ldsinv + k] = (float)hp.sinv[(size_t)r * hp.Nr + k];
}

}  // namespace

// Builds every plan that exists for this matrix.  A plan that does not exist
// (too many blocks, a zero pivot inside a block, a singular interface
// system) only disables the partitioned variant for that block length.
sbs_status build_partitions(sbs_lhs *h, const double *bands) {
    std::vector<unsigned char> b64[3], b32[3], s64[3], s32[3], r32[3];
    size_t total = 0;
    // A periodic tridiagonal matrix is partitioned directly (the blocks are
    // plain tridiagonal; the wrap is one more interface pair).
    const bool periodic = h->kind == SBS_TRI_PERIODIC;
    const bool tri = h->kind == SBS_TRI || periodic;
    for (int q = 0; q < 3; ++q) {
        HostPlan hp;
        const int lb = kPartLbs[q];
        bool ok;
        if (tri)
            ok = build_plan<TriRow<double>>(SBS_TRI, periodic, h->n, bands, lb,
                                            factor_tri_rows<std::function<double(int, int64_t)>>, solve_tri_rows, hp);
        else
            ok = build_plan<PentaRow<double>>(SBS_PENTA, false, h->n, bands, lb,
                                              factor_penta_rows<std::function<double(int, int64_t)>>, solve_penta_rows, hp);
        if (!ok) continue;
        PartPlan &pp = h->part[q];
        pp.periodic = periodic;
        if (tri)
            serialise<TriRow<double>, TriRow<float>>(hp, b64[q], b32[q], pp);
        else
            serialise<PentaRow<double>, PentaRow<float>>(hp, b64[q], b32[q], pp);
        pp.lb = hp.lb;
        pp.P = hp.P;
        pp.Nr = hp.Nr;
        pp.ok = true;
        total += align256(b64[q].size()) + align256(b32[q].size());
    }
    for (int q = 0; q < 3; ++q) {
        SepHostPlan hp;
        const int lb = kPartLbs[q];
        bool ok;
        if (tri)
            ok = build_sep_plan<TriRow<double>>(SBS_TRI, periodic, h->n, bands, lb,
                                                factor_tri_rows<std::function<double(int, int64_t)>>, solve_tri_rows,
                                                hp);
        else
            ok = build_sep_plan<PentaRow<double>>(SBS_PENTA, false, h->n, bands, lb,
                                                  factor_penta_rows<std::function<double(int, int64_t)>>,
                                                  solve_penta_rows, hp);
        if (!ok) continue;
        SepPlan &sp = h->sep[q];
        sp.periodic = periodic;
        if (tri)
            serialise_sep<TriRow<double>, TriRow<float>>(hp, s64[q], s32[q], sp);
        else
            serialise_sep<PentaRow<double>, PentaRow<float>>(hp, s64[q], s32[q], sp);
        sp.ok = true;
        total += align256(s64[q].size()) + align256(s32[q].size());
        if (!periodic && lb >= 32) {
            if (tri)
                serialise_refine<TriRow<float>>(hp, s32[q], sp, SBS_TRI, h->n, bands, r32[q], sp.refine);
            else
                serialise_refine<PentaRow<float>>(hp, s32[q], sp, SBS_PENTA, h->n, bands, r32[q], sp.refine);
            total += r32[q].size();
        }
    }
    if (total == 0) return SBS_OK;
    void *dev = nullptr;
    if (hipMalloc(&dev, total) != hipSuccess) return SBS_ERR_NO_MEMORY;
    h->pdev = dev;
    size_t at = 0;
    for (int q = 0; q < 3; ++q) {
        PartPlan &pp = h->part[q];
        if (!pp.ok) continue;
        unsigned char *base = static_cast<unsigned char *>(dev);
        if (hipMemcpy(base + at, b64[q].data(), b64[q].size(), hipMemcpyHostToDevice) != hipSuccess)
            return SBS_ERR_DEVICE;
        pp.blob64 = base + at;
        at += align256(b64[q].size());
        if (hipMemcpy(base + at, b32[q].data(), b32[q].size(), hipMemcpyHostToDevice) != hipSuccess)
            return SBS_ERR_DEVICE;
        pp.blob32 = base + at;
        at += align256(b32[q].size());
    }
    for (int q = 0; q < 3; ++q) {
        SepPlan &sp = h->sep[q];
        if (!sp.ok) continue;
        unsigned char *base = static_cast<unsigned char *>(dev);
        if (hipMemcpy(base + at, s64[q].data(), s64[q].size(), hipMemcpyHostToDevice) != hipSuccess)
            return SBS_ERR_DEVICE;
        sp.blob64 = base + at;
        at += align256(s64[q].size());
        if (hipMemcpy(base + at, s32[q].data(), s32[q].size(), hipMemcpyHostToDevice) != hipSuccess)
            return SBS_ERR_DEVICE;
        sp.blob32 = base + at;
        at += align256(s32[q].size());
        if (!r32[q].empty()) {
            if (hipMemcpy(base + at, r32[q].data(), r32[q].size(), hipMemcpyHostToDevice) != hipSuccess)
                return SBS_ERR_DEVICE;
            sp.refine.base = base + at;
            at += r32[q].size();
        }
    }
    h->device_bytes += (int64_t)total;
    return SBS_OK;
}

}  // namespace sbs
