// Host FP64 factorisation of a banded matrix into the factor rows the sweep
// kernels read, and a host solve with those rows (used to build the block
// partition).  `coef(k, i)` returns band k of row i, 0 outside the matrix.
#pragma once

#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace sbs {

inline bool finite_nonzero(double p) { return std::isfinite(p) && p != 0.0; }

// Section 3.1: den_i = b_i - a_i chat_{i-1}, chat_i = c_i / den_i.
// Rows hold {a_i / den_i, chat_i, 1 / den_i}.  Returns false (and the row)
// on a zero or non-finite pivot.
template <class Coef>
bool factor_tri_rows(int64_t n, Coef coef, TriRow<double> *rows, int64_t *bad) {
    double chat_prev = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double a = coef(0, i), b = coef(1, i), c = coef(2, i);
        const double den = b - a * chat_prev;
        if (!finite_nonzero(den)) {
            *bad = i;
            return false;
        }
        const double chat = c / den;
        rows[i] = {a / den, chat, 1.0 / den, 0.0};
        chat_prev = chat;
    }
    return true;
}

// Section 4.1, A = L R.  With everything outside the matrix equal to zero,
// one recurrence covers every row:
//   beta_i = b_i - a_i gamma_{i-2}
//   alpha_i = c_i - a_i delta_{i-2} - beta_i gamma_{i-1}
//   gamma_i = (d_i - beta_i delta_{i-1}) / alpha_i,  delta_i = e_i / alpha_i,
//   eps_i = a_i.
// Rows hold {eps_i/alpha_i, beta_i/alpha_i, 1/alpha_i, gamma_i, delta_i}.
template <class Coef>
bool factor_penta_rows(int64_t n, Coef coef, PentaRow<double> *rows, int64_t *bad) {
    double g1 = 0.0, g2 = 0.0, d1 = 0.0, d2 = 0.0;  // gamma / delta at i-1 and i-2
    for (int64_t i = 0; i < n; ++i) {
        const double a = coef(0, i), b = coef(1, i), c = coef(2, i), d = coef(3, i), e = coef(4, i);
        const double beta = b - a * g2;
        const double alpha = c - a * d2 - beta * g1;
        if (!finite_nonzero(alpha)) {
            *bad = i;
            return false;
        }
        const double gamma = (d - beta * d1) / alpha;
        const double delta = e / alpha;
        rows[i] = {a / alpha, beta / alpha, 1.0 / alpha, gamma, delta, 0.0, 0.0, 0.0};
        g2 = g1;
        g1 = gamma;
        d2 = d1;
        d1 = delta;
    }
    return true;
}

// Section 3.3, periodic tridiagonal (a_0 and c_{n-1} are the corners): the
// Sherman-Morrison splitting A = A' + u v^T, u = (-b_0, 0.., c_{n-1}),
// v = (1, 0.., -a_0/b_0), leaves A' tridiagonal with A'_00 = 2 b_0 and
// A'_{n-1,n-1} = b_{n-1} + a_0 c_{n-1} / b_0.  The rows carry A''s factor,
// z = A'^{-1} u and wt = A'^{-T} v / (1 + v.z): then v.y = wt.d (1 + v.z)
// for y = A'^{-1} d, so x = y - (wt.d) z needs no third pass.
// Returns false with *bad = the row of a bad pivot, or n when 1 + v.z is zero
// or not finite.  Needs n >= 3.
inline void solve_tri_rows(int64_t n, const TriRow<double> *r, double *x);

template <class Coef>
bool factor_periodic_rows(int64_t n, Coef coef, PeriodicRow<double> *rows, int64_t *bad) {
    const double a0 = coef(0, 0), b0 = coef(1, 0), cl = coef(2, n - 1);
    const double vlast = -a0 / b0;
    auto primed = [&](int k, int64_t i) -> double {  // bands of A' (no corners)
        if (k == 0) return i == 0 ? 0.0 : coef(0, i);
        if (k == 2) return i == n - 1 ? 0.0 : coef(2, i);
        if (i == 0) return b0 + b0;
        if (i == n - 1) return coef(1, n - 1) + a0 * cl / b0;
        return coef(1, i);
    };
    // A'^T has sub-diagonal c_{i-1} and super-diagonal a_{i+1}.
    auto transposed = [&](int k, int64_t i) -> double {
        if (k == 0) return i == 0 ? 0.0 : primed(2, i - 1);
        if (k == 2) return i == n - 1 ? 0.0 : primed(0, i + 1);
        return primed(1, i);
    };
    std::vector<TriRow<double>> f(n), ft(n);
    if (!factor_tri_rows(n, primed, f.data(), bad)) return false;
    if (!factor_tri_rows(n, transposed, ft.data(), bad)) return false;
    std::vector<double> z(n, 0.0), w(n, 0.0);
    z[0] = -b0;
    z[n - 1] = cl;
    solve_tri_rows(n, f.data(), z.data());
    w[0] = 1.0;
    w[n - 1] = vlast;
    solve_tri_rows(n, ft.data(), w.data());
    const double den = 1.0 + (z[0] + vlast * z[n - 1]);
    if (!finite_nonzero(den)) {
        *bad = n;
        return false;
    }
    for (int64_t i = 0; i < n; ++i)
        rows[i] = {f[i].a_s, f[i].chat, f[i].inv, w[i] / den, z[i], 0.0, 0.0, 0.0};
    return true;
}

// x <- A^{-1} x with factor rows (same recurrences as the kernels).
inline void solve_tri_rows(int64_t n, const TriRow<double> *r, double *x) {
    double y1 = 0.0;
    for (int64_t i = 0; i < n; ++i) y1 = x[i] = x[i] * r[i].inv - r[i].a_s * y1;
    double x1 = 0.0;
    for (int64_t i = n - 1; i >= 0; --i) x1 = x[i] = x[i] - r[i].chat * x1;
}

inline void solve_penta_rows(int64_t n, const PentaRow<double> *r, double *x) {
    double g1 = 0.0, g2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double g = x[i] * r[i].inv - r[i].eps_s * g2 - r[i].beta_s * g1;
        x[i] = g;
        g2 = g1;
        g1 = g;
    }
    double x1 = 0.0, x2 = 0.0;
    for (int64_t i = n - 1; i >= 0; --i) {
        const double v = x[i] - r[i].gamma * x1 - r[i].delta * x2;
        x[i] = v;
        x2 = x1;
        x1 = v;
    }
}

}  // namespace sbs
