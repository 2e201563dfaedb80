// Host FP64 factorisation of a banded matrix into the factor rows the sweep
// kernels read, and a host solve with those rows (used to build the block
// partition).  `coef(k, i)` returns band k of row i, 0 outside the matrix.
#pragma once

#include <cmath>
#include <cstdint>

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
