/*
 * Forward-mode dual number for the oracle's tangent build.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Compiling
 * wlseno_oracle.c as C++ with this header force-included and
 * -DOR_REAL=or_dual -DOR_TANGENT runs the oracle's own algorithm on values
 * that carry OR_NDIR directional derivatives alongside.  The result is the
 * exact Jacobian-vector product of the scheme as the oracle computes it.
 *
 * Rules:
 *   - the value part of every operation is the same IEEE double operation the
 *     plain build performs (same library call for sqrt and pow), so values are
 *     bitwise those of the FP64 oracle;
 *   - comparisons look at values only: every branch (the smallest facet
 *     indicator, pivot order and ties, numerical rank, positivity) is taken
 *     as at the point itself and held fixed, i.e. the derivative is the one
 *     of the active branch;
 *   - derivatives are the textbook ones: (ab)' = a'b + ab', (a/b)' =
 *     (a' - (a/b) b') / b, sqrt(a)' = a' / (2 sqrt a), |a|' = sign(a) a',
 *     copysign(a, b)' = sign(a) sign(b) a', (a^n)' = n a^(n-1) a' for an
 *     integer exponent n;
 *   - a value built from a plain double is a constant (no tangent work until
 *     it meets a non-constant), which keeps the geometry terms cheap.
 */
#pragma once

#include <cmath>
#include <cstring>

#ifndef OR_NDIR
#define OR_NDIR 8
#endif

// directions in use (<= OR_NDIR), set by the entry points before a run; the
// slots beyond it are never read
static int or_nd = OR_NDIR;

struct or_dual {
    double v;
    double d[OR_NDIR];
    bool k;   // constant: every d[] is zero

    or_dual() = default;
    or_dual(double x) : v(x), k(true)
    {
        for (int t = 0; t < or_nd; ++t) d[t] = 0.0;
    }
    explicit operator double() const { return v; }

    or_dual &operator+=(const or_dual &b);
    or_dual &operator-=(const or_dual &b);
    or_dual &operator*=(const or_dual &b);
    or_dual &operator/=(const or_dual &b);
};

static inline or_dual or_const(double x) { return or_dual(x); }

static inline or_dual operator+(const or_dual &a, const or_dual &b)
{
    or_dual r;
    r.v = a.v + b.v;
    r.k = a.k && b.k;
    for (int t = 0; t < or_nd; ++t) r.d[t] = r.k ? 0.0 : a.d[t] + b.d[t];
    return r;
}

static inline or_dual operator-(const or_dual &a, const or_dual &b)
{
    or_dual r;
    r.v = a.v - b.v;
    r.k = a.k && b.k;
    for (int t = 0; t < or_nd; ++t) r.d[t] = r.k ? 0.0 : a.d[t] - b.d[t];
    return r;
}

static inline or_dual operator-(const or_dual &a)
{
    or_dual r;
    r.v = -a.v;
    r.k = a.k;
    for (int t = 0; t < or_nd; ++t) r.d[t] = -a.d[t];
    return r;
}

static inline or_dual operator*(const or_dual &a, const or_dual &b)
{
    or_dual r;
    r.v = a.v * b.v;
    r.k = a.k && b.k;
    if (r.k) {
        for (int t = 0; t < or_nd; ++t) r.d[t] = 0.0;
    } else if (a.k) {
        for (int t = 0; t < or_nd; ++t) r.d[t] = a.v * b.d[t];
    } else if (b.k) {
        for (int t = 0; t < or_nd; ++t) r.d[t] = a.d[t] * b.v;
    } else {
        for (int t = 0; t < or_nd; ++t) r.d[t] = a.d[t] * b.v + a.v * b.d[t];
    }
    return r;
}

static inline or_dual operator/(const or_dual &a, const or_dual &b)
{
    or_dual r;
    r.v = a.v / b.v;
    r.k = a.k && b.k;
    if (r.k) {
        for (int t = 0; t < or_nd; ++t) r.d[t] = 0.0;
    } else {
        for (int t = 0; t < or_nd; ++t) r.d[t] = (a.d[t] - r.v * b.d[t]) / b.v;
    }
    return r;
}

inline or_dual &or_dual::operator+=(const or_dual &b) { return *this = *this + b; }
inline or_dual &or_dual::operator-=(const or_dual &b) { return *this = *this - b; }
inline or_dual &or_dual::operator*=(const or_dual &b) { return *this = *this * b; }
inline or_dual &or_dual::operator/=(const or_dual &b) { return *this = *this / b; }

// mixed operands: the double is a constant
static inline or_dual operator+(double a, const or_dual &b) { return or_dual(a) + b; }
static inline or_dual operator+(const or_dual &a, double b) { return a + or_dual(b); }
static inline or_dual operator-(double a, const or_dual &b) { return or_dual(a) - b; }
static inline or_dual operator-(const or_dual &a, double b) { return a - or_dual(b); }
static inline or_dual operator*(double a, const or_dual &b) { return or_dual(a) * b; }
static inline or_dual operator*(const or_dual &a, double b) { return a * or_dual(b); }
static inline or_dual operator/(double a, const or_dual &b) { return or_dual(a) / b; }
static inline or_dual operator/(const or_dual &a, double b) { return a / or_dual(b); }

// comparisons: values only (the branch taken at the point)
static inline bool operator<(const or_dual &a, const or_dual &b) { return a.v < b.v; }
static inline bool operator>(const or_dual &a, const or_dual &b) { return a.v > b.v; }
static inline bool operator<=(const or_dual &a, const or_dual &b) { return a.v <= b.v; }
static inline bool operator>=(const or_dual &a, const or_dual &b) { return a.v >= b.v; }
static inline bool operator==(const or_dual &a, const or_dual &b) { return a.v == b.v; }
static inline bool operator!=(const or_dual &a, const or_dual &b) { return a.v != b.v; }
static inline bool operator<(const or_dual &a, double b) { return a.v < b; }
static inline bool operator>(const or_dual &a, double b) { return a.v > b; }
static inline bool operator<=(const or_dual &a, double b) { return a.v <= b; }
static inline bool operator>=(const or_dual &a, double b) { return a.v >= b; }
static inline bool operator==(const or_dual &a, double b) { return a.v == b; }
static inline bool operator!=(const or_dual &a, double b) { return a.v != b; }
static inline bool operator<(double a, const or_dual &b) { return a < b.v; }
static inline bool operator>(double a, const or_dual &b) { return a > b.v; }

static inline or_dual sqrt(const or_dual &a)
{
    or_dual r;
    r.v = std::sqrt(a.v);
    r.k = a.k;
    const double s = 0.5 / r.v;
    for (int t = 0; t < or_nd; ++t) r.d[t] = a.k ? 0.0 : s * a.d[t];
    return r;
}

static inline or_dual fabs(const or_dual &a)
{
    or_dual r;
    r.v = std::fabs(a.v);
    r.k = a.k;
    const double s = a.v > 0.0 ? 1.0 : (a.v < 0.0 ? -1.0 : 0.0);
    for (int t = 0; t < or_nd; ++t) r.d[t] = s * a.d[t];
    return r;
}

// |a| with the sign of b; the sign of b is held (branch at the point)
static inline or_dual copysign(const or_dual &a, const or_dual &b)
{
    or_dual r;
    r.v = std::copysign(a.v, b.v);
    r.k = a.k;
    const double s = (std::signbit(a.v) == std::signbit(b.v)) ? 1.0 : -1.0;
    for (int t = 0; t < or_nd; ++t) r.d[t] = s * a.d[t];
    return r;
}

// a^e for a constant integer exponent e >= 0 (the only use: Taylor monomials)
static inline or_dual pow(const or_dual &a, const or_dual &e)
{
    or_dual r;
    r.v = std::pow(a.v, e.v);
    const int n = (int)e.v;
    r.k = a.k || n == 0;
    const double s = (r.k || n == 0) ? 0.0 : (double)n * std::pow(a.v, (double)(n - 1));
    for (int t = 0; t < or_nd; ++t) r.d[t] = r.k ? 0.0 : s * a.d[t];
    return r;
}

// a value with directional derivatives dir[t * stride] (t < ndir), the rest zero
static inline or_dual or_seed(double v, const double *dir, int ndir, size_t stride)
{
    or_dual r(v);
    bool any = false;
    for (int t = 0; t < ndir && t < or_nd; ++t) {
        r.d[t] = dir[(size_t)t * stride];
        any = any || r.d[t] != 0.0;
    }
    r.k = !any;
    if (r.k)
        for (int t = 0; t < or_nd; ++t) r.d[t] = 0.0;
    return r;
}
