/*
 * tally.hpp -- operation tally of the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY, like the oracle itself. oracle/build.py compiles dg2ref.c a
 * second time, as C++ with this header included first and every `double` of the source
 * read as `Real`: a double that counts the floating-point operations done on it. The
 * arithmetic is unchanged (each operator applies the same double operation in the same
 * order, -ffp-contract=off as in the plain build), so the tallied oracle returns the
 * plain oracle's results bit for bit; Real has the layout of a double, so it keeps the
 * oracle's C interface. The counts give the method's algorithmic operations per cell
 * and step (the oracle computes each face and each cell once, with no halo
 * recomputation). Single-threaded: the OpenMP pragmas are not compiled in.
 */
#ifndef DG2REF_TALLY_HPP
#define DG2REF_TALLY_HPP

#include <math.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

// counters: add (and subtract), multiply, divide, square root, cube root, min/max,
// absolute value, comparison
enum { TALLY_ADD, TALLY_MUL, TALLY_DIV, TALLY_SQRT, TALLY_CBRT, TALLY_MINMAX, TALLY_ABS, TALLY_CMP,
       TALLY_N };
static long long g_tally[TALLY_N];

struct Real {
  double v;
  Real() = default;
  constexpr Real(double x) : v(x) {}
  explicit operator int() const { return (int)v; }
  explicit operator long() const { return (long)v; }
  explicit operator long long() const { return (long long)v; }
};
static_assert(sizeof(Real) == sizeof(double) && alignof(Real) == alignof(double), "layout of a double");

static inline Real operator+(Real a, Real b) { ++g_tally[TALLY_ADD]; return Real(a.v + b.v); }
static inline Real operator-(Real a, Real b) { ++g_tally[TALLY_ADD]; return Real(a.v - b.v); }
static inline Real operator*(Real a, Real b) { ++g_tally[TALLY_MUL]; return Real(a.v * b.v); }
static inline Real operator/(Real a, Real b) { ++g_tally[TALLY_DIV]; return Real(a.v / b.v); }
static inline Real operator-(Real a) { return Real(-a.v); }  // a sign flip, not an operation
static inline Real operator+(Real a) { return a; }
static inline Real &operator+=(Real &a, Real b) { return a = a + b; }
static inline Real &operator-=(Real &a, Real b) { return a = a - b; }
static inline Real &operator*=(Real &a, Real b) { return a = a * b; }
static inline Real &operator/=(Real &a, Real b) { return a = a / b; }
static inline bool operator<(Real a, Real b) { ++g_tally[TALLY_CMP]; return a.v < b.v; }
static inline bool operator>(Real a, Real b) { ++g_tally[TALLY_CMP]; return a.v > b.v; }
static inline bool operator<=(Real a, Real b) { ++g_tally[TALLY_CMP]; return a.v <= b.v; }
static inline bool operator>=(Real a, Real b) { ++g_tally[TALLY_CMP]; return a.v >= b.v; }
static inline bool operator==(Real a, Real b) { ++g_tally[TALLY_CMP]; return a.v == b.v; }
static inline bool operator!=(Real a, Real b) { ++g_tally[TALLY_CMP]; return a.v != b.v; }
static inline Real sqrt(Real a) { ++g_tally[TALLY_SQRT]; return Real(sqrt(a.v)); }
static inline Real cbrt(Real a) { ++g_tally[TALLY_CBRT]; return Real(cbrt(a.v)); }
static inline Real fabs(Real a) { ++g_tally[TALLY_ABS]; return Real(fabs(a.v)); }
static inline Real fmax(Real a, Real b) { ++g_tally[TALLY_MINMAX]; return Real(fmax(a.v, b.v)); }
static inline Real fmin(Real a, Real b) { ++g_tally[TALLY_MINMAX]; return Real(fmin(a.v, b.v)); }
static inline bool isfinite(Real a) { return std::isfinite(a.v); }
static inline bool isnan(Real a) { return std::isnan(a.v); }

extern "C" {
// the counts since the last reset, in the order of the enum above
void dg2ref_tally_read(long long *out) {
  for (int k = 0; k < TALLY_N; ++k) out[k] = g_tally[k];
}
void dg2ref_tally_reset(void) {
  for (int k = 0; k < TALLY_N; ++k) g_tally[k] = 0;
}
}

#define double Real

#endif
