/*
 * Op-counting build of the oracle (test and measurement infrastructure only).
 *
 * opcount.py compiles every oracle source as C++ with this header
 * force-included.  `double` becomes `ocd`, a standard-layout wrapper of one
 * double with the same size, alignment and calling convention, whose
 * arithmetic operators and math functions count themselves into
 * orc_opc[phase][category], the phase being the one the oracle last named
 * with ORC_PHASE.  Values are computed exactly as in the plain build (same
 * operations, same order, no contraction), so the counts are those of the
 * oracle's own evaluation of the workload.
 *
 * Categories: add/sub, mul, div, sqrt, transcendental (pow, exp, log, cbrt, tanh),
 * compare/min/max/abs, negation.  A "flop" is one of the first five.
 */
#ifndef ORC_OPCOUNT_HPP
#define ORC_OPCOUNT_HPP

#include <float.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

enum { OC_ADD, OC_MUL, OC_DIV, OC_SQRT, OC_TRANS, OC_CMP, OC_NEG, OC_NCAT };

extern "C" {
extern long long orc_opc[16][OC_NCAT];
extern int orc_opc_phase;
}

#define ORC_PHASE(id) (orc_opc_phase = (id))

static inline void oc_tick(int c) { orc_opc[orc_opc_phase][c] += 1; }

struct ocd {
  double v;
  ocd() = default;
  constexpr ocd(double x) : v(x) {}
  explicit operator double() const { return v; }
  explicit operator float() const { return (float)v; }
  ocd& operator+=(ocd o) { oc_tick(OC_ADD); v = v + o.v; return *this; }
  ocd& operator-=(ocd o) { oc_tick(OC_ADD); v = v - o.v; return *this; }
  ocd& operator*=(ocd o) { oc_tick(OC_MUL); v = v * o.v; return *this; }
  ocd& operator/=(ocd o) { oc_tick(OC_DIV); v = v / o.v; return *this; }
  friend ocd operator+(ocd a, ocd b) { oc_tick(OC_ADD); return ocd(a.v + b.v); }
  friend ocd operator-(ocd a, ocd b) { oc_tick(OC_ADD); return ocd(a.v - b.v); }
  friend ocd operator*(ocd a, ocd b) { oc_tick(OC_MUL); return ocd(a.v * b.v); }
  friend ocd operator/(ocd a, ocd b) { oc_tick(OC_DIV); return ocd(a.v / b.v); }
  friend ocd operator-(ocd a) { oc_tick(OC_NEG); return ocd(-a.v); }
  friend ocd operator+(ocd a) { return a; }
  friend bool operator<(ocd a, ocd b) { oc_tick(OC_CMP); return a.v < b.v; }
  friend bool operator>(ocd a, ocd b) { oc_tick(OC_CMP); return a.v > b.v; }
  friend bool operator<=(ocd a, ocd b) { oc_tick(OC_CMP); return a.v <= b.v; }
  friend bool operator>=(ocd a, ocd b) { oc_tick(OC_CMP); return a.v >= b.v; }
  friend bool operator==(ocd a, ocd b) { oc_tick(OC_CMP); return a.v == b.v; }
  friend bool operator!=(ocd a, ocd b) { oc_tick(OC_CMP); return a.v != b.v; }
  friend bool operator!(ocd a) { return !a.v; }
};

static inline ocd sqrt(ocd a) { oc_tick(OC_SQRT); return ocd(std::sqrt(a.v)); }
static inline ocd cbrt(ocd a) { oc_tick(OC_TRANS); return ocd(std::cbrt(a.v)); }
static inline ocd pow(ocd a, ocd b) { oc_tick(OC_TRANS); return ocd(std::pow(a.v, b.v)); }
static inline ocd exp(ocd a) { oc_tick(OC_TRANS); return ocd(std::exp(a.v)); }
static inline ocd log(ocd a) { oc_tick(OC_TRANS); return ocd(std::log(a.v)); }
static inline ocd log10(ocd a) { oc_tick(OC_TRANS); return ocd(std::log10(a.v)); }
static inline ocd tanh(ocd a) { oc_tick(OC_TRANS); return ocd(std::tanh(a.v)); }
static inline ocd fabs(ocd a) { oc_tick(OC_CMP); return ocd(std::fabs(a.v)); }
static inline ocd fmax(ocd a, ocd b) { oc_tick(OC_CMP); return ocd(std::fmax(a.v, b.v)); }
static inline ocd fmin(ocd a, ocd b) { oc_tick(OC_CMP); return ocd(std::fmin(a.v, b.v)); }
static inline ocd copysign(ocd a, ocd b) { oc_tick(OC_CMP); return ocd(std::copysign(a.v, b.v)); }
static inline int isfinite(ocd a) { return std::isfinite(a.v); }
static inline int isnan(ocd a) { return std::isnan(a.v); }

#define double ocd

#endif
