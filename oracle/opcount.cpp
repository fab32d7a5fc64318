// opcount.cpp -- the reference solver with every floating-point operation
// counted.
//
// TEST INFRASTRUCTURE ONLY, like the rest of this directory.  This file
// compiles swe_oracle.c unchanged as C++, with its real type replaced by a
// type that holds one double and counts the operations done on it, so the
// arithmetic (and every result, bit for bit) is the reference solver's and
// the counts are the work its algorithm performs: the operations the method
// needs per cell update, whatever a GPU kernel does to reach them.  The
// result is the algorithmic operation count of Sec. 2's step (augmented
// Riemann solves, fluctuations, limited corrections, update, cleanup).
//
// Counted separately: additions and subtractions, multiplications,
// divisions, square roots, comparisons (not floating-point arithmetic, but
// they steer the wet/dry and limiter branches), and the rest (sign flips,
// absolute values, powers).  Built single-threaded (the OpenMP pragmas are
// ignored), so the counters need no synchronisation.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

namespace opc {
struct Counts {
    int64_t add, mul, div, sqrt, cmp, other;
};
Counts g_counts = {0, 0, 0, 0, 0, 0};
}  // namespace opc

// A double that counts what is done with it.  Construction from a double is
// implicit (literals and ints mix in as in C); the way back is explicit, so
// every operation between reals goes through the counting operators below.
struct CountedReal {
    double v;
    CountedReal() = default;
    CountedReal(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return (int)v; }
};
static_assert(sizeof(CountedReal) == sizeof(double), "layout of the solver's structs");

static inline CountedReal operator+(CountedReal a, CountedReal b) {
    ++opc::g_counts.add;
    return CountedReal(a.v + b.v);
}
static inline CountedReal operator-(CountedReal a, CountedReal b) {
    ++opc::g_counts.add;
    return CountedReal(a.v - b.v);
}
static inline CountedReal operator*(CountedReal a, CountedReal b) {
    ++opc::g_counts.mul;
    return CountedReal(a.v * b.v);
}
static inline CountedReal operator/(CountedReal a, CountedReal b) {
    ++opc::g_counts.div;
    return CountedReal(a.v / b.v);
}
static inline CountedReal operator-(CountedReal a) {
    ++opc::g_counts.other;
    return CountedReal(-a.v);
}
static inline CountedReal& operator+=(CountedReal& a, CountedReal b) { return a = a + b; }
static inline CountedReal& operator-=(CountedReal& a, CountedReal b) { return a = a - b; }
static inline CountedReal& operator*=(CountedReal& a, CountedReal b) { return a = a * b; }
static inline CountedReal& operator/=(CountedReal& a, CountedReal b) { return a = a / b; }
#define ORC_CMP(op)                                                   \
    static inline bool operator op(CountedReal a, CountedReal b) {    \
        ++opc::g_counts.cmp;                                          \
        return a.v op b.v;                                            \
    }
ORC_CMP(<)
ORC_CMP(>)
ORC_CMP(<=)
ORC_CMP(>=)
ORC_CMP(==)
ORC_CMP(!=)
#undef ORC_CMP
static inline CountedReal sqrt(CountedReal a) {
    ++opc::g_counts.sqrt;
    return CountedReal(::sqrt(a.v));
}
static inline CountedReal fabs(CountedReal a) {
    ++opc::g_counts.other;
    return CountedReal(::fabs(a.v));
}
static inline CountedReal pow(CountedReal a, CountedReal b) {
    ++opc::g_counts.other;
    return CountedReal(::pow(a.v, b.v));
}
static inline bool isfinite(CountedReal a) { return std::isfinite(a.v); }

#define double CountedReal
extern "C" {
#include "swe_oracle.c"
}
#undef double

extern "C" {

// Counters since the last reset: add, mul, div, sqrt, cmp, other.
void orc_opcount_get(int64_t out[6]) {
    out[0] = opc::g_counts.add;
    out[1] = opc::g_counts.mul;
    out[2] = opc::g_counts.div;
    out[3] = opc::g_counts.sqrt;
    out[4] = opc::g_counts.cmp;
    out[5] = opc::g_counts.other;
}

void orc_opcount_reset(void) { opc::g_counts = opc::Counts{0, 0, 0, 0, 0, 0}; }

}  // extern "C"
