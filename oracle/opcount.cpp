// opcount.cpp -- operation count of the oracle's pair integral.
//
// TEST AND MEASUREMENT INFRASTRUCTURE ONLY (like oracle.c, which it compiles
// unchanged): oracle.c is included with `double` replaced by a scalar type
// that counts every floating-point operation it takes part in.  The count
// of orc_tet_potential (the exact potential of one affinely magnetised tet,
// Sec. 2.1) per (target, tet) pair is the algorithmic work per near-field
// pair that the near-field roofline is priced with.
//
// Counted: add/subtract, multiply, divide, sqrt, log, atan (and atan2),
// comparisons.  Negation and fabs are sign operations and are not counted.
// oracle.c is built without floating-point contraction, so there are no
// fused operations to split.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

namespace {

struct Ops {
    long long add, mul, div, sqrt, log, atan, cmp, other;
};
Ops g_ops;

struct CountedDouble {
    double v;
    CountedDouble() : v(0.0) {}
    CountedDouble(double x) : v(x) {}
    CountedDouble(int x) : v(x) {}
    CountedDouble(long x) : v((double)x) {}
    CountedDouble(long long x) : v((double)x) {}
    explicit operator int() const { return (int)v; }
    explicit operator unsigned() const { return (unsigned)v; }
    explicit operator long() const { return (long)v; }
    explicit operator long long() const { return (long long)v; }
};
using CD = CountedDouble;

inline CD operator+(CD a, CD b) { ++g_ops.add; return CD(a.v + b.v); }
inline CD operator-(CD a, CD b) { ++g_ops.add; return CD(a.v - b.v); }
inline CD operator*(CD a, CD b) { ++g_ops.mul; return CD(a.v * b.v); }
inline CD operator/(CD a, CD b) { ++g_ops.div; return CD(a.v / b.v); }
inline CD operator-(CD a) { return CD(-a.v); }
inline CD &operator+=(CD &a, CD b) { return a = a + b; }
inline CD &operator-=(CD &a, CD b) { return a = a - b; }
inline CD &operator*=(CD &a, CD b) { return a = a * b; }
inline CD &operator/=(CD &a, CD b) { return a = a / b; }
inline bool operator<(CD a, CD b) { ++g_ops.cmp; return a.v < b.v; }
inline bool operator>(CD a, CD b) { ++g_ops.cmp; return a.v > b.v; }
inline bool operator<=(CD a, CD b) { ++g_ops.cmp; return a.v <= b.v; }
inline bool operator>=(CD a, CD b) { ++g_ops.cmp; return a.v >= b.v; }
inline bool operator==(CD a, CD b) { ++g_ops.cmp; return a.v == b.v; }
inline bool operator!=(CD a, CD b) { ++g_ops.cmp; return a.v != b.v; }
inline CD sqrt(CD a) { ++g_ops.sqrt; return CD(std::sqrt(a.v)); }
inline CD log(CD a) { ++g_ops.log; return CD(std::log(a.v)); }
inline CD atan(CD a) { ++g_ops.atan; return CD(std::atan(a.v)); }
inline CD atan2(CD a, CD b) { ++g_ops.atan; return CD(std::atan2(a.v, b.v)); }
inline CD fabs(CD a) { return CD(std::fabs(a.v)); }
inline CD floor(CD a) { return CD(std::floor(a.v)); }
inline CD ldexp(CD a, int e) { return CD(std::ldexp(a.v, e)); }
inline CD cos(CD a) { ++g_ops.other; return CD(std::cos(a.v)); }
inline CD sin(CD a) { ++g_ops.other; return CD(std::sin(a.v)); }
inline CD exp(CD a) { ++g_ops.other; return CD(std::exp(a.v)); }
inline CD pow(CD a, CD b) { ++g_ops.other; return CD(std::pow(a.v, b.v)); }

}  // namespace

#define double CountedDouble
#include "oracle.c"
#undef double

// Counts of orc_tet_potential over the npairs pairs (pair_tgt[k], pair_tet[k]):
// nodes [n][3], tets [T][4] node ids, targets [N][3], M [n][3] nodal values.
// out[8] += add, mul, div, sqrt, log, atan, cmp, other.  The potentials are
// summed into *u (so that the work is not optimised away).
extern "C" void opc_count_pairs(const double *nodes, const int32_t *tets, const double *targets, const double *M,
                                const int64_t *pair_tgt, const int64_t *pair_tet, int64_t npairs, long long *out,
                                double *u)
{
    double acc = 0.0;
    for (int64_t k = 0; k < npairs; ++k) {
        const int32_t *t = tets + 4 * pair_tet[k];
        CountedDouble x[3], v[12], m[12];
        for (int d = 0; d < 3; ++d) x[d] = CountedDouble(targets[3 * pair_tgt[k] + d]);
        for (int c = 0; c < 4; ++c)
            for (int d = 0; d < 3; ++d) {
                v[3 * c + d] = CountedDouble(nodes[3 * t[c] + d]);
                m[3 * c + d] = CountedDouble(M[3 * t[c] + d]);
            }
        g_ops = Ops{};
        const CountedDouble r = orc_tet_potential(x, v, m);
        acc += r.v;
        out[0] += g_ops.add;
        out[1] += g_ops.mul;
        out[2] += g_ops.div;
        out[3] += g_ops.sqrt;
        out[4] += g_ops.log;
        out[5] += g_ops.atan;
        out[6] += g_ops.cmp;
        out[7] += g_ops.other;
    }
    *u = acc;
}
