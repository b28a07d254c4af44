/*
 * opcount.cpp -- op-count build of the CPU oracle (test infrastructure only).
 *
 * The oracle's source is compiled unchanged as C++ with every `double` replaced by
 * a counting type: each floating-point addition, multiplication, division, square
 * root, transcendental call, comparison and sign/absolute/min/max operation is
 * tallied in the region (part of the method) that the oracle marks with OC_SCOPE.
 * The counting type has the size, alignment and calling convention of a double, so
 * the library exports the oracle's entry points with the same signatures and gives
 * bit-identical results (every operation is evaluated in double, in the same order,
 * with contraction off). Only the counts are new: orc_opcount_reset / _read.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <type_traits>

namespace ocnt {

enum Region { OC_OTHER, OC_METRIC, OC_SLOPE, OC_PPM_IFACE, OC_PPM_LIMIT, OC_MC_FACE, OC_FACE_STATE, OC_RIEMANN,
              OC_SOURCES, OC_C2P, OC_P2C, OC_UPDATE, OC_NREGION };
enum Kind { K_ADD, K_MUL, K_DIV, K_SQRT, K_TRANS, K_CMP, K_SIGN, K_NKIND };

static unsigned long long g_count[OC_NREGION][K_NKIND];
static unsigned long long g_calls[OC_NREGION];
static int g_region = OC_OTHER;

static inline void tally(int k) { g_count[g_region][k]++; }

struct Scope {
    int prev;
    explicit Scope(int r) : prev(g_region) { g_region = r; g_calls[r]++; }
    ~Scope() { g_region = prev; }
};

struct Real {
    double v;
    Real() = default;
    template <typename T, typename = typename std::enable_if<std::is_arithmetic<T>::value>::type>
    constexpr Real(T x) : v(static_cast<double>(x)) {}
    explicit operator double() const { return v; }
};
static_assert(sizeof(Real) == sizeof(double) && alignof(Real) == alignof(double), "layout of a double");
static_assert(std::is_trivially_copyable<Real>::value, "passed like a double");

inline Real operator+(Real a, Real b) { tally(K_ADD); return Real(a.v + b.v); }
inline Real operator-(Real a, Real b) { tally(K_ADD); return Real(a.v - b.v); }
inline Real operator*(Real a, Real b) { tally(K_MUL); return Real(a.v * b.v); }
inline Real operator/(Real a, Real b) { tally(K_DIV); return Real(a.v / b.v); }
inline Real operator-(Real a) { tally(K_SIGN); return Real(-a.v); }
inline Real operator+(Real a) { return a; }
inline Real &operator+=(Real &a, Real b) { a = a + b; return a; }
inline Real &operator-=(Real &a, Real b) { a = a - b; return a; }
inline Real &operator*=(Real &a, Real b) { a = a * b; return a; }
inline Real &operator/=(Real &a, Real b) { a = a / b; return a; }
inline bool operator<(Real a, Real b) { tally(K_CMP); return a.v < b.v; }
inline bool operator>(Real a, Real b) { tally(K_CMP); return a.v > b.v; }
inline bool operator<=(Real a, Real b) { tally(K_CMP); return a.v <= b.v; }
inline bool operator>=(Real a, Real b) { tally(K_CMP); return a.v >= b.v; }
inline bool operator==(Real a, Real b) { tally(K_CMP); return a.v == b.v; }
inline bool operator!=(Real a, Real b) { tally(K_CMP); return a.v != b.v; }

}  // namespace ocnt

inline ocnt::Real sqrt(ocnt::Real x) { ocnt::tally(ocnt::K_SQRT); return ocnt::Real(::sqrt(x.v)); }
inline ocnt::Real fabs(ocnt::Real x) { ocnt::tally(ocnt::K_SIGN); return ocnt::Real(::fabs(x.v)); }
inline ocnt::Real pow(ocnt::Real x, ocnt::Real y) { ocnt::tally(ocnt::K_TRANS); return ocnt::Real(::pow(x.v, y.v)); }
inline ocnt::Real exp(ocnt::Real x) { ocnt::tally(ocnt::K_TRANS); return ocnt::Real(::exp(x.v)); }
inline ocnt::Real sin(ocnt::Real x) { ocnt::tally(ocnt::K_TRANS); return ocnt::Real(::sin(x.v)); }
inline ocnt::Real cos(ocnt::Real x) { ocnt::tally(ocnt::K_TRANS); return ocnt::Real(::cos(x.v)); }
inline bool isfinite(ocnt::Real x) { ocnt::tally(ocnt::K_CMP); return std::isfinite(x.v); }

#define OC_SCOPE(region) ocnt::Scope oc_scope_(ocnt::region)
#define double ocnt::Real
extern "C" {
#include "oracle.c"
}
#undef double

extern "C" {

/* Zero every count. */
void orc_opcount_reset(void)
{
    memset(ocnt::g_count, 0, sizeof ocnt::g_count);
    memset(ocnt::g_calls, 0, sizeof ocnt::g_calls);
}

/* Number of regions and kinds; counts as [region][kind] and entries per region. */
void orc_opcount_shape(int *nregion, int *nkind)
{
    *nregion = ocnt::OC_NREGION;
    *nkind = ocnt::K_NKIND;
}

void orc_opcount_read(unsigned long long *counts, unsigned long long *calls)
{
    memcpy(counts, ocnt::g_count, sizeof ocnt::g_count);
    memcpy(calls, ocnt::g_calls, sizeof ocnt::g_calls);
}

}
