// Compensated arithmetic of the RK accumulation (error-free transformations).
//
// The update forms U_out = a U_base + b (U_stage + dt L) per conserved variable.
// Every product and sum below is split into its rounded value and its exact
// rounding error (Knuth's two-sum, the fused-multiply-add two-product), and the
// errors are carried to the end, so the one rounding that remains is the final
// addition: the stored value is the exact combination of the given a, U_base, b,
// U_stage, dt and L rounded once (up to the rounding of the error terms, which are
// a few units in the last place of the result smaller). L itself is the
// divergence-plus-source sum formed with a Neumaier compensation.
//
// Written for host and device, so that the CPU tests exercise the same code.
#pragma once

#include <hip/hip_runtime.h>

namespace bhac {

// s + e == a + b exactly, s = fl(a + b) (Knuth; no ordering condition)
__host__ __device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// p + e == a * b exactly, p = fl(a * b) (one fused multiply-add)
__host__ __device__ __forceinline__ void two_prod(double a, double b, double &p, double &e)
{
    p = a * b;
    e = fma(a, b, -p);
}

// sum of x0 + x1 + x2 + x3 with a Neumaier running compensation
__host__ __device__ __forceinline__ double neumaier4(double x0, double x1, double x2, double x3)
{
    double sum = x0, comp = 0.0;
    const double terms[3] = {x1, x2, x3};
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const double x = terms[q];
        const double t = sum + x;
        comp += fabs(sum) >= fabs(x) ? (sum - t) + x : (x - t) + sum;
        sum = t;
    }
    return sum + comp;
}

// a U_base + b (U_stage + dt L) rounded once. BASE = false: the a U_base term is
// absent (a == 0) and ub is not read.
template <bool BASE>
__host__ __device__ __forceinline__ double rk_combine(double a, double ub, double b, double us, double dt, double L)
{
    double p, ep, s2, e2, y, ey;
    two_prod(dt, L, p, ep);              // dt L = p + ep
    two_sum(us, p, s2, e2);              // U_stage + p = s2 + e2
    two_prod(b, s2, y, ey);              // b s2 = y + ey
    const double tail_b = ey + b * (e2 + ep);
    if constexpr (!BASE) return y + tail_b;
    double x, ex, s3, e3;
    two_prod(a, ub, x, ex);              // a U_base = x + ex
    two_sum(x, y, s3, e3);               // x + y = s3 + e3
    return s3 + (e3 + (ex + tail_b));
}

}  // namespace bhac
