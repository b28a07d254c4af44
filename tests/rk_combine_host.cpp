// Host harness for the CPU tests of the RK accumulation (test_rk_combine.py).
//
// Default mode: reads samples (a, U_base, b, U_stage, dt, L) as doubles from stdin
// and writes, per sample, the library's compensated combination and the plain
// expression a U_base + b (U_stage + dt L) (one rounding per operation).
//
// Mode "rk2": reads U0, dt and then pairs (L1, L2) of stage rates until the end of
// input, runs SSP-RK2 (U1 = U + dt L1; U <- U/2 + (U1 + dt L2)/2) once with the
// compensated combination and once with the plain one, and writes both final U.
#include <cstdio>
#include <cstring>
#include <vector>

#include "compensated.h"

static double plain(double a, double ub, double b, double us, double dt, double L)
{
    const volatile double prod = dt * L;
    const volatile double stage = us + prod;
    const volatile double sb = b * stage;
    const volatile double base = a * ub;
    return a != 0.0 ? base + sb : sb;
}

int main(int argc, char **argv)
{
    if (argc > 1 && std::strcmp(argv[1], "rk2") == 0) {
        double h[2], L[2];
        if (std::fread(h, sizeof(double), 2, stdin) != 2) return 1;
        double uc = h[0], up = h[0];
        const double dt = h[1];
        while (std::fread(L, sizeof(double), 2, stdin) == 2) {
            const double uc1 = bhac::rk_combine<false>(0.0, 0.0, 1.0, uc, dt, L[0]);
            uc = bhac::rk_combine<true>(0.5, uc, 0.5, uc1, dt, L[1]);
            const double up1 = plain(0.0, 0.0, 1.0, up, dt, L[0]);
            up = plain(0.5, up, 0.5, up1, dt, L[1]);
        }
        const double r[2] = {uc, up};
        std::fwrite(r, sizeof(double), 2, stdout);
        return 0;
    }
    double s[6];
    std::vector<double> out;
    while (std::fread(s, sizeof(double), 6, stdin) == 6) {
        const double a = s[0], ub = s[1], b = s[2], us = s[3], dt = s[4], L = s[5];
        out.push_back(a != 0.0 ? bhac::rk_combine<true>(a, ub, b, us, dt, L)
                               : bhac::rk_combine<false>(a, ub, b, us, dt, L));
        out.push_back(plain(a, ub, b, us, dt, L));
    }
    std::fwrite(out.data(), sizeof(double), out.size(), stdout);
    return 0;
}
