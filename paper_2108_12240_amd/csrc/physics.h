// Device physics of the GRMHD substep: metric records, face states and fluxes,
// reconstruction, the GLM + HLL/TVDLF face flux, geometric sources and the
// conserved-to-primitive inversion. Templated on the arithmetic type R of the
// face work (double, or float in the mixed-precision path); sources and the
// inversion are always double.
//
// Both supported metrics (flat Cartesian and Kerr-Schild in (ln r, theta, phi))
// have gamma_12 = gamma_23 = 0, beta^2 = beta^3 = 0 and no x3 dependence; the
// code below only carries those non-zero entries.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace bhac {

// Double-precision reciprocal and reciprocal square root for the inversion and the
// sources: the hardware seed refined by two Newton-Raphson steps (r <- r (2 - x r),
// y <- y (3 - x y^2) / 2), good to about one ulp for the positive, normal arguments
// used there, at a third of the cost of the correctly rounded sequences.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// Fast arithmetic of the face work: in float the hardware reciprocal and square
// root (1 ulp); in double the Newton-refined versions above (about 1 ulp).
template <typename R>
__device__ __forceinline__ R frcp(R b)
{
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(b);
    else return rcp_nr(b);
}
template <typename R>
__device__ __forceinline__ R fdiv(R a, R b)
{
    return a * frcp(b);
}
template <typename R>
__device__ __forceinline__ R fsqrt(R x)
{
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_sqrtf(x);
    else return x > 0.0 ? x * rsqrt_nr(x) : 0.0;
}

template <typename R>
struct FaceM {
    R al, b1, g11, g13, g22, g33, gi11, gi13, gi22, gi33, sg;
};

struct CentM {
    double al, b1, g11, g13, g22, g33, gi11, gi13, gi22, gi33, sg;
    double da1, da2, db1, db2, dg11_1, dg11_2, dg13_1, dg13_2, dg22_1, dg22_2, dg33_1, dg33_2;
};

template <typename R, bool KS, typename T>
__device__ __forceinline__ FaceM<R> load_face_metric(const T *__restrict__ tab, long long nrec, long long r)
{
    FaceM<R> m;
    if constexpr (!KS) {
        m.al = R(1); m.b1 = R(0); m.g11 = R(1); m.g13 = R(0); m.g22 = R(1); m.g33 = R(1);
        m.gi11 = R(1); m.gi13 = R(0); m.gi22 = R(1); m.gi33 = R(1); m.sg = R(1);
    } else {
        m.al = (R)tab[C_ALPHA * nrec + r];
        m.b1 = (R)tab[C_BETA1 * nrec + r];
        m.g11 = (R)tab[C_G11 * nrec + r];
        m.g13 = (R)tab[C_G13 * nrec + r];
        m.g22 = (R)tab[C_G22 * nrec + r];
        m.g33 = (R)tab[C_G33 * nrec + r];
        m.gi11 = (R)tab[C_GI11 * nrec + r];
        m.gi13 = (R)tab[C_GI13 * nrec + r];
        m.gi22 = (R)tab[C_GI22 * nrec + r];
        m.gi33 = (R)tab[C_GI33 * nrec + r];
        m.sg = (R)tab[C_SG * nrec + r];
    }
    return m;
}

template <bool KS>
__device__ __forceinline__ CentM load_centre_metric(const double *__restrict__ tab, long long nrec, long long r)
{
    CentM m;
    if constexpr (!KS) {
        m.al = 1; m.b1 = 0; m.g11 = 1; m.g13 = 0; m.g22 = 1; m.g33 = 1;
        m.gi11 = 1; m.gi13 = 0; m.gi22 = 1; m.gi33 = 1; m.sg = 1;
        m.da1 = m.da2 = m.db1 = m.db2 = 0;
        m.dg11_1 = m.dg11_2 = m.dg13_1 = m.dg13_2 = m.dg22_1 = m.dg22_2 = m.dg33_1 = m.dg33_2 = 0;
    } else {
        const double *t = tab + r;
        m.al = t[C_ALPHA * nrec]; m.b1 = t[C_BETA1 * nrec];
        m.g11 = t[C_G11 * nrec]; m.g13 = t[C_G13 * nrec]; m.g22 = t[C_G22 * nrec]; m.g33 = t[C_G33 * nrec];
        m.gi11 = t[C_GI11 * nrec]; m.gi13 = t[C_GI13 * nrec]; m.gi22 = t[C_GI22 * nrec]; m.gi33 = t[C_GI33 * nrec];
        m.sg = t[C_SG * nrec];
        m.da1 = t[C_DA1 * nrec]; m.da2 = t[C_DA2 * nrec]; m.db1 = t[C_DB1 * nrec]; m.db2 = t[C_DB2 * nrec];
        m.dg11_1 = t[C_DG11_1 * nrec]; m.dg11_2 = t[C_DG11_2 * nrec];
        m.dg13_1 = t[C_DG13_1 * nrec]; m.dg13_2 = t[C_DG13_2 * nrec];
        m.dg22_1 = t[C_DG22_1 * nrec]; m.dg22_2 = t[C_DG22_2 * nrec];
        m.dg33_1 = t[C_DG33_1 * nrec]; m.dg33_2 = t[C_DG33_2 * nrec];
    }
    return m;
}

__device__ __forceinline__ FaceM<double> centre_as_face(const CentM &c)
{
    return FaceM<double>{c.al, c.b1, c.g11, c.g13, c.g22, c.g33, c.gi11, c.gi13, c.gi22, c.gi33, c.sg};
}

// ---------------------------------------------------------------------------------
// Block addressing and metric records of a cell or face of a block.
// ---------------------------------------------------------------------------------
// cell (i, j, k) of a work item: returns false for the tail threads
__device__ __forceinline__ bool cell_of(const DevBlock &B, int item, int &i, int &j, int &k)
{
    const int nc = B.s[0] * B.s[1] * B.s[2];
    if (item >= nc) return false;
    i = item % B.s[0];
    const int t = item / B.s[0];
    j = t % B.s[1];
    k = t / B.s[1];
    return true;
}

__device__ __forceinline__ long long pad_index(const DevBlock &B, const KParams &kp, int i, int j, int k)
{
    return B.off + ((long long)k * B.n1 + j) * B.n0 + i;
}

// Slot of block B's ghost position (l0, l1, l2) (at least one coordinate outside the
// block): a block's ghost slots follow its interior cells, in the order of its
// (size + 2g) box with x fastest and the interior skipped.
__device__ __forceinline__ long long ghost_slot(const DevBlock &B, const KParams &kp, int l0, int l1, int l2)
{
    const int g0 = kp.g[0], g1 = kp.g[1], g2 = kp.g[2];
    const int s0 = B.s[0], s1 = B.s[1], s2 = B.s[2];
    const long long w0 = s0 + 2 * g0, w1 = s1 + 2 * g1;
    const long long bx = l0 + g0, by = l1 + g1, bz = l2 + g2;
    const long long zin = min(max(l2, 0), s2);                 // interior planes before
    long long r = bz * w0 * w1 - zin * s0 * s1;
    if (l2 < 0 || l2 >= s2) {
        r += by * w0 + bx;
    } else {
        const long long yin = min(max(l1, 0), s1);              // interior rows before
        r += by * w0 - yin * s0;
        r += (l1 < 0 || l1 >= s1 || l0 < 0) ? bx : bx - s0;
    }
    return B.off + (long long)s0 * s1 * s2 + r;
}

template <bool KS>
__device__ __forceinline__ CentM centre_metric(const GridDev &gd, const DevBlock &B, int i, int j)
{
    if constexpr (!KS) {
        return load_centre_metric<false>(nullptr, 0, 0);
    } else {
        const DevLevel &L = gd.levels[B.level];
        const long long r = L.ctab + (long long)(B.o[1] + j) * L.N0 + (B.o[0] + i);
        return load_centre_metric<true>(gd.ctab, gd.nrec_c, r);
    }
}

template <typename R, int D, bool KS>
__device__ __forceinline__ FaceM<R> face_metric(const GridDev &gd, const DevBlock &B, int i, int j)
{
    if constexpr (!KS) {
        return load_face_metric<R, false, double>(nullptr, 0, 0);
    } else {
        const DevLevel &L = gd.levels[B.level];
        const int gi = B.o[0] + i, gj = B.o[1] + j;
        long long r;
        if constexpr (D == 0) r = L.f0tab + (long long)gj * (L.N0 + 1) + gi;
        else if constexpr (D == 1) r = L.f1tab + (long long)gj * L.N0 + gi;
        else r = L.ctab + (long long)gj * L.N0 + gi;
        if constexpr (sizeof(R) == 4) {
            const float *t = D == 0 ? gd.f0tab32 : (D == 1 ? gd.f1tab32 : gd.ctab32);
            return load_face_metric<R, true, float>(t, D == 0 ? gd.nrec_f0 : (D == 1 ? gd.nrec_f1 : gd.nrec_c), r);
        } else {
            const double *t = D == 0 ? gd.f0tab : (D == 1 ? gd.f1tab : gd.ctab);
            return load_face_metric<R, true, double>(t, D == 0 ? gd.nrec_f0 : (D == 1 ? gd.nrec_f1 : gd.nrec_c), r);
        }
    }
}

// ---------------------------------------------------------------------------------
// Conserved vector, physical flux along D and the fast-speed bounds of one state.
// The normal-field and psi fluxes are left zero (the GLM solve provides them).
// ---------------------------------------------------------------------------------
template <typename R, int D, bool WANT_FLUX, bool WANT_SPEED = !WANT_FLUX>
__device__ __forceinline__ void face_state(const R *q, const FaceM<R> &m, R gam, R gfac, R *U, R *F, R &lm,
                                           R &lp)
{
    const R u1 = q[1], u2 = q[2], u3 = q[3];
    const R ul1 = m.g11 * u1 + m.g13 * u3, ul2 = m.g22 * u2, ul3 = m.g13 * u1 + m.g33 * u3;
    const R W = fsqrt(R(1) + (u1 * ul1 + u2 * ul2 + u3 * ul3));
    const R iW = frcp(W);
    const R v[3] = {u1 * iW, u2 * iW, u3 * iW};
    const R vl[3] = {ul1 * iW, ul2 * iW, ul3 * iW};
    const R v2 = v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2];
    const R B[3] = {q[5], q[6], q[7]};
    const R Bl[3] = {m.g11 * B[0] + m.g13 * B[2], m.g22 * B[1], m.g13 * B[0] + m.g33 * B[2]};
    const R B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
    const R Bv = B[0] * vl[0] + B[1] * vl[1] + B[2] * vl[2];
    const R rho = q[0], p = q[4];
    const R rhoh = rho + gfac * p;
    const R iW2 = iW * iW;
    const R b2 = B2 * iW2 + Bv * Bv;
    const R vd = v[D];
    const R bd = D == 0 ? m.b1 : R(0);
    if constexpr (WANT_FLUX) {
        const R xi = rhoh * W * W;
        const R Dd = rho * W;
        const R xb = xi + B2;
        const R S[3] = {xb * vl[0] - Bv * Bl[0], xb * vl[1] - Bv * Bl[1], xb * vl[2] - Bv * Bl[2]};
        const R tau = xb - p - R(0.5) * (Bv * Bv + B2 * iW2) - Dd;
        const R pt = p + R(0.5) * b2;
        R Sd;
        if constexpr (D == 0) Sd = m.gi11 * S[0] + m.gi13 * S[2];
        else if constexpr (D == 1) Sd = m.gi22 * S[1];
        else Sd = m.gi13 * S[0] + m.gi33 * S[2];
        const R sg = m.sg, al = m.al;
        const R fac = al * vd - bd;
        U[0] = sg * Dd;
        U[1] = sg * S[0];
        U[2] = sg * S[1];
        U[3] = sg * S[2];
        U[4] = sg * tau;
        U[5] = sg * B[0];
        U[6] = sg * B[1];
        U[7] = sg * B[2];
        U[8] = q[8];
        F[0] = sg * Dd * fac;
        const R cB = B[D] * iW2 + Bv * vd;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const R Wdj = Sd * vl[j] + (j == D ? pt : R(0)) - cB * Bl[j];
            F[1 + j] = sg * (al * Wdj - bd * S[j]);
        }
        F[4] = sg * (al * (Sd - Dd * vd) - bd * tau);
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const R bj = j == 0 ? m.b1 : R(0);
            F[5 + j] = j == D ? R(0) : sg * (fac * B[j] - (al * v[j] - bj) * B[D]);
        }
        F[8] = R(0);
    }
    if constexpr (!WANT_SPEED) return;
    const R cs2 = fdiv(gam * p, rhoh);
    const R ca2 = fdiv(b2, rhoh + b2);
    const R ce2 = cs2 + ca2 - cs2 * ca2;
    const R gdd = D == 0 ? m.gi11 : (D == 1 ? m.gi22 : m.gi33);
    R disc = ce2 * (R(1) - v2) * (gdd * (R(1) - v2 * ce2) - vd * vd * (R(1) - ce2));
    disc = disc > R(0) ? disc : R(0);
    const R sq = fsqrt(disc);
    const R pre = fdiv(m.al, R(1) - v2 * ce2);
    const R c0 = vd * (R(1) - ce2);
    lp = pre * (c0 + sq) - bd;
    lm = pre * (c0 - sq) - bd;
}

// ---------------------------------------------------------------------------------
// Reconstruction: monotonised-central slopes; PPM interface values from MC slopes
// with the two monotonicity constraints (no flattening, no steepening).
// ---------------------------------------------------------------------------------
// median of (a, b, 0): the minmod of a and b
template <typename R>
__device__ __forceinline__ R minmod0(R a, R b)
{
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_fmed3f(a, b, 0.0f);
    else return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// MC slope: zero unless both one-sided differences share a sign, else the one of
// 2|d-|, 2|d+|, |d- + d+|/2 smallest in magnitude, with that common sign.
template <typename R>
__device__ __forceinline__ R mc_slope(R qm, R q0, R qp)
{
    const R dm = q0 - qm, dp = qp - q0;
    return minmod0(minmod0(R(2) * dm, R(2) * dp), R(0.5) * (dm + dp));
}

// PPM interface value between cells a and b from their values and MC slopes
template <typename R>
__device__ __forceinline__ R ppm_iface(R qa, R qb, R sa, R sb)
{
    return R(0.5) * (qa + qb) - (sb - sa) * R(1.0 / 6.0);
}

// PPM monotonicity constraints of a cell with value q and raw face values l, r:
// flat at an extremum, else the face value that would overshoot is moved so that
// the parabola stays monotone
template <typename R>
__device__ __forceinline__ void ppm_limit(R q2, R l, R r, R &qm, R &qp)
{
    const R dq = r - l;
    const R dev = q2 - R(0.5) * (l + r);
    if constexpr (sizeof(R) == 8) {
        // double: as branches, which keep each variable's stencil in a block of its
        // own, so the face kernel fits four waves per SIMD without spilling
        R lc = l, rc = r;
        if ((r - q2) * (q2 - l) <= R(0)) {
            lc = q2;
            rc = q2;
        } else if (dq * dev > dq * dq * R(1.0 / 6.0)) {
            lc = R(3) * q2 - R(2) * r;
        } else if (-(dq * dq) * R(1.0 / 6.0) > dq * dev) {
            rc = R(3) * q2 - R(2) * l;
        }
        qm = lc;
        qp = rc;
    } else {
        // float: as selects (no branches), so the stencil loads of all variables can
        // be scheduled ahead of this arithmetic
        const bool extremum = (r - q2) * (q2 - l) <= R(0);
        const bool fix_l = dq * dev > dq * dq * R(1.0 / 6.0);
        const bool fix_r = -(dq * dq) * R(1.0 / 6.0) > dq * dev;
        qm = extremum ? q2 : (fix_l ? R(3) * q2 - R(2) * r : l);
        qp = extremum ? q2 : (!fix_l && fix_r ? R(3) * q2 - R(2) * l : r);
    }
}

// values at the lower and upper face of the centre cell q[2] of q[0..4]
template <typename R>
__device__ __forceinline__ void ppm_cell(R q0, R q1, R q2, R q3, R q4, R &qm, R &qp)
{
    const R sm = mc_slope(q0, q1, q2), s0 = mc_slope(q1, q2, q3), sp = mc_slope(q2, q3, q4);
    ppm_limit(q2, ppm_iface(q1, q2, sm, s0), ppm_iface(q2, q3, s0, sp), qm, qp);
}

// face i-1/2 from cells q[0..5] = i-3..i+2 (MC reads q[1..4])
template <typename R, int RECON>
__device__ __forceinline__ void recon_face(const R *q, R &qL, R &qR)
{
    if constexpr (RECON == BHAC_RECON_MC) {
        qL = q[2] + R(0.5) * mc_slope(q[1], q[2], q[3]);
        qR = q[3] - R(0.5) * mc_slope(q[2], q[3], q[4]);
    } else {
        R a, b;
        ppm_cell(q[0], q[1], q[2], q[3], q[4], a, qL);
        ppm_cell(q[1], q[2], q[3], q[4], q[5], qR, b);
    }
}

// ---------------------------------------------------------------------------------
// Face flux: exact (B~_normal, psi) GLM solve, then HLL or TVDLF. Returns the
// largest |lambda| of both states. qL/qR are modified (normal field replaced).
// ---------------------------------------------------------------------------------
// One pass: both face states fully evaluated once, then combined (more live
// registers than face_flux_lean, fewer instructions). CT: constrained transport, the
// caller has set both states' normal field from the face field; no GLM solve, the
// normal-field and psi fluxes vanish.
template <typename R, int D, int FLUX, bool CT = false>
__device__ __forceinline__ R face_flux(R *qL, R *qR, const FaceM<R> &m, R ch, R gam, R gfac, R *F)
{
    R bstar = R(0), psistar = R(0);
    if constexpr (!CT) {
        const R sg = m.sg;
        const R btl = sg * qL[5 + D], btr = sg * qR[5 + D];
        bstar = R(0.5) * (btl + btr) - fdiv(qR[8] - qL[8], R(2) * ch);
        psistar = R(0.5) * (qL[8] + qR[8]) - R(0.5) * ch * (btr - btl);
        const R bn = fdiv(bstar, sg);
        qL[5 + D] = bn;
        qR[5 + D] = bn;
    }
    R UL[NV], FL[NV], UR[NV], FR[NV], lmL, lpL, lmR, lpR;
    face_state<R, D, true, true>(qL, m, gam, gfac, UL, FL, lmL, lpL);
    face_state<R, D, true, true>(qR, m, gam, gfac, UR, FR, lmR, lpR);
    if constexpr (FLUX == BHAC_FLUX_HLL) {
        R sr = lpL > lpR ? lpL : lpR;
        sr = sr > R(0) ? sr : R(0);
        R sl = lmL < lmR ? lmL : lmR;
        sl = sl < R(0) ? sl : R(0);
        if constexpr (sizeof(R) == 8) {
            // double: a branch (fewer live registers than computing both forms)
            if (sr == sl) {
#pragma unroll
                for (int v = 0; v < 8; v++) F[v] = R(0.5) * (FL[v] + FR[v]);
            } else {
                const R inv = frcp(sr - sl);
                const R srsl = sr * sl;
#pragma unroll
                for (int v = 0; v < 8; v++) F[v] = (sr * FL[v] - sl * FR[v] + srsl * (UR[v] - UL[v])) * inv;
            }
        } else {
            const bool same = sr == sl;      // both bounds zero: the central average
            const R inv = frcp(same ? R(1) : sr - sl);
            const R srsl = sr * sl;
#pragma unroll
            for (int v = 0; v < 8; v++) {
                const R hll = (sr * FL[v] - sl * FR[v] + srsl * (UR[v] - UL[v])) * inv;
                F[v] = same ? R(0.5) * (FL[v] + FR[v]) : hll;
            }
        }
    } else {
        R c = fabs(lmL);
        c = fabs(lpL) > c ? fabs(lpL) : c;
        c = fabs(lmR) > c ? fabs(lmR) : c;
        c = fabs(lpR) > c ? fabs(lpR) : c;
#pragma unroll
        for (int v = 0; v < 8; v++) F[v] = R(0.5) * (FL[v] + FR[v]) - R(0.5) * c * (UR[v] - UL[v]);
    }
    F[5 + D] = psistar;
    F[8] = CT ? R(0) : ch * ch * bstar;
    R lam = fabs(lmL);
    lam = fabs(lpL) > lam ? fabs(lpL) : lam;
    lam = fabs(lmR) > lam ? fabs(lmR) : lam;
    lam = fabs(lpR) > lam ? fabs(lpR) : lam;
    return lam;
}

template <typename R, int D, int FLUX>
__device__ __forceinline__ R face_flux_lean(R *qL, R *qR, const FaceM<R> &m, R ch, R gam, R gfac, R *F)
{
    const R sg = m.sg;
    const R btl = sg * qL[5 + D], btr = sg * qR[5 + D];
    const R bstar = R(0.5) * (btl + btr) - fdiv(qR[8] - qL[8], R(2) * ch);
    const R psistar = R(0.5) * (qL[8] + qR[8]) - R(0.5) * ch * (btr - btl);
    const R bn = fdiv(bstar, sg);
    qL[5 + D] = bn;
    qR[5 + D] = bn;
    // wave-speed bounds of both states first; then each state's U and F are folded
    // into F = cL F_L + cR F_R + cU (U_R - U_L) one state at a time (few live registers)
    R dummy[NV], lmL, lpL, lmR, lpR;
    face_state<R, D, false>(qL, m, gam, gfac, dummy, dummy, lmL, lpL);
    face_state<R, D, false>(qR, m, gam, gfac, dummy, dummy, lmR, lpR);
    R cL, cR, cU;
    if constexpr (FLUX == BHAC_FLUX_HLL) {
        R sr = lpL > lpR ? lpL : lpR;
        sr = sr > R(0) ? sr : R(0);
        R sl = lmL < lmR ? lmL : lmR;
        sl = sl < R(0) ? sl : R(0);
        if (sr == sl) {
            cL = R(0.5);
            cR = R(0.5);
            cU = R(0);
        } else {
            const R inv = frcp(sr - sl);
            cL = sr * inv;
            cR = -sl * inv;
            cU = sr * sl * inv;
        }
    } else {
        R c = fabs(lmL);
        c = fabs(lpL) > c ? fabs(lpL) : c;
        c = fabs(lmR) > c ? fabs(lmR) : c;
        c = fabs(lpR) > c ? fabs(lpR) : c;
        cL = R(0.5);
        cR = R(0.5);
        cU = R(-0.5) * c;
    }
    {
        R U[NV], Fs[NV], a, b;
        face_state<R, D, true>(qL, m, gam, gfac, U, Fs, a, b);
#pragma unroll
        for (int v = 0; v < 8; v++) F[v] = cL * Fs[v] - cU * U[v];
    }
    {
        R U[NV], Fs[NV], a, b;
        face_state<R, D, true>(qR, m, gam, gfac, U, Fs, a, b);
#pragma unroll
        for (int v = 0; v < 8; v++) F[v] += cR * Fs[v] + cU * U[v];
    }
    F[5 + D] = psistar;
    F[8] = ch * ch * bstar;
    R lam = fabs(lmL);
    lam = fabs(lpL) > lam ? fabs(lpL) : lam;
    lam = fabs(lmR) > lam ? fabs(lmR) : lam;
    lam = fabs(lpR) > lam ? fabs(lpR) : lam;
    return lam;
}

// ---------------------------------------------------------------------------------
// Primitive -> conserved at a cell centre (double).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void prim_to_cons(const double *q, const CentM &m, double gfac, double *U)
{
    const double u1 = q[1], u2 = q[2], u3 = q[3];
    const double ul1 = m.g11 * u1 + m.g13 * u3, ul2 = m.g22 * u2, ul3 = m.g13 * u1 + m.g33 * u3;
    const double W = sqrt(1.0 + (u1 * ul1 + u2 * ul2 + u3 * ul3));
    const double iW = 1.0 / W;
    const double vl[3] = {ul1 * iW, ul2 * iW, ul3 * iW};
    const double B[3] = {q[5], q[6], q[7]};
    const double Bl[3] = {m.g11 * B[0] + m.g13 * B[2], m.g22 * B[1], m.g13 * B[0] + m.g33 * B[2]};
    const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
    const double Bv = B[0] * vl[0] + B[1] * vl[1] + B[2] * vl[2];
    const double rho = q[0], p = q[4];
    const double xi = (rho + gfac * p) * W * W;
    const double Dd = rho * W;
    const double xb = xi + B2;
    const double sg = m.sg;
    U[0] = sg * Dd;
    for (int i = 0; i < 3; i++) U[1 + i] = sg * (xb * vl[i] - Bv * Bl[i]);
    U[4] = sg * (xb - p - 0.5 * (Bv * Bv + B2 * iW * iW) - Dd);
    for (int i = 0; i < 3; i++) U[5 + i] = sg * B[i];
    U[8] = q[8];
}

// ---------------------------------------------------------------------------------
// Geometric sources of the stationary metric (3+1 form with metric derivatives)
// and GLM damping. Conserved D, S_j, tau from U; velocity, pressure and field
// from the primitives. Only x1 and x2 derivatives exist.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void geometric_sources(const double *q, const double *U, const CentM &m, double kappa,
                                                  double *S)
{
    const double isg = rcp_nr(m.sg);
    const double D = U[0] * isg, tau = U[4] * isg;
    const double Sl1 = U[1] * isg, Sl2 = U[2] * isg, Sl3 = U[3] * isg;
    const double Su[3] = {m.gi11 * Sl1 + m.gi13 * Sl3, m.gi22 * Sl2, m.gi13 * Sl1 + m.gi33 * Sl3};
    const double u1 = q[1], u2 = q[2], u3 = q[3];
    const double ul1 = m.g11 * u1 + m.g13 * u3, ul2 = m.g22 * u2, ul3 = m.g13 * u1 + m.g33 * u3;
    const double iW = rsqrt_nr(1.0 + (u1 * ul1 + u2 * ul2 + u3 * ul3)), iW2 = iW * iW;
    const double v[3] = {u1 * iW, u2 * iW, u3 * iW};
    const double B[3] = {q[5], q[6], q[7]};
    const double Bl[3] = {m.g11 * B[0] + m.g13 * B[2], m.g22 * B[1], m.g13 * B[0] + m.g33 * B[2]};
    const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
    const double Bv = (B[0] * ul1 + B[1] * ul2 + B[2] * ul3) * iW;
    const double pt = q[4] + 0.5 * (B2 * iW2 + Bv * Bv);
    // W^{ik} = S^i v^k + p_t gamma^{ik} - (B^i/W^2 + (B.v) v^i) B^k
    double c[3];
    for (int i = 0; i < 3; i++) c[i] = B[i] * iW2 + Bv * v[i];
    const double W11 = Su[0] * v[0] + pt * m.gi11 - c[0] * B[0];
    const double W13 = Su[0] * v[2] + pt * m.gi13 - c[0] * B[2];
    const double W31 = Su[2] * v[0] + pt * m.gi13 - c[2] * B[0];
    const double W22 = Su[1] * v[1] + pt * m.gi22 - c[1] * B[1];
    const double W33 = Su[2] * v[2] + pt * m.gi33 - c[2] * B[2];
    const double W21 = Su[1] * v[0] - c[1] * B[0];
    const double W23 = Su[1] * v[2] - c[1] * B[2];
    // contractions with d_j gamma_ik for j = 1, 2
    const double X1 = W11 * m.dg11_1 + (W13 + W31) * m.dg13_1 + W22 * m.dg22_1 + W33 * m.dg33_1;
    const double X2 = W11 * m.dg11_2 + (W13 + W31) * m.dg13_2 + W22 * m.dg22_2 + W33 * m.dg33_2;
    const double E = tau + D;
    S[0] = 0.0;
    S[1] = m.sg * (0.5 * m.al * X1 + Sl1 * m.db1 - E * m.da1);
    S[2] = m.sg * (0.5 * m.al * X2 + Sl1 * m.db2 - E * m.da2);
    S[3] = 0.0;
    // W^j_1 = W^{j1} gamma_11 + W^{j3} gamma_31
    const double Wm11 = W11 * m.g11 + W13 * m.g13;
    const double Wm21 = W21 * m.g11 + W23 * m.g13;
    S[4] = m.sg * (0.5 * m.b1 * X1 + Wm11 * m.db1 + Wm21 * m.db2 - (Su[0] * m.da1 + Su[1] * m.da2));
    S[5] = S[6] = S[7] = 0.0;
    S[8] = -kappa * U[8];
}

// ---------------------------------------------------------------------------------
// Conserved -> primitive: 1-D Newton on xi = rho h W^2 with a safeguard, floors and
// a backup (keep the guess). Returns 1 on failure.
// ---------------------------------------------------------------------------------
struct C2PSys {
    double D, E, S2, B2, SB, SB2, gfac_inv;
};

__device__ __forceinline__ double c2p_vsq(const C2PSys &c, double xi)
{
    const double xb = xi + c.B2;
    return (xi * xi * c.S2 + c.SB2 * (c.B2 + 2.0 * xi)) * rcp_nr(xi * xi * xb * xb);
}

__device__ __forceinline__ double c2p_newton_step(const C2PSys &c, double xi)
{
    const double xb = xi + c.B2;
    const double ixi = rcp_nr(xi), ixb = rcp_nr(xb);
    const double ixi2 = ixi * ixi, ixb2 = ixb * ixb;
    const double v2 = (xi * xi * c.S2 + c.SB2 * (c.B2 + 2.0 * xi)) * ixi2 * ixb2;
    const double w2inv = 1.0 - v2;
    const double iW = w2inv * rsqrt_nr(w2inv);      // 1/W = sqrt(1 - v^2)
    const double W = rsqrt_nr(w2inv);
    const double p = c.gfac_inv * (xi * w2inv - c.D * iW);
    const double f = xi - p + c.B2 - 0.5 * (c.B2 * w2inv + c.SB2 * ixi2) - c.E;
    const double dv2 = -2.0 * c.S2 * ixb2 * ixb
                       - 2.0 * c.SB2 * (3.0 * xi * xi + 3.0 * xi * c.B2 + c.B2 * c.B2) * ixi2 * ixi * ixb2 * ixb;
    const double dp = c.gfac_inv * (w2inv + (0.5 * c.D * W - xi) * dv2);
    const double df = 1.0 - dp + 0.5 * c.B2 * dv2 + c.SB2 * ixi2 * ixi;
    double xn = xi - f * rcp_nr(df);
    for (int h = 0; h < 64 && (xn <= 0.0 || c2p_vsq(c, xn) >= 1.0); h++) xn = 0.5 * (xn + xi);
    if (xn <= 0.0 || !(c2p_vsq(c, xn) < 1.0)) return __builtin_nan("");
    return xn;
}

// Entropy backup of the inversion (entropy field carried, rows 9 of U and P).
// With p = K rho^gamma and rho = D / W the enthalpy density is a function of W:
//   xi(W) = D W + Gamma/(Gamma-1) K D^Gamma W^(2-Gamma),
// and the momentum relation leaves the one equation
//   f(W) = (xi + B^2)^2 (1 - W^-2) - (S.B)^2 (2 xi + B^2) / xi^2 - S^2 = 0,
// whose left side grows with W for Gamma <= 2 (f(1) <= 0): one root on [1, inf).
// Newton steps in W inside a bracket that every evaluation narrows; a step that
// leaves the bracket is replaced by the bracket's midpoint.
constexpr int ENT_MAXIT = 100;

__device__ __forceinline__ void ent_eval(const C2PSys &c, double KDg, double gam, double W, double &xi, double &f,
                                         double &df)
{
    const double Wp = pow(W, 1.0 - gam);            // W^(1-Gamma)
    xi = c.D * W + KDg * (W * Wp);
    const double dxi = c.D + KDg * (2.0 - gam) * Wp;
    const double xb = xi + c.B2, iW = 1.0 / W, w2i = iW * iW, ixi = 1.0 / xi;
    const double ixi2 = ixi * ixi;
    f = xb * xb * (1.0 - w2i) - c.SB2 * (2.0 * xi + c.B2) * ixi2 - c.S2;
    df = 2.0 * xb * dxi * (1.0 - w2i) + 2.0 * xb * xb * w2i * iW + c.SB2 * dxi * (2.0 * ixi2 + 2.0 * c.B2 * ixi2 * ixi);
}

// Inlined: as a call, the update kernel kept a scratch stack frame for it and moved
// 12-20 % slower, although the root is taken in few cells.
__device__ __forceinline__ bool ent_root(const C2PSys &c, double K, double gam, double gfac, double Wg, double tol,
                                         double &W, double &xi)
{
    const double KDg = gfac * K * pow(c.D, gam);
    double f, df, lo = 1.0, hi = 2.0;
    ent_eval(c, KDg, gam, hi, xi, f, df);
    for (int n = 0; n < 60 && f < 0.0; n++) {
        lo = hi;
        hi *= 2.0;
        ent_eval(c, KDg, gam, hi, xi, f, df);
    }
    if (!(f >= 0.0)) return false;
    W = (Wg > lo && Wg < hi) ? Wg : 0.5 * (lo + hi);
    for (int it = 0; it < ENT_MAXIT; it++) {
        ent_eval(c, KDg, gam, W, xi, f, df);
        if (!isfinite(f) || !isfinite(df)) return false;
        if (f == 0.0) return true;
        if (f < 0.0) lo = W;
        else hi = W;
        double Wn = W - f / df;
        if (!(Wn > lo && Wn < hi)) Wn = 0.5 * (lo + hi);
        const bool done = fabs(Wn - W) <= tol * Wn;
        W = Wn;
        if (done) {
            ent_eval(c, KDg, gam, W, xi, f, df);
            return true;
        }
    }
    return false;
}

// U: conserved (densitised); g: guess primitives; out: primitives. nit: steps taken.
// ENT: the entropy field is carried (U[9] = U[0] K, P[9] = K); where the energy
// inversion fails the entropy root is taken instead and `backup` is set.
template <bool ENT = false>
__device__ __forceinline__ int con_to_prim(const double *U, const double *g, const CentM &m, const KParams &kp,
                                           double *out, int &nit, int &floored, int &backup)
{
    nit = 0;
    floored = 0;
    backup = 0;
    const double isg = rcp_nr(m.sg);
    C2PSys c;
    c.gfac_inv = kp.gfac_inv;
    c.D = U[0] * isg;
    const double Sl[3] = {U[1] * isg, U[2] * isg, U[3] * isg};
    const double B[3] = {U[5] * isg, U[6] * isg, U[7] * isg};
    c.E = U[4] * isg + c.D;
    const double Su[3] = {m.gi11 * Sl[0] + m.gi13 * Sl[2], m.gi22 * Sl[1], m.gi13 * Sl[0] + m.gi33 * Sl[2]};
    c.S2 = Sl[0] * Su[0] + Sl[1] * Su[1] + Sl[2] * Su[2];
    const double Bl[3] = {m.g11 * B[0] + m.g13 * B[2], m.g22 * B[1], m.g13 * B[0] + m.g33 * B[2]};
    c.B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
    c.SB = Sl[0] * B[0] + Sl[1] * B[1] + Sl[2] * B[2];
    c.SB2 = c.SB * c.SB;
    bool fail = !(c.D > 0.0) || !isfinite(c.E) || !isfinite(c.S2) || !isfinite(c.B2);
    double xi = 0.0;
    if (!fail) {
        // initial guess xi = rho h W^2 of the guess state
        const double u1 = g[1], u2 = g[2], u3 = g[3];
        const double usq = u1 * (m.g11 * u1 + m.g13 * u3) + u2 * m.g22 * u2 + u3 * (m.g13 * u1 + m.g33 * u3);
        xi = (g[0] + kp.gfac * g[4]) * (1.0 + usq);
        if (!(xi > 0.0) || !isfinite(xi)) xi = c.E > c.D ? c.E : c.D;
        for (int r = 0; r < 200 && c2p_vsq(c, xi) >= 1.0; r++) xi *= 2.0;
        fail = !(c2p_vsq(c, xi) < 1.0);
    }
    if (!fail) {
        bool conv = false;
        int it = 0;
        while (it < kp.c2p_maxit) {
            const double xn = c2p_newton_step(c, xi);
            it++;
            if (!isfinite(xn)) { fail = true; break; }
            const bool done = fabs(xn - xi) <= kp.c2p_tol * xn;
            xi = xn;
            if (done) { conv = true; break; }
        }
        if (!fail && !conv) fail = true;
        if (!fail) {
            xi = c2p_newton_step(c, xi);
            it++;
            if (!isfinite(xi)) fail = true;
        }
        nit = it;
    }
    double rho = 0.0, p = 0.0, W = 1.0;
    if (!fail) {
        const double v2 = c2p_vsq(c, xi);
        if (!(v2 < 1.0)) fail = true;
        else {
            const double w2inv = 1.0 - v2;
            W = rsqrt_nr(w2inv);
            rho = c.D * (w2inv * W);
            p = c.gfac_inv * (xi * w2inv - rho);
            if (!(rho > 0.0) || !(p >= 0.0) || !isfinite(rho) || !isfinite(p)) fail = true;
        }
    }
    if constexpr (ENT) {
        if (fail) {
            const double K = U[9] / U[0];
            if (c.D > 0.0 && K > 0.0 && isfinite(K) && isfinite(c.S2) && isfinite(c.B2)) {
                const double u1 = g[1], u2 = g[2], u3 = g[3];
                const double Wg =
                    sqrt(1.0 + (u1 * (m.g11 * u1 + m.g13 * u3) + u2 * m.g22 * u2 + u3 * (m.g13 * u1 + m.g33 * u3)));
                double Wb, xib;
                if (ent_root(c, K, kp.gam, kp.gfac, Wg, kp.c2p_tol, Wb, xib)) {
                    const double rb = c.D / Wb, pb = K * pow(rb, kp.gam);
                    if (rb > 0.0 && pb >= 0.0 && isfinite(rb) && isfinite(pb) && xib > 0.0) {
                        W = Wb;
                        xi = xib;
                        rho = rb;
                        p = pb;
                        fail = false;
                        backup = 1;
                    }
                }
            }
        }
    }
    if (fail) {
        for (int v = 0; v < NV + (ENT ? 1 : 0); v++) out[v] = g[v];
        return 1;
    }
    const double ixb = rcp_nr(xi + c.B2), sbx = c.SB * rcp_nr(xi);
    const double vl[3] = {(Sl[0] + sbx * Bl[0]) * ixb, (Sl[1] + sbx * Bl[1]) * ixb, (Sl[2] + sbx * Bl[2]) * ixb};
    double ut[3] = {W * (m.gi11 * vl[0] + m.gi13 * vl[2]), W * (m.gi22 * vl[1]), W * (m.gi13 * vl[0] + m.gi33 * vl[2])};
    if (rho < kp.rho_floor) { rho = kp.rho_floor; floored = 1; }
    if (p < kp.p_floor) { p = kp.p_floor; floored = 1; }
    if (W > kp.w_max) {
        const double f = sqrt(kp.w_max * kp.w_max - 1.0) / sqrt(W * W - 1.0);
        ut[0] *= f;
        ut[1] *= f;
        ut[2] *= f;
        floored = 1;
    }
    out[0] = rho;
    out[1] = ut[0];
    out[2] = ut[1];
    out[3] = ut[2];
    out[4] = p;
    out[5] = B[0];
    out[6] = B[1];
    out[7] = B[2];
    out[8] = U[8];
    if constexpr (ENT) out[9] = U[9] / U[0];
    return 0;
}

// ---------------------------------------------------------------------------------
// Global maxima kept by many work-groups: read the current value first and only
// issue the atomic when this work-group raises it (thousands of same-address
// atomics per launch would otherwise serialise at one L2 channel).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void raise_max(unsigned long long *acc, double v)
{
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    if (bits > __hip_atomic_load(acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(acc, bits);
}
__device__ __forceinline__ void raise_max(int *acc, int v)
{
    if (v > __hip_atomic_load(acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(acc, v);
}

// ---------------------------------------------------------------------------------
// Work-group reductions (wave64 shuffles, then LDS across the 4 waves).
// ---------------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double wg_max(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; i++) r = red[i] > r ? red[i] : r;
    return r;
}

template <int NT>
__device__ __forceinline__ long long wg_sum(long long v, long long *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    long long r = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) r += red[i];
    return r;
}

template <int NT>
__device__ __forceinline__ int wg_imax(int v, int *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    int r = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; i++) r = red[i] > r ? red[i] : r;
    return r;
}

}  // namespace bhac
