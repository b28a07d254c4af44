// Block-tiled substep for gfx950 (mixed precision, PPM): no separate ghost fill.
//
// k_block_flux: one work-group (256 threads = 4 wave64) per block. Thread (i, j)
// owns one column of the block and marches along x3 (phi), plane by plane:
//   - the plane's cells plus their x1/x2 halo (gathered from the same-level
//     neighbour blocks' interiors through the halo tables) are staged in LDS;
//   - MC slopes, PPM interface values and the monotonicity constraints are
//     computed once per cell and direction (LDS for x1/x2, a rolling register
//     window for x3), instead of twice per face;
//   - face fluxes (GLM + HLL/TVDLF) for the x1 and x2 faces go through LDS, the x3
//     face stays in registers and is carried to the next plane;
//   - the flux divergence of every interior cell is written once (FP32).
// k_update_div: one thread per cell adds the FP64 sources, does the compensated RK
// combine and the FP64 inversion.
//
// Work-group -> block mapping is XCD-aware: consecutive blocks (neighbours along
// phi, which share metric-table rows) are handed to the same XCD so its L2 holds
// those rows.
#include <hip/hip_runtime.h>

#include "compensated.h"
#include "physics.h"

namespace bhac {

constexpr int FSM = 16;            // largest block edge along x1 and x2
constexpr int FG = 3;              // halo width read by PPM
constexpr int TWX = FSM + 2 * FG;  // staged row length along x1
constexpr int FWG = 256;           // threads per work-group

// LDS carve-up, in floats.
struct Lay {
    static constexpr int XS = 0;                                  // plane rows with x1 halo [NV][FSM][TWX]
    static constexpr int YH = XS + NV * FSM * TWX;                // x2 halo rows        [NV][2*FG][FSM]
    static constexpr int SX = YH + NV * 2 * FG * FSM;             // x1 slopes, i in [-2, s0+1]  [NV][FSM][FSM+4]
    static constexpr int SY = SX + NV * FSM * (FSM + 4);          // x2 slopes, j in [-2, s1+1]  [NV][FSM+4][FSM]
    static constexpr int QX = SY + NV * (FSM + 4) * FSM;          // x1 face values, i in [-1, s0] [2][NV][FSM][FSM+2]
    static constexpr int QY = QX + 2 * NV * FSM * (FSM + 2);      // x2 face values, j in [-1, s1] [2][NV][FSM+2][FSM]
    static constexpr int TOTAL = QY + 2 * NV * (FSM + 2) * FSM;
    static constexpr int FX = 0;                                  // x1 fluxes [NV][FSM][FSM+1] (reuses XS..SY)
    static constexpr int FY = FX + NV * FSM * (FSM + 1);          // x2 fluxes [NV][FSM+1][FSM]
};
static_assert(Lay::FY + NV * (FSM + 1) * FSM <= Lay::QX, "flux buffers must not overlap the face values");
static_assert(Lay::TOTAL * 4 <= 81920, "two work-groups must fit in 160 KB of LDS");

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Padded index of local cell (li, lj, lk) of block b as the same-level ghost rule
// defines it: inside the block, itself; outside, the neighbour's interior cell or
// the own block's nearest interior cell.
__device__ __forceinline__ long long gather_index(const GridDev &gd, const KParams &kp, int b, const DevBlock &B,
                                                  int li, int lj, int lk)
{
    const HaloAxis *h = gd.halo + (size_t)b * 3 * gd.hmax;
    const HaloAxis hx = h[li + kp.g[0]];
    const HaloAxis hy = h[gd.hmax + lj + kp.g[1]];
    const HaloAxis hz = h[2 * gd.hmax + lk + kp.g[2]];
    const int nbk = gd.nbr[(size_t)b * 27 + (hx.dir + 1) + 3 * (hy.dir + 1) + 9 * (hz.dir + 1)];
    long long off;
    int si, sj, sk;
    if (nbk >= 0) {
        off = gd.blocks[nbk].off;
        si = hx.src;
        sj = hy.src;
        sk = hz.src;
    } else {
        off = B.off;
        si = clampi(li, 0, B.s[0] - 1);
        sj = clampi(lj, 0, B.s[1] - 1);
        sk = clampi(lk, 0, B.s[2] - 1);
    }
    return off + ((long long)sk * B.n1 + sj) * B.n0 + si;
}

__device__ __forceinline__ void load_cell(const float *__restrict__ P, long long ncp, long long c, float *q)
{
#pragma unroll
    for (int v = 0; v < NV; v++) q[v] = P[v * ncp + c];
}

// PPM: interface value between cells a and b from their values and MC slopes
__device__ __forceinline__ float iface(float qa, float qb, float sa, float sb)
{
    return 0.5f * (qa + qb) - (sb - sa) * (1.0f / 6.0f);
}

// PPM monotonicity constraints for a cell with value q and raw face values l, r
__device__ __forceinline__ void ppm_limit(float q, float &l, float &r)
{
    const float dq = r - l;
    const float dev = q - 0.5f * (l + r);
    if ((r - q) * (q - l) <= 0.0f) {
        l = q;
        r = q;
    } else if (dq * dev > dq * dq * (1.0f / 6.0f)) {
        l = 3.0f * q - 2.0f * r;
    } else if (-(dq * dq) * (1.0f / 6.0f) > dq * dev) {
        r = 3.0f * q - 2.0f * l;
    }
}

template <int FLUX, bool KS>
__global__ __launch_bounds__(FWG, 2) void k_block_flux(KParams kp, GridDev gd, int nblocks, int per_xcd,
                                                       const float *__restrict__ P, float *__restrict__ dU,
                                                       long long nci)
{
    __shared__ float sm[Lay::TOTAL];
    __shared__ double red[FWG / 64];
    const int w = blockIdx.x;
    const int b = (w % NXCD) * per_xcd + w / NXCD;
    if (b >= nblocks) return;                     // uniform over the work-group
    const DevBlock B = gd.blocks[b];
    const int s0 = B.s[0], s1 = B.s[1], s2 = B.s[2];
    const int t = threadIdx.x;
    const bool own = t < s0 * s1;
    const int i = own ? t % s0 : 0, j = own ? t / s0 : 0;
    const long long ncp = kp.ncp;
    const float gam = (float)kp.gam, gfac = (float)kp.gfac;
    const float ch = (float)gd.st->ch;
    const float idx0 = (float)gd.levels[B.level].inv_dx[0], idx1 = (float)gd.levels[B.level].inv_dx[1],
                idx2 = (float)gd.levels[B.level].inv_dx[2];

    float *XS = sm + Lay::XS, *YH = sm + Lay::YH, *SX = sm + Lay::SX, *SY = sm + Lay::SY;
    float *QX = sm + Lay::QX, *QY = sm + Lay::QY, *FXb = sm + Lay::FX, *FYb = sm + Lay::FY;
    auto xs = [&](int v, int jj, int ii) -> float & { return XS[(v * FSM + jj) * TWX + ii + FG]; };
    auto ty = [&](int v, int ii, int jj) -> float {   // plane value at (ii in [0,s0), jj in [-3, s1+3))
        if (jj >= 0 && jj < s1) return XS[(v * FSM + jj) * TWX + ii + FG];
        const int r = jj < 0 ? jj + FG : jj - s1 + FG;
        return YH[(v * 2 * FG + r) * FSM + ii];
    };
    auto sx = [&](int v, int jj, int ii) -> float & { return SX[(v * FSM + jj) * (FSM + 4) + ii + 2]; };
    auto sy = [&](int v, int jj, int ii) -> float & { return SY[(v * (FSM + 4) + jj + 2) * FSM + ii]; };
    auto qx = [&](int side, int v, int jj, int ii) -> float & {
        return QX[((side * NV + v) * FSM + jj) * (FSM + 2) + ii + 1];
    };
    auto qy = [&](int side, int v, int jj, int ii) -> float & {
        return QY[((side * NV + v) * (FSM + 2) + jj + 1) * FSM + ii];
    };
    auto fx = [&](int v, int jj, int ii) -> float & { return FXb[(v * FSM + jj) * (FSM + 1) + ii]; };
    auto fy = [&](int v, int jj, int ii) -> float & { return FYb[(v * (FSM + 1) + jj) * FSM + ii]; };

    // x3 register window of the own column: q_k, q_{k+1}, q_{k+2}, slope of k+1,
    // interface k+1/2, upper face value of cell k, flux through face k-1/2
    float qk[NV], q1[NV], q2[NV], sg1[NV], ih[NV], qp[NV], fzp[NV];
    float lam0 = 0.0f, lam1 = 0.0f, lam2 = 0.0f;
    FaceM<float> mz;
    if (own) {
        mz = face_metric<float, 2, KS>(gd, B, i, j);
        float w[6][NV];
#pragma unroll
        for (int m = 0; m < 6; m++) {
            const int lk = m - 3;
            const long long c = (lk >= 0 && lk < s2)
                                    ? B.off + ((long long)lk * B.n1 + j) * B.n0 + i
                                    : gather_index(gd, kp, b, B, i, j, lk);
            load_cell(P, ncp, c, w[m]);
        }
        float qmL[NV], qpL[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const float sa = mc_slope(w[0][v], w[1][v], w[2][v]);   // cell -2
            const float sb = mc_slope(w[1][v], w[2][v], w[3][v]);   // cell -1
            const float sc = mc_slope(w[2][v], w[3][v], w[4][v]);   // cell 0
            const float sd = mc_slope(w[3][v], w[4][v], w[5][v]);   // cell 1
            float l = iface(w[1][v], w[2][v], sa, sb), r = iface(w[2][v], w[3][v], sb, sc);
            ppm_limit(w[2][v], l, r);
            qpL[v] = r;                                               // upper face value of cell -1
            float l0 = iface(w[2][v], w[3][v], sb, sc), r0 = iface(w[3][v], w[4][v], sc, sd);
            ih[v] = r0;
            ppm_limit(w[3][v], l0, r0);
            qmL[v] = l0;
            qp[v] = r0;
            qk[v] = w[3][v];
            q1[v] = w[4][v];
            q2[v] = w[5][v];
            sg1[v] = sd;
        }
        lam2 = fmaxf(lam2, face_flux_lean<float, 2, FLUX>(qpL, qmL, mz, ch, gam, gfac, fzp));
    }

    const int nhx = 6 * s1, nhy = 6 * s0;
    // the one halo cell this thread stages on every plane (if any)
    const bool hal = t < nhx + nhy;
    int hi = 0, hj = 0;
    if (hal) {
        if (t < nhx) {
            const int side = t / (3 * s1), r = t % (3 * s1);
            hi = side ? s0 + r / s1 : -FG + r / s1;
            hj = r % s1;
        } else {
            const int u = t - nhx, side = u / (3 * s0), r = u % (3 * s0);
            hj = side ? s1 + r / s0 : -FG + r / s0;
            hi = r % s0;
        }
    }
    auto own_index = [&](int lk) -> long long {
        return (lk >= 0 && lk < s2) ? B.off + ((long long)lk * B.n1 + j) * B.n0 + i
                                    : gather_index(gd, kp, b, B, i, j, lk);
    };
    // loads for plane 0 (prefetched one plane ahead from here on)
    float nq3[NV], nh[NV];
    if (own) load_cell(P, ncp, own_index(3), nq3);
    if (hal) load_cell(P, ncp, gather_index(gd, kp, b, B, hi, hj, 0), nh);

    for (int k = 0; k < s2; k++) {
        // ---- stage the plane and its x1/x2 halo in LDS; prefetch the next plane's cells
        float q3[NV];
        if (own) {
#pragma unroll
            for (int v = 0; v < NV; v++) {
                q3[v] = nq3[v];
                xs(v, j, i) = qk[v];
            }
            if (k + 1 < s2) load_cell(P, ncp, own_index(k + 4), nq3);
        }
        if (hal) {
            if (t < nhx) {
#pragma unroll
                for (int v = 0; v < NV; v++) xs(v, hj, hi) = nh[v];
            } else {
                const int r = hj < 0 ? hj + FG : hj - s1 + FG;
#pragma unroll
                for (int v = 0; v < NV; v++) YH[(v * 2 * FG + r) * FSM + hi] = nh[v];
            }
            if (k + 1 < s2) load_cell(P, ncp, gather_index(gd, kp, b, B, hi, hj, k + 1), nh);
        }
        __syncthreads();

        // ---- MC slopes along x1 (i in [-2, s0+1]) and x2 (j in [-2, s1+1])
        if (own) {
#pragma unroll 1
            for (int v = 0; v < NV; v++) {
                sx(v, j, i) = mc_slope(xs(v, j, i - 1), xs(v, j, i), xs(v, j, i + 1));
                sy(v, j, i) = mc_slope(ty(v, i, j - 1), ty(v, i, j), ty(v, i, j + 1));
            }
        }
        if (t < 4 * (s0 + s1)) {
            if (t < 4 * s1) {
                const int c = t / s1, jj = t % s1;
                const int ii = c < 2 ? c - 2 : s0 + c - 2;
#pragma unroll 1
                for (int v = 0; v < NV; v++) sx(v, jj, ii) = mc_slope(xs(v, jj, ii - 1), xs(v, jj, ii), xs(v, jj, ii + 1));
            } else {
                const int u = t - 4 * s1, c = u / s0, ii = u % s0;
                const int jj = c < 2 ? c - 2 : s1 + c - 2;
#pragma unroll 1
                for (int v = 0; v < NV; v++) sy(v, jj, ii) = mc_slope(ty(v, ii, jj - 1), ty(v, ii, jj), ty(v, ii, jj + 1));
            }
        }
        __syncthreads();

        // ---- PPM face values per cell: x1 for i in [-1, s0], x2 for j in [-1, s1]
        auto recon_x = [&](int jj, int ii) {
#pragma unroll 1
            for (int v = 0; v < NV; v++) {
                const float q = xs(v, jj, ii);
                float l = iface(xs(v, jj, ii - 1), q, sx(v, jj, ii - 1), sx(v, jj, ii));
                float r = iface(q, xs(v, jj, ii + 1), sx(v, jj, ii), sx(v, jj, ii + 1));
                ppm_limit(q, l, r);
                qx(0, v, jj, ii) = l;
                qx(1, v, jj, ii) = r;
            }
        };
        auto recon_y = [&](int jj, int ii) {
#pragma unroll 1
            for (int v = 0; v < NV; v++) {
                const float q = ty(v, ii, jj);
                float l = iface(ty(v, ii, jj - 1), q, sy(v, jj - 1, ii), sy(v, jj, ii));
                float r = iface(q, ty(v, ii, jj + 1), sy(v, jj, ii), sy(v, jj + 1, ii));
                ppm_limit(q, l, r);
                qy(0, v, jj, ii) = l;
                qy(1, v, jj, ii) = r;
            }
        };
        if (own) {
            recon_x(j, i);
            recon_y(j, i);
        }
        if (t < 2 * (s0 + s1)) {
            if (t < 2 * s1) recon_x(t % s1, t < s1 ? -1 : s0);
            else {
                const int u = t - 2 * s1;
                recon_y(u < s0 ? -1 : s1, u % s0);
            }
        }
        __syncthreads();

        // ---- face fluxes: x1 faces i in [0, s0], x2 faces j in [0, s1] (through LDS),
        // then the own x3 face k+1/2 (registers). The flux buffers overwrite the staged
        // plane and the slopes, last read before the barrier above.
        // (the face-metric rows are re-read from cache every plane rather than held in
        // registers across the march: the opaque copy stops them being hoisted)
        GridDev gk = gd;
        asm volatile("" : "+s"(gk.f0tab32), "+s"(gk.f1tab32));
        auto flux_x = [&](int jj, int ii) {
            float qL[NV], qR[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                qL[v] = qx(1, v, jj, ii - 1);
                qR[v] = qx(0, v, jj, ii);
            }
            const FaceM<float> m = face_metric<float, 0, KS>(gk, B, ii, jj);
            lam0 = fmaxf(lam0, face_flux_lean<float, 0, FLUX>(qL, qR, m, ch, gam, gfac, F));
#pragma unroll
            for (int v = 0; v < NV; v++) fx(v, jj, ii) = F[v];
        };
        auto flux_y = [&](int jj, int ii) {
            float qL[NV], qR[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                qL[v] = qy(1, v, jj - 1, ii);
                qR[v] = qy(0, v, jj, ii);
            }
            const FaceM<float> m = face_metric<float, 1, KS>(gk, B, ii, jj);
            lam1 = fmaxf(lam1, face_flux_lean<float, 1, FLUX>(qL, qR, m, ch, gam, gfac, F));
#pragma unroll
            for (int v = 0; v < NV; v++) fy(v, jj, ii) = F[v];
        };
        if (own) {
            flux_x(j, i);
            __builtin_amdgcn_sched_barrier(0);
            flux_y(j, i);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (t < s0 + s1) {
            if (t < s1) flux_x(t, s0);
            else flux_y(s1, t - s1);
        }
        __builtin_amdgcn_sched_barrier(0);
        float fz[NV], sg2[NV], ih2[NV], qp1[NV];
        if (own) {
            float qm1[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {        // x3: cell k+1 from the register window
                sg2[v] = mc_slope(q1[v], q2[v], q3[v]);
                ih2[v] = iface(q1[v], q2[v], sg1[v], sg2[v]);
                float l = ih[v], r = ih2[v];
                ppm_limit(q1[v], l, r);
                qm1[v] = l;
                qp1[v] = r;
            }
            float qL[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) qL[v] = qp[v];
            lam2 = fmaxf(lam2, face_flux_lean<float, 2, FLUX>(qL, qm1, mz, ch, gam, gfac, fz));
        }
        __syncthreads();

        // ---- divergence of the own cell, then roll the x3 window
        if (own) {
            float *out = dU + B.ioff + ((long long)k * s1 + j) * s0 + i;
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const float d = (fx(v, j, i + 1) - fx(v, j, i)) * idx0 + (fy(v, j + 1, i) - fy(v, j, i)) * idx1 +
                                (fz[v] - fzp[v]) * idx2;
                out[v * nci] = d;
                qk[v] = q1[v];
                q1[v] = q2[v];
                q2[v] = q3[v];
                sg1[v] = sg2[v];
                ih[v] = ih2[v];
                qp[v] = qp1[v];
                fzp[v] = fz[v];
            }
        }
        __syncthreads();
    }

    const double m0 = wg_max<FWG>((double)lam0, red);
    if (t == 0) raise_max(&gd.st->lam_acc[0], m0);
    const double m1 = wg_max<FWG>((double)lam1, red);
    if (t == 0) raise_max(&gd.st->lam_acc[1], m1);
    const double m2 = wg_max<FWG>((double)lam2, red);
    if (t == 0) raise_max(&gd.st->lam_acc[2], m2);
}

// ---------------------------------------------------------------------------------
// Update from the stored divergence: sources (FP64), compensated RK combine,
// inversion (FP64). One thread per interior cell.
// ---------------------------------------------------------------------------------
// BASE: a != 0, so U_base is read (a template parameter keeps the loads in one block)
template <bool KS, bool BASE>
__global__ __launch_bounds__(WG) void k_update_div(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                                   const double *Ub, const double *Us, const float *__restrict__ Ps,
                                                   double *Uo, float *__restrict__ Po, const float *__restrict__ dU,
                                                   long long nci, double a, double b)
{
    __shared__ long long redl[WG / 64];
    __shared__ int redi[WG / 64];
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    const DevBlock B = gd.blocks[w.block];
    int i, j, k;
    int fail = 0, floored = 0, nit = 0;
    const int item = w.start + threadIdx.x;
    if (cell_of(B, item, i, j, k)) {
        const long long c = pad_index(B, kp, i, j, k);
        const long long ic = B.ioff + item;
        double q[NV], Uc[NV], S[NV], Un[NV], Pn[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            q[v] = (double)Ps[v * kp.ncp + c];
            Uc[v] = Us[v * kp.nci + ic];
        }
        const CentM m = centre_metric<KS>(gd, B, i, j);
        const double dt = gd.st->dt, kappa = gd.st->kappa;
        geometric_sources(q, Uc, m, kappa, S);
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const double L = S[v] - (double)dU[v * nci + ic];
            Un[v] = rk_combine<BASE>(a, BASE ? Ub[v * kp.nci + ic] : 0.0, b, Uc[v], dt, L);
        }
        int backup;
        fail = con_to_prim(Un, q, m, kp, Pn, nit, floored, backup);
        if (fail || floored) prim_to_cons(Pn, m, kp.gfac, Un);
        floored = fail ? 0 : floored;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            Uo[v * kp.nci + ic] = Un[v];
            Po[v * kp.ncp + c] = (float)Pn[v];
        }
    }
    const long long nfail = wg_sum<WG>(fail, redl);
    const long long nfl = wg_sum<WG>(floored, redl);
    const int mit = wg_imax<WG>(nit, redi);
    if (threadIdx.x == 0) {
        if (nfail) atomicAdd(&gd.st->c2p_fail, (unsigned long long)nfail);
        if (nfl) atomicAdd(&gd.st->floor_hits, (unsigned long long)nfl);
        if (mit) raise_max(&gd.st->max_iter, mit);
    }
}

// ---------------------------------------------------------------------------------
// Launcher of the block-tiled substep (the time-step bookkeeping kernels around it
// are launched by launch_substep).
// ---------------------------------------------------------------------------------
template <int FLUX, bool KS>
static hipError_t fused_typed(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                              void *Po, double a, double b, hipStream_t s)
{
    const int nb = (int)G.plan.dblocks.size();
    const int per = (nb + NXCD - 1) / NXCD;
    {
        TimedLaunch tl(G.timer, K_BLOCK_FLUX, s);
        hipLaunchKernelGGL((k_block_flux<FLUX, KS>), dim3(NXCD * per), dim3(FWG), 0, s, G.kp, G.gd, nb, per,
                           (const float *)Ps, (float *)G.d_div, G.plan.ncell_interior);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    TimedLaunch tl(G.timer, K_UPDATE_DIV, s);
    auto kern = a != 0.0 ? k_update_div<KS, true> : k_update_div<KS, false>;
    hipLaunchKernelGGL(kern, dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wcell, Ub, Us,
                       (const float *)Ps, Uo, (float *)Po, (const float *)G.d_div, G.plan.ncell_interior, a, b);
    return hipGetLastError();
}

hipError_t launch_fused_body(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                             void *Po, double a, double b, hipStream_t s)
{
    if (G.kp.flux == BHAC_FLUX_HLL)
        return G.ks ? fused_typed<BHAC_FLUX_HLL, true>(G, Ub, Us, Ps, Uo, Po, a, b, s)
                    : fused_typed<BHAC_FLUX_HLL, false>(G, Ub, Us, Ps, Uo, Po, a, b, s);
    return G.ks ? fused_typed<BHAC_FLUX_TVDLF, true>(G, Ub, Us, Ps, Uo, Po, a, b, s)
                : fused_typed<BHAC_FLUX_TVDLF, false>(G, Ub, Us, Ps, Uo, Po, a, b, s);
}

}  // namespace bhac
