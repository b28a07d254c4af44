// Face fluxes along one direction by columns (gfx950, wave64).
//
// One thread walks a line of cells along D through a block and produces the
// fluxes of that line's faces in order. Each cell is loaded once and its MC slope,
// PPM interface value and limited face values are computed once (the face kernel
// recomputes them for both faces of a cell); the Riemann solve per face is the same
// code. The line's halo past either end of the block is read from the neighbouring
// block's interior (or the own edge cell where the halo is zero-gradient), by the
// same rule as the face kernel. Lanes run along the fastest other axis, so every
// load and store is coalesced.
//
// A work item is one wave of lines of one block and a range [f0, f1) of faces
// along D (long lines may be cut into segments for parallelism; each segment
// starts with its own three-cell warm-up).
#include <hip/hip_runtime.h>

#include "physics.h"

namespace bhac {

// XL (block trees): a halo side marked cross-level is read from the block's own
// ghost slots (which the substep refreshes first), reached by the slot rule.
// ENT (entropy field): the entropy function K (row NV of P) marches with the other
// variables and is carried by each face's mass flux from the side that flux comes
// from (row NV of F).
// CT (constrained transport): the normal field of both states of a face is the face
// field phi there (direction D's array, the layout of F) over sqrt(gamma), and there
// is no GLM solve, as in the face kernel.
template <typename R, bool ENT>
struct MarchLds {
    static constexpr int NM = NV + (ENT ? 1 : 0); // marched variables
    static constexpr bool LST = sizeof(R) == 8;   // march state declared in LDS (double)
    double red[MWG / 64];
    R lst[LST ? 3 : 1][NM][LST ? MWG : 1];
};

// one work item: the faces [f0, f1) of MWG lines of one block (the work-group's
// LDS passed in, so that a kernel running items of two directions declares it once)
template <typename R, int D, int RECON, int FLUX, bool KS, bool XL, bool ENT, bool CT>
__device__ __forceinline__ void march_item(const KParams &kp, const GridDev &gd, const MarchItem &w,
                                           const R *__restrict__ P, R *__restrict__ F, long long nftot,
                                           const double *__restrict__ phi, MarchLds<R, ENT> &sm)
{
    constexpr int NM = MarchLds<R, ENT>::NM;
    constexpr bool LST = MarchLds<R, ENT>::LST;
    auto &lst = sm.lst;
    const DevBlock B = gd.blocks[w.block];
    constexpr int A = D == 0 ? 1 : 0;             // fastest axis across the lines
    constexpr int C = D == 2 ? 1 : 2;
    const int sD = B.s[D];
    const int line = w.line0 + threadIdx.x;
    double lam = 0.0;
    if (line < B.s[A] * B.s[C]) {
        int ix[3];
        ix[A] = line % B.s[A];
        ix[C] = line / B.s[A];
        ix[D] = 0;
        const long long base = pad_index(B, kp, ix[0], ix[1], ix[2]);
        const long long st = D == 0 ? 1 : (D == 1 ? (long long)B.n0 : (long long)B.n0 * B.n1);
        const bool clo = (B.hclamp >> (2 * D)) & 1, chi = (B.hclamp >> (2 * D + 1)) & 1;
        const long long sh_lo = B.hshift[D][0], sh_hi = B.hshift[D][1];
        const long long ncp = kp.ncp;
        // padded index of cell l of the line (l in [-3, sD + 2])
        auto cell = [&](int l) -> long long {
            const long long in = base + l * st;
            if constexpr (XL) {
                if ((l < 0 && ((B.hxl >> (2 * D)) & 1)) || (l >= sD && ((B.hxl >> (2 * D + 1)) & 1))) {
                    int q[3] = {ix[0], ix[1], ix[2]};
                    q[D] = l;
                    return ghost_slot(B, kp, q[0], q[1], q[2]);
                }
            }
            if (l < 0) return clo ? base : in + sh_lo;
            if (l >= sD) return chi ? base + (sD - 1) * st : in + sh_hi;
            return in;
        };
        auto load = [&](int l, R *q) {
            const long long c = cell(l);
#pragma unroll
            for (int v = 0; v < NM; v++) q[v] = P[v * ncp + c];
        };
        // index of face f of the line in the direction-D face array
        const int fs0 = B.s[0] + (D == 0), fs1 = B.s[1] + (D == 1);
        const long long fA = D == 0 ? 1 : (D == 1 ? (long long)fs0 : (long long)fs0 * fs1);
        int f0ix[3] = {ix[0], ix[1], ix[2]};
        const long long face0 = B.fofs[D] + ((long long)f0ix[2] * fs1 + f0ix[1]) * fs0 + f0ix[0];
        const R ch = (R)gd.st->ch, gam = (R)kp.gam, gfac = (R)kp.gfac;
        // x3 faces of a line share one metric record (the metrics do not depend on
        // x3); along x1 and x2 the record of the next face is fetched one face ahead
        auto metric = [&](int f) -> FaceM<R> {
            if constexpr (D == 2) return face_metric<R, D, KS>(gd, B, ix[0], ix[1]);
            else if constexpr (D == 0) return face_metric<R, D, KS>(gd, B, f, ix[1]);
            else return face_metric<R, D, KS>(gd, B, ix[0], f);
        };
        FaceM<R> mnext;
        if constexpr (D == 2 || !LST) mnext = metric(w.f0);
        R lmax = R(0);
        // double along x1/x2 (nine variables, independent patches): the face's metric
        // record is loaded at the top of the iteration that solves it, so its latency
        // overlaps that cell's reconstruction (a record fetched one face ahead would
        // not fit the register budget; with the entropy field or tree halos this one
        // would not either, and those variants load it at the solve)
        constexpr bool PRE = LST && D != 2 && !ENT && !XL;
        FaceM<R> mcur;
        auto fetch = [&](int f) {
            if constexpr (PRE) {
                if (f >= w.f0 && f < w.f1) mcur = metric(f);
            }
        };

        auto solve = [&](int f, R *qL, R *qR) {
            FaceM<R> m;
            if constexpr (D == 2) {
                m = mnext;
            } else if constexpr (PRE) {
                m = mcur;
            } else if constexpr (LST) {
                m = metric(f);
            } else {
                m = mnext;
                if (f + 1 < w.f1) mnext = metric(f + 1);
            }
            if constexpr (CT) {
                const R bn = (R)phi[face0 + f * fA] / m.sg;
                qL[5 + D] = bn;
                qR[5 + D] = bn;
            }
            R Ff[NV];
            const R l = face_flux<R, D, FLUX, CT>(qL, qR, m, ch, gam, gfac, Ff);
            lmax = l > lmax ? l : lmax;
            R *out = F + face0 + f * fA;
#pragma unroll
            for (int v = 0; v < NV; v++) out[v * nftot] = Ff[v];
            if constexpr (ENT) out[NV * nftot] = Ff[0] * (Ff[0] >= R(0) ? qL[NV] : qR[NV]);
        };

        if constexpr (RECON == BHAC_RECON_PPM) {
            // state before cell c: q_c, q_{c+1}, q_{c+2} (registers), and per
            // variable the MC slope s_c, the interface value a_{c-1/2} and the
            // limited upper value qp_{c-1} of cell c-1 (registers in float; double
            // declares them in LDS slots, kept in registers in the loop by the
            // compiler: fits two waves/SIMD unspilled, as arrays spills 64-224 B/lane)
            R qc[NM], qn[NM], q2[NM];
            R sreg[LST ? 1 : 3][NM];
            auto get = [&](int a, int v) -> R {
                if constexpr (LST) return lst[a][v][threadIdx.x];
                else return sreg[a][v];
            };
            auto put = [&](int a, int v, R x) {
                if constexpr (LST) lst[a][v][threadIdx.x] = x;
                else sreg[a][v] = x;
            };
            {
                R qa[NM], qb[NM];
                load(w.f0 - 3, qa);
                load(w.f0 - 2, qb);
                load(w.f0 - 1, qc);
                load(w.f0, qn);
                if constexpr (!LST) load(w.f0 + 1, q2);
#pragma unroll
                for (int v = 0; v < NM; v++) {
                    const R sb = mc_slope(qa[v], qb[v], qc[v]);
                    const R s0 = mc_slope(qb[v], qc[v], qn[v]);
                    put(0, v, s0);
                    put(1, v, ppm_iface(qb[v], qc[v], sb, s0));
                    put(2, v, R(0));
                }
            }
            for (int c = w.f0 - 1; c < w.f1; c++) {
                // float: q_{c+3} is fetched one cell ahead; double loads q_{c+2} here
                // (no room for a second set, neither in registers nor, beside the march
                // state, in LDS without spilling; the other wave on the SIMD hides it)
                R q3[LST ? 1 : NM];
                if constexpr (LST) load(c + 2, q2);
                else if (c + 1 < w.f1) load(c + 3, q3);
                fetch(c);
                R qm[NM], qL[NM];
#pragma unroll
                for (int v = 0; v < NM; v++) {
                    const R sn = mc_slope(qc[v], qn[v], q2[v]);
                    const R ap = ppm_iface(qc[v], qn[v], get(0, v), sn);
                    R qp;
                    ppm_limit(qc[v], get(1, v), ap, qm[v], qp);
                    qL[v] = get(2, v);                      // qp_{c-1}
                    put(0, v, sn);
                    put(1, v, ap);
                    put(2, v, qp);
                }
                if (c >= w.f0) solve(c, qL, qm);           // face c: cell c-1 | cell c
#pragma unroll
                for (int v = 0; v < NM; v++) {
                    qc[v] = qn[v];
                    qn[v] = q2[v];
                    if constexpr (!LST) q2[v] = q3[v];
                }
            }
        } else {
            // MC: state before face c: q_{c-1}, q_c, q_{c+1}, slope s_{c-1}
            R qa[NM], qc[NM], qn[NM], sa[NM];
            {
                R qb[NM];
                load(w.f0 - 2, qb);
                load(w.f0 - 1, qa);
                load(w.f0, qc);
                load(w.f0 + 1, qn);
#pragma unroll
                for (int v = 0; v < NM; v++) sa[v] = mc_slope(qb[v], qa[v], qc[v]);
            }
            for (int c = w.f0; c < w.f1; c++) {
                R q2[NM];
                if (c + 1 < w.f1) load(c + 2, q2);
                fetch(c);
                R qL[NM], qR[NM];
#pragma unroll
                for (int v = 0; v < NM; v++) {
                    const R s = mc_slope(qa[v], qc[v], qn[v]);
                    qL[v] = qa[v] + R(0.5) * sa[v];
                    qR[v] = qc[v] - R(0.5) * s;
                    sa[v] = s;
                }
                solve(c, qL, qR);
#pragma unroll
                for (int v = 0; v < NM; v++) {
                    qa[v] = qc[v];
                    qc[v] = qn[v];
                    qn[v] = q2[v];
                }
            }
        }
        lam = (double)lmax;
    }
    const double mx = wg_max<MWG>(lam, sm.red);
    if (threadIdx.x == 0) raise_max(&gd.st->lam_acc[D], mx);
}

template <typename R, int D, int RECON, int FLUX, bool KS, bool XL, bool ENT, bool CT = false>
__global__ __launch_bounds__(MWG, sizeof(R) == 8 ? 2 : 1) void k_flux_march(KParams kp, GridDev gd, const MarchItem *__restrict__ work,
                                                    const R *__restrict__ P, R *__restrict__ F, long long nftot,
                                                    const double *__restrict__ phi)
{
    __shared__ MarchLds<R, ENT> sm;
    const MarchItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    march_item<R, D, RECON, FLUX, KS, XL, ENT, CT>(kp, gd, w, P, F, nftot, phi, sm);
}

// The x2 and x3 line marches of a substep as one launch: work-groups [0, n2) take
// the x2 work list, the rest the x3 list (n2 is a multiple of the XCD count, so both
// keep their XCD order). One graph node instead of two kernels on two streams and
// the join between them (independent patches, no entropy field, GLM).
template <typename R, int RECON, int FLUX, bool KS>
__global__ __launch_bounds__(MWG, sizeof(R) == 8 ? 2 : 1) void k_flux_march_x23(KParams kp, GridDev gd,
                                                        const MarchItem *__restrict__ work2, long long n2,
                                                        const MarchItem *__restrict__ work3, const R *__restrict__ P,
                                                        R *__restrict__ F2, long long nf2, R *__restrict__ F3,
                                                        long long nf3)
{
    __shared__ MarchLds<R, false> sm;
    if (blockIdx.x < n2) {
        const MarchItem w = work2[blockIdx.x];
        if (w.block < 0) return;
        march_item<R, 1, RECON, FLUX, KS, false, false, false>(kp, gd, w, P, F2, nf2, nullptr, sm);
    } else {
        const MarchItem w = work3[blockIdx.x - n2];
        if (w.block < 0) return;
        march_item<R, 2, RECON, FLUX, KS, false, false, false>(kp, gd, w, P, F3, nf3, nullptr, sm);
    }
}

template <typename R, int D, int RECON, int FLUX, bool KS>
hipError_t launch_flux_march_typed(const DeviceGrid &G, const void *Ps, hipStream_t s, void *const *flux,
                                   const double *phi)
{
    const std::vector<MarchItem> &w = G.plan.wmarch[D];
    TimedLaunch tl(G.timer, K_FLUX0 + D, s);
    auto kern = G.plan.p.amr ? k_flux_march<R, D, RECON, FLUX, KS, true, false>
                             : (G.kp.nvar > NV ? k_flux_march<R, D, RECON, FLUX, KS, false, true>
                                               : k_flux_march<R, D, RECON, FLUX, KS, false, false>);
    if (phi) kern = k_flux_march<R, D, RECON, FLUX, KS, false, false, true>;
    hipLaunchKernelGGL(kern, dim3(w.size()), dim3(MWG), 0, s, G.kp, G.gd, G.d_wmarch[D], (const R *)Ps,
                       (R *)flux[D], G.plan.nface[D], phi);
    return hipGetLastError();
}

template <typename R, int D>
static hipError_t march_dir(const DeviceGrid &G, const void *Ps, hipStream_t s, void *const *flux, const double *phi)
{
    const int r = G.kp.recon, f = G.kp.flux;
#define MARCH_CASE(RC, FL, KSV) return launch_flux_march_typed<R, D, RC, FL, KSV>(G, Ps, s, flux, phi)
    if (G.ks) {
        if (r == BHAC_RECON_PPM) {
            if (f == BHAC_FLUX_HLL) MARCH_CASE(BHAC_RECON_PPM, BHAC_FLUX_HLL, true);
            MARCH_CASE(BHAC_RECON_PPM, BHAC_FLUX_TVDLF, true);
        }
        if (f == BHAC_FLUX_HLL) MARCH_CASE(BHAC_RECON_MC, BHAC_FLUX_HLL, true);
        MARCH_CASE(BHAC_RECON_MC, BHAC_FLUX_TVDLF, true);
    }
    if (r == BHAC_RECON_PPM) {
        if (f == BHAC_FLUX_HLL) MARCH_CASE(BHAC_RECON_PPM, BHAC_FLUX_HLL, false);
        MARCH_CASE(BHAC_RECON_PPM, BHAC_FLUX_TVDLF, false);
    }
    if (f == BHAC_FLUX_HLL) MARCH_CASE(BHAC_RECON_MC, BHAC_FLUX_HLL, false);
    MARCH_CASE(BHAC_RECON_MC, BHAC_FLUX_TVDLF, false);
#undef MARCH_CASE
}

template <typename R, int RECON, int FLUX, bool KS>
static hipError_t launch_x23_typed(const DeviceGrid &G, const void *Ps, hipStream_t s, void *const *flux)
{
    const size_t n2 = G.plan.wmarch[1].size(), n3 = G.plan.wmarch[2].size();
    hipLaunchKernelGGL((k_flux_march_x23<R, RECON, FLUX, KS>), dim3(n2 + n3), dim3(MWG), 0, s, G.kp, G.gd,
                       G.d_wmarch[1], (long long)n2, G.d_wmarch[2], (const R *)Ps, (R *)flux[1], G.plan.nface[1],
                       (R *)flux[2], G.plan.nface[2]);
    return hipGetLastError();
}

template <typename R>
static hipError_t x23_dir(const DeviceGrid &G, const void *Ps, hipStream_t s, void *const *flux)
{
    const int r = G.kp.recon, f = G.kp.flux;
#define X23_CASE(RC, FL, KSV) return launch_x23_typed<R, RC, FL, KSV>(G, Ps, s, flux)
    if (G.ks) {
        if (r == BHAC_RECON_PPM) {
            if (f == BHAC_FLUX_HLL) X23_CASE(BHAC_RECON_PPM, BHAC_FLUX_HLL, true);
            X23_CASE(BHAC_RECON_PPM, BHAC_FLUX_TVDLF, true);
        }
        if (f == BHAC_FLUX_HLL) X23_CASE(BHAC_RECON_MC, BHAC_FLUX_HLL, true);
        X23_CASE(BHAC_RECON_MC, BHAC_FLUX_TVDLF, true);
    }
    if (r == BHAC_RECON_PPM) {
        if (f == BHAC_FLUX_HLL) X23_CASE(BHAC_RECON_PPM, BHAC_FLUX_HLL, false);
        X23_CASE(BHAC_RECON_PPM, BHAC_FLUX_TVDLF, false);
    }
    if (f == BHAC_FLUX_HLL) X23_CASE(BHAC_RECON_MC, BHAC_FLUX_HLL, false);
    X23_CASE(BHAC_RECON_MC, BHAC_FLUX_TVDLF, false);
#undef X23_CASE
}

hipError_t launch_flux_march_x23(const DeviceGrid &G, const void *Ps, hipStream_t s, void *const *flux)
{
    return G.mixed ? x23_dir<float>(G, Ps, s, flux) : x23_dir<double>(G, Ps, s, flux);
}

hipError_t launch_flux_march(const DeviceGrid &G, int D, const void *Ps, hipStream_t s, void *const *flux,
                             const double *phi)
{
    if (G.mixed) {
        if (D == 0) return march_dir<float, 0>(G, Ps, s, flux, phi);
        if (D == 1) return march_dir<float, 1>(G, Ps, s, flux, phi);
        return march_dir<float, 2>(G, Ps, s, flux, phi);
    }
    if (D == 0) return march_dir<double, 0>(G, Ps, s, flux, phi);
    if (D == 1) return march_dir<double, 1>(G, Ps, s, flux, phi);
    return march_dir<double, 2>(G, Ps, s, flux, phi);
}

}  // namespace bhac
