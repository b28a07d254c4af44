// Unfused kernels of the GRMHD substep for gfx950 (wave64), plus the pointwise
// kernels (ghost fill, prim2con, con2prim, wave-speed reduction) and their launchers.
//
// Unfused substep = one face-flux kernel per direction (reconstruct P_stage at the
// face from a stencil that reaches into the neighbouring blocks' interiors, GLM +
// HLL/TVDLF, |lambda| max) -> one update kernel per interior cell (flux divergence,
// sources, RK combine, inversion). No ghost fill is needed between substeps.
// State rows are structure-of-arrays, so every load and store below is coalesced
// along x inside a block.
#include <hip/hip_runtime.h>

#include "compensated.h"
#include "physics.h"

namespace bhac {

// ---------------------------------------------------------------------------------
// Ghost fill: one thread per ghost slot copies the NQ rows (bit-exact copies).
// Pin and Pout are the same state: the kernel reads interior cells and writes ghost
// slots only, so the two views never meet and every row's load can be issued
// before the first store.
// ---------------------------------------------------------------------------------
template <typename T, int NQ>
__global__ __launch_bounds__(WG) void k_fill(const int32_t *__restrict__ dst, const int32_t *__restrict__ src,
                                             long long n, const T *__restrict__ Pin, T *__restrict__ Pout,
                                             long long ncp)
{
    // XCD-ordered chunks: XCD x copies the contiguous slot range of chunks [x per, (x+1) per)
    const unsigned per = (gridDim.x + NXCD - 1) / NXCD;
    const long long chunk = (long long)(blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
    const long long i = chunk * WG + threadIdx.x;
    if (i >= n) return;
    const long long d = dst[i], s = src[i];
#pragma unroll
    for (int v = 0; v < NQ; v++) Pout[v * ncp + d] = Pin[v * ncp + s];
}

// ---------------------------------------------------------------------------------
// Cross-level ghost fill of block trees: one thread per recipe (built by the
// planner), restriction or limited prolongation evaluated in double from interior
// cells only, stored in R. Recipes: [0, dst, the 2^ndim fine cells]
// (restriction), or [1, nchildren, coarse cell, the counts of the lower and upper
// neighbour per axis (0 = no slope), the neighbours' cells, then (dst, upper-half
// bits) per child] (prolongation of the ghost cells of one block that lie in one
// coarse cell, which share its slopes). Pin and Pout are the same state, read at
// interior cells and written at ghost slots only.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double minmod_xl(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}

// mean of the NC cells listed at idx (restriction of 2^ndim fine cells), summed in
// double in list order; the count is a compile-time constant, so all the loads of
// a variable (and, the views being disjoint, of all variables) are issued at once
template <int NC, typename R>
__device__ __forceinline__ double mean_n(const R *__restrict__ row, const int32_t *__restrict__ idx)
{
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < NC; q++) sum += (double)row[idx[q]];
    return sum * (NC == 8 ? 0.125 : 0.25);
}

template <typename R, int ND>
__global__ __launch_bounds__(WG) void k_fill_xl(const int32_t *__restrict__ xoff, const int32_t *__restrict__ xdat,
                                                long long n, const R *__restrict__ Pin, R *__restrict__ Pout,
                                                long long ncp)
{
#pragma clang fp contract(off)
    constexpr int NC = ND == 3 ? 8 : 4;           // fine cells per coarse cell
    const long long q = (long long)blockIdx.x * WG + threadIdx.x;
    if (q >= n) return;
    const int32_t *r = xdat + xoff[q];
    if (r[0] == 0) {
        int32_t idx[NC];
#pragma unroll
        for (int k = 0; k < NC; k++) idx[k] = r[2 + k];
        const int32_t dst = r[1];
#pragma unroll
        for (int v = 0; v < NV; v++) Pout[v * ncp + dst] = (R)mean_n<NC>(Pin + v * ncp, idx);
        return;
    }
    const int nk = r[1];
    const int32_t c = r[2];
    int cnt[6], at[6];
    int pos = 9;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        cnt[k] = r[3 + k];
        at[k] = pos;
        pos += cnt[k];
    }
    const int32_t *kids = r + pos;
    // a neighbour of the coarse cell is one cell (count 1) or the restriction of
    // NC fine cells (count NC); count 0 means no slope along that axis
    auto neighbour = [&](const R *__restrict__ row, int k) -> double {
        return cnt[k] == 1 ? (double)row[r[at[k]]] : mean_n<NC>(row, r + at[k]);
    };
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const R *row = Pin + v * ncp;
        const double qc = (double)row[c];
        double sl[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int d = 0; d < ND; d++) {
            if (cnt[2 * d] > 0 && cnt[2 * d + 1] > 0) {
                const double lo = neighbour(row, 2 * d);
                const double hi = neighbour(row, 2 * d + 1);
                sl[d] = minmod_xl(qc - lo, hi - qc);
            }
        }
        for (int k = 0; k < nk; k++) {
            const int bits = kids[2 * k + 1];
            double val = qc;
#pragma unroll
            for (int d = 0; d < ND; d++) val += (((bits >> d) & 1) ? 0.25 : -0.25) * sl[d];
            Pout[v * ncp + kids[2 * k]] = (R)val;
        }
    }
}

// ---------------------------------------------------------------------------------
// Flux correction of block trees: one thread per coarse face on a level boundary,
// which takes the mean of the fine faces covering it (records [direction, coarse
// face, 4 fine faces], 2 used in 2-D), summed in double in record order.
// ---------------------------------------------------------------------------------
template <typename R, int NSUB>
__global__ __launch_bounds__(WG) void k_flux_fix(const int32_t *__restrict__ fx, long long n,
                                                 const R *__restrict__ F0i, const R *__restrict__ F1i,
                                                 const R *__restrict__ F2i, R *__restrict__ F0o, R *__restrict__ F1o,
                                                 R *__restrict__ F2o, long long nf0, long long nf1, long long nf2)
{
    const long long t = (long long)blockIdx.x * WG + threadIdx.x;
    if (t >= n) return;
    const int32_t *r = fx + 6 * t;
    const int d = r[0];
    // a face is written by at most one record and never read by another (its far
    // side is either finer or coarser), so the input and output views never meet
    const R *Fi = d == 0 ? F0i : (d == 1 ? F1i : F2i);
    R *Fo = d == 0 ? F0o : (d == 1 ? F1o : F2o);
    const long long nf = d == 0 ? nf0 : (d == 1 ? nf1 : nf2);
    constexpr double w = NSUB == 4 ? 0.25 : 0.5;
    int32_t fine[NSUB];
#pragma unroll
    for (int q = 0; q < NSUB; q++) fine[q] = r[2 + q];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < NSUB; q++) sum += (double)Fi[v * nf + fine[q]];
        Fo[v * nf + r[1]] = (R)(sum * w);
    }
}

// ---------------------------------------------------------------------------------
// Face fluxes along D: one thread per face of a block (faces 0..s_D along D).
// ---------------------------------------------------------------------------------
// waves per SIMD the face kernels are compiled for: the scheduler hoists the
// stencil loads of all nine variables as far as this register budget allows
#ifndef BHAC_FLUX_OCC_F32
#define BHAC_FLUX_OCC_F32 6
#endif
#ifndef BHAC_FLUX_OCC_F64
#define BHAC_FLUX_OCC_F64 4
#endif
// (double MC, whose branch-free slopes let the scheduler hoist more, gets one less)
template <typename R, int RECON>
constexpr int flux_occupancy()
{
    return sizeof(R) == 4 ? BHAC_FLUX_OCC_F32 : (RECON == BHAC_RECON_MC ? BHAC_FLUX_OCC_F64 - 1 : BHAC_FLUX_OCC_F64);
}

// XL (block trees): a halo side marked cross-level is read from the block's own
// ghost slots (which the substep refreshes first), reached by the slot rule.
// ENT (entropy field): the entropy function K (row NV of P) is reconstructed at the
// face like the other variables, from the same stencil cells, and carried by the
// face's mass flux from the side that flux comes from (row NV of F).
// CT: constrained transport, the normal field of the face is the face field phi
// (direction D's array) for both states and there is no GLM solve.
template <typename R, int D, int RECON, int FLUX, bool KS, bool XL, bool ENT, bool CT = false>
__global__ __launch_bounds__(WG, (flux_occupancy<R, RECON>())) void k_flux(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                             const R *__restrict__ P, R *__restrict__ F, long long nftot,
                                             const double *__restrict__ phi)
{
    __shared__ double red[WG / 64];
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    const DevBlock B = gd.blocks[w.block];
    const int fs0 = B.s[0] + (D == 0), fs1 = B.s[1] + (D == 1), fs2 = B.s[2] + (D == 2);
    const int item = w.start + threadIdx.x;
    double lam = 0.0;
    if (item < fs0 * fs1 * fs2) {
        const int i = item % fs0;
        const int t = item / fs0;
        const int j = t % fs1;
        const int k = t / fs1;
        const long long pc = pad_index(B, kp, i, j, k);
        const long long st = D == 0 ? 1 : (D == 1 ? (long long)B.n0 : (long long)B.n0 * B.n1);
        // stencil cells l = f-3 .. f+2 along D; past either end of the block they are
        // read from the neighbour's interior (or the own edge cell where the halo is
        // zero-gradient), so no ghost slot of P is read
        const int f = D == 0 ? i : (D == 1 ? j : k);
        const int sD = B.s[D];
        const bool clo = (B.hclamp >> (2 * D)) & 1, chi = (B.hclamp >> (2 * D + 1)) & 1;
        constexpr int S0 = RECON == BHAC_RECON_PPM ? 0 : 1, S1 = RECON == BHAC_RECON_PPM ? 6 : 5;
        long long cell[6];
#pragma unroll
        for (int s = S0; s < S1; s++) {
            const int l = f + s - 3;
            const long long in = pc + (s - 3) * st;
            const long long lo = clo ? pc - f * st : in + B.hshift[D][0];
            const long long hi = chi ? pc + (sD - 1 - f) * st : in + B.hshift[D][1];
            cell[s] = l < 0 ? lo : (l >= sD ? hi : in);
            if constexpr (XL) {
                if ((l < 0 && ((B.hxl >> (2 * D)) & 1)) || (l >= sD && ((B.hxl >> (2 * D + 1)) & 1))) {
                    int q[3] = {i, j, k};
                    q[D] = l;
                    cell[s] = ghost_slot(B, kp, q[0], q[1], q[2]);
                }
            }
        }
        // In float the reconstruction is branch-free and every stencil load of the
        // face is written first, so all of them are in flight before the first wait.
        // In double the nine variables' stencils do not fit the register budget
        // together; the loop keeps them a variable at a time.
        R q[NV][6];
        R qL[NV], qR[NV];
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int v = 0; v < NV; v++) {
                q[v][0] = q[v][5] = R(0);
#pragma unroll
                for (int s = S0; s < S1; s++) q[v][s] = P[v * kp.ncp + cell[s]];
            }
#pragma unroll
            for (int v = 0; v < NV; v++) recon_face<R, RECON>(q[v], qL[v], qR[v]);
        } else {
#pragma unroll
            for (int v = 0; v < NV; v++) {
                q[v][0] = q[v][5] = R(0);
#pragma unroll
                for (int s = S0; s < S1; s++) q[v][s] = P[v * kp.ncp + cell[s]];
                recon_face<R, RECON>(q[v], qL[v], qR[v]);
            }
        }
        R KL = R(0), KR = R(0);
        if constexpr (ENT) {
            R qk[6];
            qk[0] = qk[5] = R(0);
#pragma unroll
            for (int s = S0; s < S1; s++) qk[s] = P[NV * kp.ncp + cell[s]];
            recon_face<R, RECON>(qk, KL, KR);
        }
        const FaceM<R> m = face_metric<R, D, KS>(gd, B, i, j);
        const R ch = (R)gd.st->ch;
        if constexpr (CT) {
            const R bn = (R)phi[B.fofs[D] + item] / m.sg;
            qL[5 + D] = bn;
            qR[5 + D] = bn;
        }
        R Ff[NV];
        lam = (double)face_flux<R, D, FLUX, CT>(qL, qR, m, ch, (R)kp.gam, (R)kp.gfac, Ff);
        R *out = F + B.fofs[D] + item;
#pragma unroll
        for (int v = 0; v < NV; v++) out[v * nftot] = Ff[v];
        if constexpr (ENT) out[NV * nftot] = Ff[0] * (Ff[0] >= R(0) ? KL : KR);
    }
    const double m = wg_max<WG>(lam, red);
    if (threadIdx.x == 0) raise_max(&gd.st->lam_acc[D], m);
}

// ---------------------------------------------------------------------------------
// x1 face fluxes with the work-group's rows staged in LDS: the cells of every row
// its 256 faces touch (halo included, from the neighbours as above) are loaded
// once, coalesced along the row; each face then reads its stencil from LDS.
// Along x1 a face's stencil lies in one padded row, so without staging every
// load instruction of a wave touches several rows and the neighbours' halo lines.
// ---------------------------------------------------------------------------------
// CT: constrained transport, as in the face kernel (phi: the x1 face field).
template <typename R, int RECON, int FLUX, bool KS, bool XL, bool ENT, bool CT = false>
__global__ __launch_bounds__(WG, (flux_occupancy<R, RECON>())) void k_flux_x1s(KParams kp, GridDev gd,
                                                                            const WorkItem *__restrict__ work,
                                                                            const R *__restrict__ P,
                                                                            R *__restrict__ F, long long nftot,
                                                                            const double *__restrict__ phi)
{
    constexpr int NS = NV + (ENT ? 1 : 0);        // staged rows of P (the entropy function last)
    __shared__ R tile[NS][x1s_max_cells<R>()];
    __shared__ double red[WG / 64];
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    const DevBlock B = gd.blocks[w.block];
    const int s0 = B.s[0], fs0 = s0 + 1, nface = fs0 * B.s[1] * B.s[2];
    const int r0 = w.start / fs0;
    const int r1 = (min(w.start + WG, nface) - 1) / fs0;
    const int rowlen = s0 + 6;                    // cells -3 .. s0+2 of a row
    const int ncell = (r1 - r0 + 1) * rowlen;
    const bool clo = B.hclamp & 1, chi = (B.hclamp >> 1) & 1;
    for (int t = threadIdx.x; t < ncell; t += WG) {
        const int row = r0 + t / rowlen, l = t % rowlen - 3;
        const long long base = pad_index(B, kp, 0, row % B.s[1], row / B.s[1]);
        long long c = base + l;
        if (l < 0) c = clo ? base : c + B.hshift[0][0];
        else if (l >= s0) c = chi ? base + s0 - 1 : c + B.hshift[0][1];
        if constexpr (XL) {
            if ((l < 0 && (B.hxl & 1)) || (l >= s0 && ((B.hxl >> 1) & 1)))
                c = ghost_slot(B, kp, l, row % B.s[1], row / B.s[1]);
        }
#pragma unroll
        for (int v = 0; v < NS; v++) tile[v][t] = P[v * kp.ncp + c];
    }
    // the face's metric record is requested before the barrier, so its latency
    // overlaps the staging
    const int item = w.start + threadIdx.x;
    const int iface = item % fs0, rface = item / fs0;
    FaceM<R> m;
    if (item < nface) m = face_metric<R, 0, KS>(gd, B, iface, rface % B.s[1]);
    __syncthreads();
    double lam = 0.0;
    if (item < nface) {
        const int i = iface, row = rface;
        const int t0 = (row - r0) * rowlen + i;   // tile slot of cell i - 3
        R qL[NV], qR[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            R q[6];
#pragma unroll
            for (int s = 0; s < 6; s++) q[s] = tile[v][t0 + s];
            recon_face<R, RECON>(q, qL[v], qR[v]);
        }
        R KL = R(0), KR = R(0);
        if constexpr (ENT) {
            R q[6];
#pragma unroll
            for (int s = 0; s < 6; s++) q[s] = tile[NV][t0 + s];
            recon_face<R, RECON>(q, KL, KR);
        }
        if constexpr (CT) {
            const R bn = (R)phi[B.fofs[0] + item] / m.sg;
            qL[5] = bn;
            qR[5] = bn;
        }
        R Ff[NV];
        lam = (double)face_flux<R, 0, FLUX, CT>(qL, qR, m, (R)gd.st->ch, (R)kp.gam, (R)kp.gfac, Ff);
        R *out = F + B.fofs[0] + item;
#pragma unroll
        for (int v = 0; v < NV; v++) out[v * nftot] = Ff[v];
        if constexpr (ENT) out[NV * nftot] = Ff[0] * (Ff[0] >= R(0) ? KL : KR);
    }
    const double mx = wg_max<WG>(lam, red);
    if (threadIdx.x == 0) raise_max(&gd.st->lam_acc[0], mx);
}

// ---------------------------------------------------------------------------------
// Update: divergence (in R), sources, RK combine (double), inversion (double).
// ---------------------------------------------------------------------------------
// ND3: three dimensions (else two); BASE: a != 0, so U_base is read. Both are
// template parameters so that every load of a cell sits in one basic block and is
// issued before the first wait (a uniform run-time branch per value would split
// the loads into serial round trips).
// CT: constrained transport; the field rows of U_out along the resolved directions are
// the means of the cell's two updated faces of the face field (Ph0..Ph2: directions'
// arrays of phi_out, written earlier in the substep).
template <typename R, bool KS, bool ND3, bool BASE, bool ENT, bool CT = false>
__global__ __launch_bounds__(WG, 3) void k_update(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                               const double *Ub, const double *Us, const R *__restrict__ Ps,
                                               double *Uo, R *__restrict__ Po, const R *__restrict__ F0,
                                               const R *__restrict__ F1, const R *__restrict__ F2, long long nf0,
                                               long long nf1, long long nf2, double a, double b,
                                               const double *__restrict__ Ph0, const double *__restrict__ Ph1,
                                               const double *__restrict__ Ph2)
{
    constexpr int NQ = NV + (ENT ? 1 : 0);        // rows: GRMHD variables (+ entropy field)
    __shared__ long long redl[WG / 64];
    __shared__ int redi[WG / 64];
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    const DevBlock B = gd.blocks[w.block];
    int i, j, k;
    int fail = 0, floored = 0, nit = 0, backup = 0;
    if (cell_of(B, w.start + threadIdx.x, i, j, k)) {
        const long long c = pad_index(B, kp, i, j, k);
        const long long ci = B.ioff + w.start + threadIdx.x;   // interior-packed index of U
        const DevLevel &L = gd.levels[B.level];
        // flux divergence, formed per direction in R, summed in double
        double div[3][NQ];
        double bface[3] = {0.0, 0.0, 0.0};        // CT: mean of the updated face fields
#pragma unroll
        for (int v = 0; v < NQ; v++) div[2][v] = 0.0;
#pragma unroll
        for (int d = 0; d < (ND3 ? 3 : 2); d++) {
            const R *Fd = d == 0 ? F0 : (d == 1 ? F1 : F2);
            const long long nf = d == 0 ? nf0 : (d == 1 ? nf1 : nf2);
            const int fs0 = B.s[0] + (d == 0), fs1 = B.s[1] + (d == 1);
            const long long lo = B.fofs[d] + ((long long)k * fs1 + j) * fs0 + i;
            const long long hi = lo + (d == 0 ? 1 : (d == 1 ? fs0 : (long long)fs0 * fs1));
            const R idx = (R)L.inv_dx[d];
#pragma unroll
            for (int v = 0; v < NQ; v++) div[d][v] = (double)((Fd[v * nf + hi] - Fd[v * nf + lo]) * idx);
            if constexpr (CT) {
                const double *Ph = d == 0 ? Ph0 : (d == 1 ? Ph1 : Ph2);
                bface[d] = 0.5 * (Ph[lo] + Ph[hi]);
            }
        }
        double q[NQ], Uc[NQ], S[NQ];
#pragma unroll
        for (int v = 0; v < NQ; v++) {
            q[v] = (double)Ps[v * kp.ncp + c];
            Uc[v] = Us[v * kp.nci + ci];
        }
        const CentM m = centre_metric<KS>(gd, B, i, j);
        const double dt = gd.st->dt, kappa = gd.st->kappa;
        geometric_sources(q, Uc, m, kappa, S);
        if constexpr (ENT) S[NV] = 0.0;           // the entropy field has no source
        double Un[NQ];
#pragma unroll
        for (int v = 0; v < NQ; v++) {
            // L = -(div_1 + div_2 + div_3) + S with a Neumaier compensation, then
            // U_out = a U_base + b (U_stage + dt L) rounded once
            const double Lv = neumaier4(-div[0][v], -div[1][v], -div[2][v], S[v]);
            Un[v] = rk_combine<BASE>(a, BASE ? Ub[v * kp.nci + ci] : 0.0, b, Uc[v], dt, Lv);
        }
        if constexpr (CT) {
#pragma unroll
            for (int d = 0; d < (ND3 ? 3 : 2); d++) Un[5 + d] = bface[d];
        }
        double Pn[NQ];
        fail = con_to_prim<ENT>(Un, q, m, kp, Pn, nit, floored, backup);
        // failed, floored or backed-up cells take the conserved state of their primitives
        if (fail || floored || backup) {
            prim_to_cons(Pn, m, kp.gfac, Un);
            if constexpr (ENT) Un[NV] = Un[0] * Pn[NV];
        }
        floored = fail ? 0 : floored;
#pragma unroll
        for (int v = 0; v < NQ; v++) {
            Uo[v * kp.nci + ci] = Un[v];
            Po[v * kp.ncp + c] = (R)Pn[v];
        }
    }
    const long long nfail = wg_sum<WG>(fail, redl);
    const long long nfl = wg_sum<WG>(floored, redl);
    const int mit = wg_imax<WG>(nit, redi);
    long long nbk = 0;
    if constexpr (ENT) nbk = wg_sum<WG>(backup, redl);
    if (threadIdx.x == 0) {
        if (nfail) atomicAdd(&gd.st->c2p_fail, (unsigned long long)nfail);
        if (nfl) atomicAdd(&gd.st->floor_hits, (unsigned long long)nfl);
        if (mit) raise_max(&gd.st->max_iter, mit);
        if (nbk) atomicAdd(&gd.st->c2p_backup, (unsigned long long)nbk);
    }
}

// ---------------------------------------------------------------------------------
// Update with the x1 faces computed in place (independent patches, no entropy
// field). A work item is x1u_rows(s0) whole rows of one block. The rows' cells with
// their x1 halo (from the neighbours as in the face kernels) are staged in LDS;
// each thread computes one x1 face flux exactly as the staged x1 face kernel does
// and leaves it in LDS; after a barrier each thread updates one cell of the rows
// exactly as k_update does, taking its x1 faces and its stage primitives from LDS
// and its x2/x3 faces from the face arrays. The x1 fluxes never reach HBM, P_stage
// is read once, and the Riemann arithmetic of one work-group overlaps the memory
// traffic of the others on the CU.
// ---------------------------------------------------------------------------------
template <typename R, int RECON, int FLUX, bool KS, bool ND3, bool BASE>
__global__ __launch_bounds__(WG, 3) void k_update_x1(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                                  const double *Ub, const double *Us, const R *__restrict__ Ps,
                                                  double *Uo, R *__restrict__ Po, const R *__restrict__ F1,
                                                  const R *__restrict__ F2, long long nf1, long long nf2, double a,
                                                  double b)
{
    __shared__ R tile[NV][x1s_max_cells<R>()];
    __shared__ R fx[NV][WG];
    __shared__ double red[WG / 64];
    __shared__ long long redl[WG / 64];
    __shared__ int redi[WG / 64];
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    const DevBlock B = gd.blocks[w.block];
    const int s0 = B.s[0], fs0 = s0 + 1, r0 = w.start;
    const int nr = min(x1u_rows(s0), B.s[1] * B.s[2] - r0);
    const int rowlen = s0 + 6;                    // cells -3 .. s0+2 of a row
    const int ncell = nr * rowlen;
    const bool clo = B.hclamp & 1, chi = (B.hclamp >> 1) & 1;
    for (int t = threadIdx.x; t < ncell; t += WG) {
        const int row = r0 + t / rowlen, l = t % rowlen - 3;
        const long long base = pad_index(B, kp, 0, row % B.s[1], row / B.s[1]);
        long long c = base + l;
        if (l < 0) c = clo ? base : c + B.hshift[0][0];
        else if (l >= s0) c = chi ? base + s0 - 1 : c + B.hshift[0][1];
#pragma unroll
        for (int v = 0; v < NV; v++) tile[v][t] = Ps[v * kp.ncp + c];
    }
    // the face's metric record is requested before the barrier (its latency
    // overlaps the staging)
    const int frow = threadIdx.x / fs0, fi = threadIdx.x % fs0;
    FaceM<R> mf;
    if (threadIdx.x < nr * fs0) mf = face_metric<R, 0, KS>(gd, B, fi, (r0 + frow) % B.s[1]);
    __syncthreads();
    // x1 face t of the item (faces 0 .. s0 of each row, row-major)
    double lam = 0.0;
    if (threadIdx.x < nr * fs0) {
        const int t0 = frow * rowlen + fi;        // tile slot of cell fi - 3
        R qL[NV], qR[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            R q[6];
#pragma unroll
            for (int s = 0; s < 6; s++) q[s] = tile[v][t0 + s];
            recon_face<R, RECON>(q, qL[v], qR[v]);
        }
        R Ff[NV];
        lam = (double)face_flux<R, 0, FLUX>(qL, qR, mf, (R)gd.st->ch, (R)kp.gam, (R)kp.gfac, Ff);
#pragma unroll
        for (int v = 0; v < NV; v++) fx[v][threadIdx.x] = Ff[v];
    }
    const double mx = wg_max<WG>(lam, red);       // (its barrier also publishes fx)
    if (threadIdx.x == 0) raise_max(&gd.st->lam_acc[0], mx);
    // cell t of the item (cells 0 .. s0-1 of each row, row-major = interior order)
    int fail = 0, floored = 0, nit = 0, backup = 0;
    if (threadIdx.x < nr * s0) {
        const int crow = threadIdx.x / s0, i = threadIdx.x % s0;
        const int row = r0 + crow, j = row % B.s[1], k = row / B.s[1];
        const long long cl = (long long)row * s0 + i;           // interior index within the block
        const long long c = B.off + cl;
        const long long ci = B.ioff + cl;
        const DevLevel &L = gd.levels[B.level];
        double div[3][NV];
#pragma unroll
        for (int v = 0; v < NV; v++) div[2][v] = 0.0;
        {
            const int lo = crow * fs0 + i;
            const R idx = (R)L.inv_dx[0];
#pragma unroll
            for (int v = 0; v < NV; v++) div[0][v] = (double)((fx[v][lo + 1] - fx[v][lo]) * idx);
        }
#pragma unroll
        for (int d = 1; d < (ND3 ? 3 : 2); d++) {
            const R *Fd = d == 1 ? F1 : F2;
            const long long nf = d == 1 ? nf1 : nf2;
            const int fs1 = B.s[1] + (d == 1);
            const long long lo = B.fofs[d] + ((long long)k * fs1 + j) * s0 + i;
            const long long hi = lo + (d == 1 ? s0 : (long long)s0 * fs1);
            const R idx = (R)L.inv_dx[d];
#pragma unroll
            for (int v = 0; v < NV; v++) div[d][v] = (double)((Fd[v * nf + hi] - Fd[v * nf + lo]) * idx);
        }
        // from here on the same statements as k_update, in the same order (kept
        // inline: as a shared function the compiler split the cell's loads into
        // more serial batches and the update ran 12 % slower)
        double q[NV], Uc[NV], S[NV];
        const int ts = crow * rowlen + i + 3;     // tile slot of the cell
#pragma unroll
        for (int v = 0; v < NV; v++) {
            q[v] = (double)tile[v][ts];
            Uc[v] = Us[v * kp.nci + ci];
        }
        const CentM m = centre_metric<KS>(gd, B, i, j);
        const double dt = gd.st->dt, kappa = gd.st->kappa;
        geometric_sources(q, Uc, m, kappa, S);
        double Un[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const double Lv = neumaier4(-div[0][v], -div[1][v], -div[2][v], S[v]);
            Un[v] = rk_combine<BASE>(a, BASE ? Ub[v * kp.nci + ci] : 0.0, b, Uc[v], dt, Lv);
        }
        double Pn[NV];
        fail = con_to_prim<false>(Un, q, m, kp, Pn, nit, floored, backup);
        if (fail || floored) prim_to_cons(Pn, m, kp.gfac, Un);
        floored = fail ? 0 : floored;
#pragma unroll
        for (int v = 0; v < NV; v++) {
            Uo[v * kp.nci + ci] = Un[v];
            Po[v * kp.ncp + c] = (R)Pn[v];
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
// Pointwise kernels.
// ---------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------
// Staggered-mesh constrained transport. The face field phi^d = sqrt(gamma) B^d lives
// on every face of a block (the layout of the face-flux arrays). Its update needs the
// edge electric fields E_k = F^j(B~^i) = -F^i(B~^j) ((i, j, k) cyclic), each the mean
// of the induction fluxes of the four faces around the edge; a face beyond the block
// is read from the neighbouring block's face array (or, where the halo rule is the
// zero-gradient clamp, from the block's own nearest face), so the two copies of a
// face shared by two blocks receive identical updates.
// ---------------------------------------------------------------------------------
struct CtFlux {
    const void *F[3];                // face-flux arrays of the three directions (R)
    long long nf[3];
};

// flux row v of direction d at block b's face (f0, f1, f2): f[d] a face index, the
// others cell indices, at most one of them beyond the block
template <typename R>
__device__ __forceinline__ double ct_flux(const GridDev &gd, const DevBlock &B, int b, const CtFlux &cf, int d, int v,
                                          int f0, int f1, int f2)
{
    int f[3] = {f0, f1, f2};
    int nb = b;
#pragma unroll
    for (int e = 0; e < 3; e++) {
        if (e == d) continue;
        const int pe = e == 0 ? 1 : (e == 1 ? 3 : 9);
        if (f[e] < 0) {
            if ((B.hclamp >> (2 * e)) & 1) f[e] = 0;
            else { nb = gd.nbr[(long long)b * 27 + 13 - pe]; f[e] += B.s[e]; }
        } else if (f[e] >= B.s[e]) {
            if ((B.hclamp >> (2 * e + 1)) & 1) f[e] = B.s[e] - 1;
            else { nb = gd.nbr[(long long)b * 27 + 13 + pe]; f[e] -= B.s[e]; }
        }
    }
    const long long fofs = nb == b ? B.fofs[d] : gd.blocks[nb].fofs[d];
    const int fs0 = B.s[0] + (d == 0), fs1 = B.s[1] + (d == 1);
    const R *F = (const R *)cf.F[d];
    return (double)F[v * cf.nf[d] + fofs + ((long long)f[2] * fs1 + f[1]) * fs0 + f[0]];
}

// E along axis AX at the edge whose corner is c in face units along the two axes
// normal to it (cell index along AX)
template <typename R, int AX>
__device__ __forceinline__ double ct_emf(const GridDev &gd, const DevBlock &B, int b, const CtFlux &cf, int c0, int c1,
                                         int c2)
{
    constexpr int A = (AX + 1) % 3, Bx = (AX + 2) % 3;
    int lo_a[3] = {c0, c1, c2}, lo_b[3] = {c0, c1, c2};
    lo_a[A] -= 1;           // Bx-faces of the cells on both sides along A
    lo_b[Bx] -= 1;          // A-faces of the cells on both sides along Bx
    const double fb = ct_flux<R>(gd, B, b, cf, Bx, 5 + A, lo_a[0], lo_a[1], lo_a[2]) +
                      ct_flux<R>(gd, B, b, cf, Bx, 5 + A, c0, c1, c2);
    const double fa = ct_flux<R>(gd, B, b, cf, A, 5 + Bx, lo_b[0], lo_b[1], lo_b[2]) +
                      ct_flux<R>(gd, B, b, cf, A, 5 + Bx, c0, c1, c2);
    return 0.25 * (fb - fa);
}

// Edge fields stored per direction K: block b's edges along K start at eofs[3 b + K],
// (size_d + [d != K]) of them along each axis d, x fastest.
struct CtEdge {
    double *E[3];
    const long long *eofs;
};

template <int K>
__device__ __forceinline__ long long edge_index(const DevBlock &B, const CtEdge &ce, int b, int c0, int c1, int c2)
{
    const int e0 = B.s[0] + (K != 0), e1 = B.s[1] + (K != 1);
    return ce.eofs[(long long)b * 3 + K] + ((long long)c2 * e1 + c1) * e0 + c0;
}

// every edge along K of a block, once: E_K from the four induction fluxes around it
template <typename R, int K>
__global__ __launch_bounds__(WG) void k_ct_edge(KParams kp, GridDev gd, const WorkItem *__restrict__ work, CtFlux cf,
                                                CtEdge ce)
{
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;
    const DevBlock B = gd.blocks[w.block];
    const int e0 = B.s[0] + (K != 0), e1 = B.s[1] + (K != 1), e2 = B.s[2] + (K != 2);
    const int item = w.start + threadIdx.x;
    if (item >= e0 * e1 * e2) return;
    const int c0 = item % e0, t = item / e0, c1 = t % e1, c2 = t / e1;
    ce.E[K][edge_index<K>(B, ce, w.block, c0, c1, c2)] = ct_emf<R, K>(gd, B, w.block, cf, c0, c1, c2);
}

// phi_out = a phi_base + b (phi_stage + dt L), L = -(d_j E_k - d_k E_j) on the faces of
// direction D ((D, j, k) cyclic), from the block's stored edge fields; with ndim = 2
// only the edges along x3 exist
template <int D, bool ND3, bool BASE>
__global__ __launch_bounds__(WG) void k_ct_face(KParams kp, GridDev gd, const WorkItem *__restrict__ work, CtEdge ce,
                                                const double *Phb, const double *Phs, double *Pho, double a, double b)
{
    constexpr int DJ = (D + 1) % 3, DK = (D + 2) % 3;
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;
    const DevBlock B = gd.blocks[w.block];
    const int fs0 = B.s[0] + (D == 0), fs1 = B.s[1] + (D == 1), fs2 = B.s[2] + (D == 2);
    const int item = w.start + threadIdx.x;
    if (item >= fs0 * fs1 * fs2) return;
    const int i = item % fs0, t = item / fs0, j = t % fs1, k = t / fs1;
    const DevLevel &L = gd.levels[B.level];
    double Lv = 0.0;
    if constexpr (DJ < 2 || ND3) {
        int h[3] = {i, j, k};
        h[DJ] += 1;
        const double eh = ce.E[DK][edge_index<DK>(B, ce, w.block, h[0], h[1], h[2])];
        const double el = ce.E[DK][edge_index<DK>(B, ce, w.block, i, j, k)];
        Lv -= (eh - el) * L.inv_dx[DJ];
    }
    if constexpr (DK < 2 || ND3) {
        int h[3] = {i, j, k};
        h[DK] += 1;
        const double eh = ce.E[DJ][edge_index<DJ>(B, ce, w.block, h[0], h[1], h[2])];
        const double el = ce.E[DJ][edge_index<DJ>(B, ce, w.block, i, j, k)];
        Lv += (eh - el) * L.inv_dx[DK];
    }
    const long long q = B.fofs[D] + item;
    Pho[q] = rk_combine<BASE>(a, BASE ? Phb[q] : 0.0, b, Phs[q], gd.st->dt, Lv);
}

// cell-centred field from a face field: P rows B^d = mean of the two faces / sqrt(gamma)
template <typename R, bool KS>
__global__ __launch_bounds__(WG) void k_ct_center(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                                  const double *__restrict__ Ph0, const double *__restrict__ Ph1,
                                                  const double *__restrict__ Ph2, R *__restrict__ P)
{
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;
    const DevBlock B = gd.blocks[w.block];
    int i, j, k;
    if (!cell_of(B, w.start + threadIdx.x, i, j, k)) return;
    const double sg = centre_metric<KS>(gd, B, i, j).sg;
    const long long c = pad_index(B, kp, i, j, k);
    for (int d = 0; d < kp.ndim; d++) {
        const double *Ph = d == 0 ? Ph0 : (d == 1 ? Ph1 : Ph2);
        const int fs0 = B.s[0] + (d == 0), fs1 = B.s[1] + (d == 1);
        const long long lo = B.fofs[d] + ((long long)k * fs1 + j) * fs0 + i;
        const long long hi = lo + (d == 0 ? 1 : (d == 1 ? fs0 : (long long)fs0 * fs1));
        P[(5 + d) * kp.ncp + c] = (R)(0.5 * (Ph[lo] + Ph[hi]) / sg);
    }
}

// discrete divergence of a face field per interior cell (interior-packed)
__global__ __launch_bounds__(WG) void k_ct_div(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                               const double *__restrict__ Ph0, const double *__restrict__ Ph1,
                                               const double *__restrict__ Ph2, double *__restrict__ div)
{
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;
    const DevBlock B = gd.blocks[w.block];
    int i, j, k;
    if (!cell_of(B, w.start + threadIdx.x, i, j, k)) return;
    const DevLevel &L = gd.levels[B.level];
    double sdiv = 0.0;
    for (int d = 0; d < kp.ndim; d++) {
        const double *Ph = d == 0 ? Ph0 : (d == 1 ? Ph1 : Ph2);
        const int fs0 = B.s[0] + (d == 0), fs1 = B.s[1] + (d == 1);
        const long long lo = B.fofs[d] + ((long long)k * fs1 + j) * fs0 + i;
        const long long hi = lo + (d == 0 ? 1 : (d == 1 ? fs0 : (long long)fs0 * fs1));
        sdiv += (Ph[hi] - Ph[lo]) * L.inv_dx[d];
    }
    div[B.ioff + w.start + threadIdx.x] = sdiv;
}

template <typename R, bool KS>
__global__ __launch_bounds__(WG) void k_prim2con(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                                 const R *__restrict__ P, double *__restrict__ U)
{
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    const DevBlock B = gd.blocks[w.block];
    int i, j, k;
    if (!cell_of(B, w.start + threadIdx.x, i, j, k)) return;
    const long long c = pad_index(B, kp, i, j, k);
    const long long ci = B.ioff + w.start + threadIdx.x;
    double q[NV], Uc[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) q[v] = (double)P[v * kp.ncp + c];
    prim_to_cons(q, centre_metric<KS>(gd, B, i, j), kp.gfac, Uc);
#pragma unroll
    for (int v = 0; v < NV; v++) U[v * kp.nci + ci] = Uc[v];
    if (kp.nvar > NV) U[NV * kp.nci + ci] = Uc[0] * (double)P[NV * kp.ncp + c];
}

template <typename R, bool KS, bool ENT>
__global__ __launch_bounds__(WG) void k_con2prim(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                                 const double *__restrict__ U, R *__restrict__ P,
                                                 int8_t *__restrict__ flags)
{
    __shared__ long long redl[WG / 64];
    __shared__ int redi[WG / 64];
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    const DevBlock B = gd.blocks[w.block];
    int i, j, k;
    constexpr int NQ = NV + (ENT ? 1 : 0);
    int fail = 0, floored = 0, nit = 0, backup = 0;
    if (cell_of(B, w.start + threadIdx.x, i, j, k)) {
        const long long c = pad_index(B, kp, i, j, k);
        const long long ci = B.ioff + w.start + threadIdx.x;
        double q[NQ], Uc[NQ], Pn[NQ];
#pragma unroll
        for (int v = 0; v < NQ; v++) {
            q[v] = (double)P[v * kp.ncp + c];
            Uc[v] = U[v * kp.nci + ci];
        }
        fail = con_to_prim<ENT>(Uc, q, centre_metric<KS>(gd, B, i, j), kp, Pn, nit, floored, backup);
        floored = fail ? 0 : floored;
#pragma unroll
        for (int v = 0; v < NQ; v++) P[v * kp.ncp + c] = (R)Pn[v];
        if (flags) flags[ci] = (int8_t)fail;
    }
    const long long nfail = wg_sum<WG>(fail, redl);
    const long long nfl = wg_sum<WG>(floored, redl);
    const int mit = wg_imax<WG>(nit, redi);
    const long long nbk = wg_sum<WG>(backup, redl);
    if (threadIdx.x == 0) {
        if (nfail) atomicAdd(&gd.st->c2p_fail, (unsigned long long)nfail);
        if (nfl) atomicAdd(&gd.st->floor_hits, (unsigned long long)nfl);
        if (mit) raise_max(&gd.st->max_iter, mit);
        if (nbk) atomicAdd(&gd.st->c2p_backup, (unsigned long long)nbk);
    }
}

template <typename R, bool KS>
__global__ __launch_bounds__(WG) void k_cell_speeds(KParams kp, GridDev gd, const WorkItem *__restrict__ work,
                                                    const R *__restrict__ P)
{
    __shared__ double red[WG / 64];
    const WorkItem w = work[blockIdx.x];
    if (w.block < 0) return;                      // padding of the XCD order (whole work-group)
    const DevBlock B = gd.blocks[w.block];
    int i, j, k;
    double lam[3] = {0.0, 0.0, 0.0};
    if (cell_of(B, w.start + threadIdx.x, i, j, k)) {
        const long long c = pad_index(B, kp, i, j, k);
        double q[NV], dummy[NV], lm, lp;
#pragma unroll
        for (int v = 0; v < NV; v++) q[v] = (double)P[v * kp.ncp + c];
        const FaceM<double> m = centre_as_face(centre_metric<KS>(gd, B, i, j));
        face_state<double, 0, false>(q, m, kp.gam, kp.gfac, dummy, dummy, lm, lp);
        lam[0] = fmax(fabs(lm), fabs(lp));
        face_state<double, 1, false>(q, m, kp.gam, kp.gfac, dummy, dummy, lm, lp);
        lam[1] = fmax(fabs(lm), fabs(lp));
        if (kp.ndim == 3) {
            face_state<double, 2, false>(q, m, kp.gam, kp.gfac, dummy, dummy, lm, lp);
            lam[2] = fmax(fabs(lm), fabs(lp));
        }
    }
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double mx = wg_max<WG>(lam[d], red);
        if (threadIdx.x == 0) raise_max(&gd.st->lam_acc[d], mx);
    }
}

// ---------------------------------------------------------------------------------
// Time-step bookkeeping (single thread).
// ---------------------------------------------------------------------------------
// dt_next from the wave-speed maxima of the substep that last filled lam_acc
__device__ __forceinline__ void finish_step(const KParams &kp, DevState *st)
{
    double s = 0.0;
    for (int d = 0; d < kp.ndim; d++) {
        const double l = __longlong_as_double((long long)st->lam_acc[d]);
        st->lam_last[d] = l;
        s += l * kp.inv_dx_fine[d];
    }
    st->dt_next = st->dt_fixed > 0.0 ? st->dt_fixed : kp.cfl / s;
    st->lam_pending = 0;
}

// Start of a substep: first the previous substep's maxima become dt_next (a substep
// ends without a kernel of its own, so the step graph has one node fewer per
// substep; host reads finish it through k_end), then the latch, then the reset.
__global__ void k_begin(KParams kp, DevState *st, int latch)
{
    if (st->lam_pending) finish_step(kp, st);
    if (latch) {
        st->dt = st->dt_fixed > 0.0 ? st->dt_fixed : st->dt_next;
        st->ch = kp.cfl / (st->dt * kp.sinv_fine);
        st->kappa = kp.glm_alpha * st->ch / kp.dmin_fine;
    }
    st->lam_acc[0] = st->lam_acc[1] = st->lam_acc[2] = 0ull;
    st->lam_pending = 1;
}

// the pending maxima, if any, become dt_next (before a host read, and after the
// standalone reduction)
__global__ void k_end(KParams kp, DevState *st)
{
    if (st->lam_pending) finish_step(kp, st);
}

__global__ void k_set_dt(KParams kp, DevState *st, double dt)
{
    if (st->lam_pending) finish_step(kp, st);      // the last substep's dt_next, under the old setting
    st->dt_fixed = dt;
    if (dt > 0.0) st->dt_next = dt;
}

__global__ void k_reset_stats(DevState *st)
{
    st->c2p_fail = 0ull;
    st->floor_hits = 0ull;
    st->c2p_backup = 0ull;
    st->max_iter = 0;
}

// ---------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------
namespace {
inline unsigned nblk(long long n) { return (unsigned)((n + WG - 1) / WG); }
}

const char *const kKernelNames[K_COUNT] = {"fill_ghosts", "flux_x1", "flux_x2", "flux_x3", "update",
                                           "prim2con", "con2prim", "cell_speeds", "step_begin", "step_end",
                                           "block_flux", "update_div", "fill_cross_level", "flux_fix",
                                           "update_x1", "ct_faces", "ct_edges"};

hipError_t launch_fill(const DeviceGrid &G, void *P, hipStream_t s, bool faces_only)
{
    // same-level copies, then the cross-level slots of block trees (whose recipes
    // read interior cells only, so the order does not matter)
    hipError_t e = launch_fill_copies(G, P, s, faces_only);
    if (e != hipSuccess) return e;
    return launch_fill_cross(G, P, s, faces_only);
}

hipError_t launch_fill_copies(const DeviceGrid &G, void *P, hipStream_t s, bool faces_only)
{
    // the face-adjacent slots come first in the gather map (see make_plan)
    const long long n = faces_only ? G.nface_slots : G.nghost_slots;
    if (n == 0) return hipSuccess;
    TimedLaunch tl(G.timer, K_FILL, s);
    const unsigned nchunk = nblk(n);
    const unsigned grid = ((nchunk + NXCD - 1) / NXCD) * NXCD;
    const bool ent = G.kp.nvar > NV;
    if (G.mixed) {
        auto kern = ent ? k_fill<float, NV + 1> : k_fill<float, NV>;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), 0, s, G.d_gdst, G.d_gsrc, n, (const float *)P, (float *)P,
                           G.kp.ncp);
    } else {
        auto kern = ent ? k_fill<double, NV + 1> : k_fill<double, NV>;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(WG), 0, s, G.d_gdst, G.d_gsrc, n, (const double *)P, (double *)P,
                           G.kp.ncp);
    }
    return hipGetLastError();
}

hipError_t launch_fill_cross(const DeviceGrid &G, void *P, hipStream_t s, bool faces_only)
{
    const long long n = faces_only ? G.nxl_face : G.nxl;
    if (n == 0) return hipSuccess;
    TimedLaunch tl(G.timer, K_FILL_XL, s);
    const bool nd3 = G.kp.ndim == 3;
    if (G.mixed) {
        auto kern = nd3 ? k_fill_xl<float, 3> : k_fill_xl<float, 2>;
        hipLaunchKernelGGL(kern, dim3(nblk(n)), dim3(WG), 0, s, G.d_xoff, G.d_xdat, n, (const float *)P, (float *)P,
                           G.kp.ncp);
    } else {
        auto kern = nd3 ? k_fill_xl<double, 3> : k_fill_xl<double, 2>;
        hipLaunchKernelGGL(kern, dim3(nblk(n)), dim3(WG), 0, s, G.d_xoff, G.d_xdat, n, (const double *)P,
                           (double *)P, G.kp.ncp);
    }
    return hipGetLastError();
}

template <typename R, bool KS>
static hipError_t p2c_typed(const DeviceGrid &G, const void *P, double *U, hipStream_t s)
{
    TimedLaunch tl(G.timer, K_PRIM2CON, s);
    hipLaunchKernelGGL((k_prim2con<R, KS>), dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wcell,
                       (const R *)P, U);
    return hipGetLastError();
}

hipError_t launch_prim2con(const DeviceGrid &G, const void *P, double *U, hipStream_t s)
{
    if (G.mixed) return G.ks ? p2c_typed<float, true>(G, P, U, s) : p2c_typed<float, false>(G, P, U, s);
    return G.ks ? p2c_typed<double, true>(G, P, U, s) : p2c_typed<double, false>(G, P, U, s);
}

template <typename R, bool KS>
static hipError_t c2p_typed(const DeviceGrid &G, const double *U, void *P, int8_t *f, hipStream_t s)
{
    TimedLaunch tl(G.timer, K_CON2PRIM, s);
    auto kern = G.kp.nvar > NV ? k_con2prim<R, KS, true> : k_con2prim<R, KS, false>;
    hipLaunchKernelGGL(kern, dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wcell, U, (R *)P, f);
    return hipGetLastError();
}

hipError_t launch_con2prim(const DeviceGrid &G, const double *U, void *P, int8_t *fail, hipStream_t s)
{
    if (G.mixed) return G.ks ? c2p_typed<float, true>(G, U, P, fail, s) : c2p_typed<float, false>(G, U, P, fail, s);
    return G.ks ? c2p_typed<double, true>(G, U, P, fail, s) : c2p_typed<double, false>(G, U, P, fail, s);
}

template <typename R, bool KS>
static hipError_t speeds_typed(const DeviceGrid &G, const void *P, hipStream_t s)
{
    TimedLaunch tl(G.timer, K_SPEEDS, s);
    hipLaunchKernelGGL((k_cell_speeds<R, KS>), dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wcell,
                       (const R *)P);
    return hipGetLastError();
}

static hipError_t begin_step(const DeviceGrid &G, int latch, hipStream_t s)
{
    TimedLaunch tl(G.timer, K_BEGIN, s);
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, s, G.kp, G.d_state, latch);
    return hipGetLastError();
}

static hipError_t end_step(const DeviceGrid &G, hipStream_t s)
{
    TimedLaunch tl(G.timer, K_END, s);
    hipLaunchKernelGGL(k_end, dim3(1), dim3(1), 0, s, G.kp, G.d_state);
    return hipGetLastError();
}

hipError_t launch_compute_dt(const DeviceGrid &G, const void *P, hipStream_t s)
{
    hipError_t e = begin_step(G, 0, s);
    if (e != hipSuccess) return e;
    if (G.mixed) e = G.ks ? speeds_typed<float, true>(G, P, s) : speeds_typed<float, false>(G, P, s);
    else e = G.ks ? speeds_typed<double, true>(G, P, s) : speeds_typed<double, false>(G, P, s);
    if (e != hipSuccess) return e;
    return end_step(G, s);
}

hipError_t launch_set_dt(const DeviceGrid &G, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(1), 0, s, G.kp, G.d_state, dt);
    return hipGetLastError();
}

hipError_t launch_reset_stats(const DeviceGrid &G, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(1), 0, s, G.d_state);
    return hipGetLastError();
}

// block trees (XL) and the entropy field (ENT) never come together (the planner
// rejects that combination), so three variants per direction are launched
template <typename R, int D, int RECON, int FLUX, bool KS>
static hipError_t flux_dir(const DeviceGrid &G, const void *Ps, hipStream_t s, void *const *flux)
{
    const std::vector<WorkItem> &w = G.plan.wface[D];
    TimedLaunch tl(G.timer, K_FLUX0 + D, s);
    const bool xl = G.plan.p.amr != 0, ent = G.kp.nvar > NV;
    if (D == 0 && G.plan.x1_staged) {
        auto kern = xl ? k_flux_x1s<R, RECON, FLUX, KS, true, false>
                       : (ent ? k_flux_x1s<R, RECON, FLUX, KS, false, true> : k_flux_x1s<R, RECON, FLUX, KS, false, false>);
        hipLaunchKernelGGL(kern, dim3(w.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wface[0], (const R *)Ps,
                           (R *)flux[0], G.plan.nface[0], (const double *)nullptr);
        return hipGetLastError();
    }
    auto kern = xl ? k_flux<R, D, RECON, FLUX, KS, true, false>
                   : (ent ? k_flux<R, D, RECON, FLUX, KS, false, true> : k_flux<R, D, RECON, FLUX, KS, false, false>);
    hipLaunchKernelGGL(kern, dim3(w.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wface[D], (const R *)Ps,
                       (R *)flux[D], G.plan.nface[D], (const double *)nullptr);
    return hipGetLastError();
}

template <typename R, bool KS>
static hipError_t update_typed(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                               void *Po, double a, double b, hipStream_t s, void *const *flux)
{
    TimedLaunch tl(G.timer, K_UPDATE, s);
    const bool nd3 = G.kp.ndim == 3, base = a != 0.0;
    auto kern = nd3 ? (base ? k_update<R, KS, true, true, false> : k_update<R, KS, true, false, false>)
                    : (base ? k_update<R, KS, false, true, false> : k_update<R, KS, false, false, false>);
    if (G.kp.nvar > NV)
        kern = nd3 ? (base ? k_update<R, KS, true, true, true> : k_update<R, KS, true, false, true>)
                   : (base ? k_update<R, KS, false, true, true> : k_update<R, KS, false, false, true>);
    hipLaunchKernelGGL(kern, dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wcell, Ub, Us,
                       (const R *)Ps, Uo, (R *)Po, (const R *)flux[0], (const R *)flux[1],
                       (const R *)flux[2], G.plan.nface[0], G.plan.nface[1], G.plan.nface[2], a, b,
                       (const double *)nullptr, (const double *)nullptr, (const double *)nullptr);
    return hipGetLastError();
}

template <typename R, int RECON, int FLUX, bool KS>
static hipError_t update_x1_typed(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps,
                                  double *Uo, void *Po, double a, double b, hipStream_t s, void *const *flux)
{
    TimedLaunch tl(G.timer, K_UPDATE_X1, s);
    const bool nd3 = G.kp.ndim == 3, base = a != 0.0;
    auto kern = nd3 ? (base ? k_update_x1<R, RECON, FLUX, KS, true, true> : k_update_x1<R, RECON, FLUX, KS, true, false>)
                    : (base ? k_update_x1<R, RECON, FLUX, KS, false, true> : k_update_x1<R, RECON, FLUX, KS, false, false>);
    hipLaunchKernelGGL(kern, dim3(G.plan.wupd1.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wupd1, Ub, Us,
                       (const R *)Ps, Uo, (R *)Po, (const R *)flux[1], (const R *)flux[2],
                       G.plan.nface[1], G.plan.nface[2], a, b);
    return hipGetLastError();
}

template <typename R, int RECON, int FLUX, bool KS>
static hipError_t substep_typed(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                                void *Po, double a, double b, hipStream_t s, void *const *flux)
{
    // each direction by faces or by lines, as planned; in 3-D the x2 and x3 kernels
    // run on the grid's side streams, concurrently with x1 on the caller's stream
    // (while kernel timing is on they run one after another on the caller's
    // stream, so that each kernel's measured duration is its own)
    const int mm = G.plan.march_mask;
    auto dir = [&](int d, hipStream_t st) -> hipError_t {
        if (mm >> d & 1) return launch_flux_march(G, d, Ps, st, flux);
        if (d == 0) return flux_dir<R, 0, RECON, FLUX, KS>(G, Ps, st, flux);
        if (d == 1) return flux_dir<R, 1, RECON, FLUX, KS>(G, Ps, st, flux);
        return flux_dir<R, 2, RECON, FLUX, KS>(G, Ps, st, flux);
    };
    hipError_t e = hipSuccess;
    // both x2 and x3 marched on independent patches (GLM, no entropy field): one
    // launch runs both directions' line marches
    const bool x23 = G.kp.ndim == 3 && !G.timer.on && (mm & 6) == 6 && !G.plan.p.amr && G.kp.nvar == NV;
    if (G.plan.x1_in_update) {
        // x2 (and x3 on a side stream, concurrently) by face kernels, then the update,
        // which computes the x1 faces itself
        if (x23) {
            e = launch_flux_march_x23(G, Ps, s, flux);
        } else if (G.kp.ndim == 3 && !G.timer.on) {
            e = hipEventRecord(G.ev_fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(G.side[0], G.ev_fork, 0);
            if (e == hipSuccess) e = dir(2, G.side[0]);
            if (e == hipSuccess) e = dir(1, s);
            if (e == hipSuccess) e = hipEventRecord(G.ev_join[0], G.side[0]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, G.ev_join[0], 0);
        } else {
            e = dir(1, s);
            if (e == hipSuccess && G.kp.ndim == 3) e = dir(2, s);
        }
        if (e == hipSuccess) e = update_x1_typed<R, RECON, FLUX, KS>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
        return e;
    }
    if (x23 && G.side[0]) {
        // x1 on the caller's stream, x2 and x3 in one launch on a side stream
        e = hipEventRecord(G.ev_fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(G.side[0], G.ev_fork, 0);
        if (e == hipSuccess) e = launch_flux_march_x23(G, Ps, G.side[0], flux);
        if (e == hipSuccess) e = dir(0, s);
        if (e == hipSuccess) e = hipEventRecord(G.ev_join[0], G.side[0]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, G.ev_join[0], 0);
    } else if (G.kp.ndim == 3 && G.side[0] && G.side[1] && !G.timer.on) {
        e = hipEventRecord(G.ev_fork, s);
        for (int q = 0; q < 2 && e == hipSuccess; q++) e = hipStreamWaitEvent(G.side[q], G.ev_fork, 0);
        if (e == hipSuccess) e = dir(1, G.side[0]);
        if (e == hipSuccess) e = dir(2, G.side[1]);
        if (e == hipSuccess) e = dir(0, s);
        for (int q = 0; q < 2 && e == hipSuccess; q++) e = hipEventRecord(G.ev_join[q], G.side[q]);
        for (int q = 0; q < 2 && e == hipSuccess; q++) e = hipStreamWaitEvent(s, G.ev_join[q], 0);
    } else {
        e = dir(0, s);
        if (e == hipSuccess) e = dir(1, s);
        if (e == hipSuccess && G.kp.ndim == 3) e = dir(2, s);
    }
    if (e == hipSuccess && G.nffix > 0) {
        TimedLaunch tl(G.timer, K_FLUX_FIX, s);
        auto kern = G.kp.ndim == 3 ? k_flux_fix<R, 4> : k_flux_fix<R, 2>;
        hipLaunchKernelGGL(kern, dim3(nblk(G.nffix)), dim3(WG), 0, s, G.d_ffix, G.nffix,
                           (const R *)flux[0], (const R *)flux[1],
                           (const R *)flux[2], (R *)flux[0], (R *)flux[1], (R *)flux[2],
                           G.plan.nface[0], G.plan.nface[1], G.plan.nface[2]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = update_typed<R, KS>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
    return e;
}

template <typename R, int RECON, int FLUX>
static hipError_t substep_metric(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                                 void *Po, double a, double b, hipStream_t s, void *const *flux)
{
    if (G.ks) return substep_typed<R, RECON, FLUX, true>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
    return substep_typed<R, RECON, FLUX, false>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
}

template <typename R>
static hipError_t substep_prec(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                               void *Po, double a, double b, hipStream_t s, void *const *flux)
{
    const int r = G.kp.recon, f = G.kp.flux;
    if (r == BHAC_RECON_PPM && f == BHAC_FLUX_HLL)
        return substep_metric<R, BHAC_RECON_PPM, BHAC_FLUX_HLL>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
    if (r == BHAC_RECON_PPM)
        return substep_metric<R, BHAC_RECON_PPM, BHAC_FLUX_TVDLF>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
    if (f == BHAC_FLUX_HLL) return substep_metric<R, BHAC_RECON_MC, BHAC_FLUX_HLL>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
    return substep_metric<R, BHAC_RECON_MC, BHAC_FLUX_TVDLF>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
}

hipError_t launch_substep(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                          void *Po, double a, double b, hipStream_t s, void *const *flux)
{
    if (!flux) flux = G.d_flux;
    hipError_t e = begin_step(G, a == 0.0 ? 1 : 0, s);
    if (e != hipSuccess) return e;
    // block trees: the face ghosts bordering other levels are read from P_stage's
    // own ghost slots, refreshed here from its interiors
    if (G.nxl_face > 0) e = launch_fill_cross(G, const_cast<void *>(Ps), s, true);
    if (e != hipSuccess) return e;
    if (G.plan.p.fused) e = launch_fused_body(G, Ub, Us, Ps, Uo, Po, a, b, s);
    else if (G.mixed) e = substep_prec<float>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
    else e = substep_prec<double>(G, Ub, Us, Ps, Uo, Po, a, b, s, flux);
    return e;      // dt_next follows at the next substep's start (or on a host read)
}

hipError_t launch_finish_step(const DeviceGrid &G, hipStream_t s)
{
    return end_step(G, s);
}

// ---------------------------------------------------------------------------------
// Constrained-transport substep: face fluxes (one thread per face, normal field from
// the face field), face-field update per direction, then the cell update.
// ---------------------------------------------------------------------------------
struct CtPtrs {
    const double *b[3], *s[3];
    double *o[3];
};

static CtPtrs ct_split(const DeviceGrid &G, const double *Phb, const double *Phs, double *Pho)
{
    CtPtrs c{};
    long long base = 0;
    for (int d = 0; d < 3; d++) {
        if (d < G.kp.ndim) {
            c.b[d] = Phb ? Phb + base : nullptr;
            c.s[d] = Phs ? Phs + base : nullptr;
            c.o[d] = Pho ? Pho + base : nullptr;
            base += G.plan.nface[d];
        } else {
            c.b[d] = c.s[d] = nullptr;
            c.o[d] = nullptr;
        }
    }
    return c;
}

// face fluxes of direction D under constrained transport, by the form the plan gives
// that direction (line march, LDS-staged x1 faces or one thread per face)
template <typename R, int D, int RECON, int FLUX, bool KS>
static hipError_t ct_flux_dir(const DeviceGrid &G, const void *Ps, const double *phs, hipStream_t s)
{
    void *const *flux = G.d_flux;
    if (G.plan.march_mask >> D & 1) return launch_flux_march(G, D, Ps, s, flux, phs);
    TimedLaunch tl(G.timer, K_FLUX0 + D, s);
    if (D == 0 && G.plan.x1_staged) {
        hipLaunchKernelGGL((k_flux_x1s<R, RECON, FLUX, KS, false, false, true>), dim3(G.plan.wface[0].size()), dim3(WG),
                           0, s, G.kp, G.gd, G.d_wface[0], (const R *)Ps, (R *)G.d_flux[0], G.plan.nface[0], phs);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_flux<R, D, RECON, FLUX, KS, false, false, true>), dim3(G.plan.wface[D].size()), dim3(WG), 0,
                       s, G.kp, G.gd, G.d_wface[D], (const R *)Ps, (R *)G.d_flux[D], G.plan.nface[D], phs);
    return hipGetLastError();
}

template <typename R, int K>
static hipError_t ct_edge_dir(const DeviceGrid &G, const CtFlux &cf, const CtEdge &ce, hipStream_t s)
{
    TimedLaunch tl(G.timer, K_CT_EDGE, s);
    hipLaunchKernelGGL((k_ct_edge<R, K>), dim3(G.plan.wedge[K].size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wedge[K], cf,
                       ce);
    return hipGetLastError();
}

template <int D, bool ND3>
static hipError_t ct_face_dir(const DeviceGrid &G, const CtEdge &ce, const CtPtrs &c, double a, double b, hipStream_t s)
{
    TimedLaunch tl(G.timer, K_CT_FACE, s);
    auto kern = a != 0.0 ? k_ct_face<D, ND3, true> : k_ct_face<D, ND3, false>;
    hipLaunchKernelGGL(kern, dim3(G.plan.wface[D].size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wface[D], ce, c.b[D],
                       c.s[D], c.o[D], a, b);
    return hipGetLastError();
}

template <typename R, int RECON, int FLUX, bool KS>
static hipError_t substep_ct_typed(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps,
                                   const CtPtrs &c, double *Uo, void *Po, double a, double b, hipStream_t s)
{
    const bool nd3 = G.kp.ndim == 3;
    hipError_t e = hipSuccess;
    if (nd3 && G.side[0] && G.side[1] && !G.timer.on) {
        // x2 and x3 on the grid's side streams, concurrently with x1 (as in the GLM substep)
        e = hipEventRecord(G.ev_fork, s);
        for (int q = 0; q < 2 && e == hipSuccess; q++) e = hipStreamWaitEvent(G.side[q], G.ev_fork, 0);
        if (e == hipSuccess) e = ct_flux_dir<R, 1, RECON, FLUX, KS>(G, Ps, c.s[1], G.side[0]);
        if (e == hipSuccess) e = ct_flux_dir<R, 2, RECON, FLUX, KS>(G, Ps, c.s[2], G.side[1]);
        if (e == hipSuccess) e = ct_flux_dir<R, 0, RECON, FLUX, KS>(G, Ps, c.s[0], s);
        for (int q = 0; q < 2 && e == hipSuccess; q++) e = hipEventRecord(G.ev_join[q], G.side[q]);
        for (int q = 0; q < 2 && e == hipSuccess; q++) e = hipStreamWaitEvent(s, G.ev_join[q], 0);
    } else {
        e = ct_flux_dir<R, 0, RECON, FLUX, KS>(G, Ps, c.s[0], s);
        if (e == hipSuccess) e = ct_flux_dir<R, 1, RECON, FLUX, KS>(G, Ps, c.s[1], s);
        if (e == hipSuccess && nd3) e = ct_flux_dir<R, 2, RECON, FLUX, KS>(G, Ps, c.s[2], s);
    }
    // edge fields once per edge, then every face's Stokes update from its four edges
    const CtFlux cf{{G.d_flux[0], G.d_flux[1], G.d_flux[2]}, {G.plan.nface[0], G.plan.nface[1], G.plan.nface[2]}};
    const CtEdge ce{{G.d_edge[0], G.d_edge[1], G.d_edge[2]}, G.d_eofs};
    if (nd3) {
        if (e == hipSuccess) e = ct_edge_dir<R, 0>(G, cf, ce, s);
        if (e == hipSuccess) e = ct_edge_dir<R, 1>(G, cf, ce, s);
    }
    if (e == hipSuccess) e = ct_edge_dir<R, 2>(G, cf, ce, s);
    if (nd3) {
        if (e == hipSuccess) e = ct_face_dir<0, true>(G, ce, c, a, b, s);
        if (e == hipSuccess) e = ct_face_dir<1, true>(G, ce, c, a, b, s);
        if (e == hipSuccess) e = ct_face_dir<2, true>(G, ce, c, a, b, s);
    } else {
        if (e == hipSuccess) e = ct_face_dir<0, false>(G, ce, c, a, b, s);
        if (e == hipSuccess) e = ct_face_dir<1, false>(G, ce, c, a, b, s);
    }
    if (e != hipSuccess) return e;
    TimedLaunch tl(G.timer, K_UPDATE, s);
    const bool base = a != 0.0;
    auto kern = nd3 ? (base ? k_update<R, KS, true, true, false, true> : k_update<R, KS, true, false, false, true>)
                    : (base ? k_update<R, KS, false, true, false, true> : k_update<R, KS, false, false, false, true>);
    hipLaunchKernelGGL(kern, dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wcell, Ub, Us, (const R *)Ps,
                       Uo, (R *)Po, (const R *)G.d_flux[0], (const R *)G.d_flux[1], (const R *)G.d_flux[2],
                       G.plan.nface[0], G.plan.nface[1], G.plan.nface[2], a, b, (const double *)c.o[0],
                       (const double *)c.o[1], (const double *)c.o[2]);
    return hipGetLastError();
}

template <typename R>
static hipError_t substep_ct_prec(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps,
                                  const CtPtrs &c, double *Uo, void *Po, double a, double b, hipStream_t s)
{
    const int r = G.kp.recon, f = G.kp.flux;
#define CT_CASE(RC, FL)                                                                                              \
    return G.ks ? substep_ct_typed<R, RC, FL, true>(G, Ub, Us, Ps, c, Uo, Po, a, b, s)                               \
                : substep_ct_typed<R, RC, FL, false>(G, Ub, Us, Ps, c, Uo, Po, a, b, s)
    if (r == BHAC_RECON_PPM && f == BHAC_FLUX_HLL) CT_CASE(BHAC_RECON_PPM, BHAC_FLUX_HLL);
    if (r == BHAC_RECON_PPM) CT_CASE(BHAC_RECON_PPM, BHAC_FLUX_TVDLF);
    if (f == BHAC_FLUX_HLL) CT_CASE(BHAC_RECON_MC, BHAC_FLUX_HLL);
    CT_CASE(BHAC_RECON_MC, BHAC_FLUX_TVDLF);
#undef CT_CASE
}

hipError_t launch_substep_ct(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, const double *Phb,
                             const double *Phs, double *Uo, void *Po, double *Pho, double a, double b, hipStream_t s)
{
    hipError_t e = begin_step(G, a == 0.0 ? 1 : 0, s);
    if (e != hipSuccess) return e;
    const CtPtrs c = ct_split(G, Phb, Phs, Pho);
    e = G.mixed ? substep_ct_prec<float>(G, Ub, Us, Ps, c, Uo, Po, a, b, s)
                : substep_ct_prec<double>(G, Ub, Us, Ps, c, Uo, Po, a, b, s);
    return e;      // dt_next follows at the next substep's start (or on a host read)
}

hipError_t launch_ct_center(const DeviceGrid &G, const double *Ph, void *P, hipStream_t s)
{
    const CtPtrs c = ct_split(G, Ph, Ph, nullptr);
    if (G.mixed) {
        if (G.ks)
            hipLaunchKernelGGL((k_ct_center<float, true>), dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd,
                               G.d_wcell, c.s[0], c.s[1], c.s[2], (float *)P);
        else
            hipLaunchKernelGGL((k_ct_center<float, false>), dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd,
                               G.d_wcell, c.s[0], c.s[1], c.s[2], (float *)P);
    } else {
        if (G.ks)
            hipLaunchKernelGGL((k_ct_center<double, true>), dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd,
                               G.d_wcell, c.s[0], c.s[1], c.s[2], (double *)P);
        else
            hipLaunchKernelGGL((k_ct_center<double, false>), dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd,
                               G.d_wcell, c.s[0], c.s[1], c.s[2], (double *)P);
    }
    return hipGetLastError();
}

hipError_t launch_ct_div(const DeviceGrid &G, const double *Ph, double *div, hipStream_t s)
{
    const CtPtrs c = ct_split(G, Ph, Ph, nullptr);
    hipLaunchKernelGGL(k_ct_div, dim3(G.plan.wcell.size()), dim3(WG), 0, s, G.kp, G.gd, G.d_wcell, c.s[0], c.s[1],
                       c.s[2], div);
    return hipGetLastError();
}

}  // namespace bhac
