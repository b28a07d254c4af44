// Host-side planning for the GRMHD substep library: parameter and block-list
// validation, the padded state layout, the same-level ghost gather map, fused-kernel
// halo tables, FP64 metric tables and the work lists of the unfused kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <tuple>
#include <type_traits>
#include <unordered_map>

#include "internal.h"

namespace bhac {
namespace {

// ---------------------------------------------------------------------------------
// Kerr-Schild metric in (ln r, theta, phi), M = 1, written once over a scalar type
// so that forward-mode dual numbers give exact first derivatives of every table
// entry (no hand-derived derivative formulas).
// ---------------------------------------------------------------------------------
struct Dual {
    double v, d;
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
inline Dual operator+(double s, Dual a) { return {s + a.v, a.d}; }
inline Dual dsqrt(Dual a) { double r = std::sqrt(a.v); return {r, 0.5 * a.d / r}; }
inline Dual dexp(Dual a) { double e = std::exp(a.v); return {e, e * a.d}; }
inline Dual dsin(Dual a) { return {std::sin(a.v), std::cos(a.v) * a.d}; }
inline Dual dcos(Dual a) { return {std::cos(a.v), -std::sin(a.v) * a.d}; }

// alpha, beta^1, gamma_11, gamma_13, gamma_22, gamma_33 (the only non-zero entries)
struct KsParts { Dual alpha, beta1, g11, g13, g22, g33; };

KsParts ks_parts(double spin, Dual x1, Dual x2)
{
    const Dual r = dexp(x1), st = dsin(x2), ct = dcos(x2);
    const Dual a2c2 = (spin * spin) * (ct * ct);
    const Dual sigma = r * r + a2c2;
    const Dual z = 2.0 * r / sigma;
    const Dual one_z = 1.0 + z;
    const Dual st2 = st * st;
    KsParts k;
    k.alpha = Dual{1.0, 0.0} / dsqrt(one_z);
    k.beta1 = z / (r * one_z);                       // beta^r = z/(1+z), and beta^1 = beta^r / r
    k.g11 = r * r * one_z;                           // gamma_rr r^2
    k.g13 = (-spin) * r * st2 * one_z;               // gamma_r-phi r
    k.g22 = sigma;
    k.g33 = st2 * (sigma + (spin * spin) * st2 * one_z);
    return k;
}

void ks_record(double spin, double x1, double x2, double *rec)
{
    const KsParts v = ks_parts(spin, {x1, 0.0}, {x2, 0.0});
    const KsParts d1 = ks_parts(spin, {x1, 1.0}, {x2, 0.0});
    const KsParts d2 = ks_parts(spin, {x1, 0.0}, {x2, 1.0});
    const double g11 = v.g11.v, g13 = v.g13.v, g22 = v.g22.v, g33 = v.g33.v;
    const double det13 = g11 * g33 - g13 * g13;
    rec[C_ALPHA] = v.alpha.v;
    rec[C_BETA1] = v.beta1.v;
    rec[C_G11] = g11;
    rec[C_G13] = g13;
    rec[C_G22] = g22;
    rec[C_G33] = g33;
    rec[C_GI11] = g33 / det13;
    rec[C_GI13] = -g13 / det13;
    rec[C_GI22] = 1.0 / g22;
    rec[C_GI33] = g11 / det13;
    rec[C_SG] = std::sqrt(det13 * g22);
    rec[C_DA1] = d1.alpha.d;
    rec[C_DA2] = d2.alpha.d;
    rec[C_DB1] = d1.beta1.d;
    rec[C_DB2] = d2.beta1.d;
    rec[C_DG11_1] = d1.g11.d;
    rec[C_DG11_2] = d2.g11.d;
    rec[C_DG13_1] = d1.g13.d;
    rec[C_DG13_2] = d2.g13.d;
    rec[C_DG22_1] = d1.g22.d;
    rec[C_DG22_2] = d2.g22.d;
    rec[C_DG33_1] = d1.g33.d;
    rec[C_DG33_2] = d2.g33.d;
}

// Lattice key of a same-(level, size) slot.
struct Key {
    int level, s0, s1, s2, c0, c1, c2;
    bool operator==(const Key &o) const
    {
        return level == o.level && s0 == o.s0 && s1 == o.s1 && s2 == o.s2 && c0 == o.c0 && c1 == o.c1 &&
               c2 == o.c2;
    }
};
struct KeyHash {
    size_t operator()(const Key &k) const
    {
        uint64_t h = 1469598103934665603ull;
        const int v[7] = {k.level, k.s0, k.s1, k.s2, k.c0, k.c1, k.c2};
        for (int x : v) { h ^= (uint64_t)(uint32_t)x; h *= 1099511628211ull; }
        return (size_t)h;
    }
};

bool bad(std::string &err, const std::string &msg)
{
    err = msg;
    return false;
}

// Index of local position l of block D by the linear rule the kernels use
// (strides 1, s0, s0 s1 from the block's first interior cell): the position's slot
// when it lies inside the block, and the base of the halo shifts otherwise.
long long linear_index(const Plan &, const DevBlock &D, const int l[3])
{
    return D.off + ((long long)l[2] * D.n1 + l[1]) * D.n0 + l[0];
}

// Slot of local position l (interior cell or ghost slot) in block D's region of P:
// the interior cells (x fastest), then the ghost slots of the (size + 2g) box in
// box order (x fastest) with the interior skipped.
long long slot_index(const Plan &P, const DevBlock &D, const int l[3])
{
    bool in = true;
    for (int e = 0; e < 3; e++) in = in && l[e] >= 0 && l[e] < D.s[e];
    if (in) return linear_index(P, D, l);
    const int g0 = P.gd[0], g1 = P.gd[1], g2 = P.gd[2];
    const long long n0 = D.s[0] + 2 * g0, n1 = D.s[1] + 2 * g1;
    const int pi = l[0] + g0, pj = l[1] + g1, pk = l[2] + g2;
    long long r = pk * n0 * n1 - (long long)D.s[0] * D.s[1] * std::clamp(pk - g2, 0, D.s[2]);
    if (pk < g2 || pk >= D.s[2] + g2) {
        r += pj * n0 + pi;
    } else {
        r += pj * n0 - (long long)D.s[0] * std::clamp(pj - g1, 0, D.s[1]);
        r += (pj < g1 || pj >= D.s[1] + g1) ? pi : (pi < g0 ? pi : pi - D.s[0]);
    }
    return D.off + (long long)D.s[0] * D.s[1] * D.s[2] + r;
}

bool check_params(const bhac_params &p, std::string &err)
{
    if (p.ndim != 2 && p.ndim != 3) return bad(err, "ndim must be 2 or 3");
    if (p.metric != BHAC_METRIC_MINKOWSKI_CART && p.metric != BHAC_METRIC_KS_SPH_LOGR)
        return bad(err, "unknown metric");
    if (p.recon != BHAC_RECON_MC && p.recon != BHAC_RECON_PPM) return bad(err, "unknown reconstruction");
    if (p.flux != BHAC_FLUX_HLL && p.flux != BHAC_FLUX_TVDLF) return bad(err, "unknown flux");
    if (p.precision != BHAC_PREC_FP64 && p.precision != BHAC_PREC_MIXED) return bad(err, "unknown precision");
    if (p.fused != 0 && p.fused != 1) return bad(err, "fused must be 0 or 1");
    if (p.amr != 0 && p.amr != 1) return bad(err, "amr must be 0 or 1");
    if (p.entropy != 0 && p.entropy != 1) return bad(err, "entropy must be 0 or 1");
    if (p.ct != 0 && p.ct != 1) return bad(err, "ct must be 0 or 1");
    if (p.entropy && !(p.gamma_ad <= 2.0)) return bad(err, "the entropy backup needs gamma_ad <= 2");
    if (p.sched.set != 0 && p.sched.set != 1) return bad(err, "sched.set must be 0 or 1");
    if (p.sched.set) {
        if (p.sched.march_mask < 0 || p.sched.march_mask > 7) return bad(err, "sched.march_mask must be in [0, 7]");
        if (p.sched.march_faces < 4 || p.sched.march_faces > 256) return bad(err, "sched.march_faces must be in [4, 256]");
        if (p.sched.x1_staged < 0 || p.sched.x1_staged > 2) return bad(err, "sched.x1_staged must be 0, 1 or 2");
    }
    const int gmin = p.recon == BHAC_RECON_PPM ? 3 : 2;
    if (p.nghost < gmin || p.nghost > 8) return bad(err, "nghost must be >= 2 (MC) or >= 3 (PPM) and <= 8");
    if (!(std::fabs(p.spin) < 1.0)) return bad(err, "|spin| must be < 1");
    if (!(p.gamma_ad > 1.0)) return bad(err, "gamma_ad must be > 1");
    if (!(p.cfl > 0.0) || !(p.glm_alpha >= 0.0)) return bad(err, "cfl must be > 0 and glm_alpha >= 0");
    if (!(p.rho_floor >= 0.0) || !(p.p_floor >= 0.0) || !(p.w_max > 1.0)) return bad(err, "bad floors");
    if (!(p.c2p_tol > 0.0) || p.c2p_maxit < 1 || p.c2p_maxit > 1000) return bad(err, "bad inversion controls");
    for (int e = 0; e < 3; e++) {
        if (p.ncell0[e] < 1) return bad(err, "ncell0 must be >= 1");
        if (e >= p.ndim) {
            if (p.ncell0[e] != 1) return bad(err, "ncell0 along an unused axis must be 1");
            continue;
        }
        if (!(p.x_hi[e] > p.x_lo[e])) return bad(err, "x_hi must exceed x_lo");
        for (int s = 0; s < 2; s++)
            if (p.bc[e][s] != BHAC_BC_PERIODIC && p.bc[e][s] != BHAC_BC_OUTFLOW) return bad(err, "unknown bc");
        if ((p.bc[e][0] == BHAC_BC_PERIODIC) != (p.bc[e][1] == BHAC_BC_PERIODIC))
            return bad(err, "periodic boundaries must be periodic on both sides");
    }
    if (p.metric == BHAC_METRIC_KS_SPH_LOGR && !(p.x_lo[1] > 0.0 && p.x_hi[1] < M_PI))
        return bad(err, "Kerr-Schild theta range must lie inside (0, pi)");
    return true;
}

}  // namespace

int make_plan(const bhac_params *pp, const bhac_block_desc *blocks, int64_t nb, bool tables, Plan &P,
              std::string &err)
{
    if (!pp || !blocks || nb <= 0) { err = "null params/blocks or nblocks <= 0"; return BHAC_EINVAL; }
    const bhac_params &p = *pp;
    if (!check_params(p, err)) return BHAC_EINVAL;
    if (nb > (1ll << 30)) { err = "too many blocks"; return BHAC_EINVAL; }
    P.p = p;
    P.blocks.assign(blocks, blocks + nb);
    for (int e = 0; e < 3; e++) P.gd[e] = e < p.ndim ? p.nghost : 0;
    // State layout of a block's region of P: the interior cells first, contiguous
    // and x fastest like U (consecutive 16-cell interior rows fill whole 128-byte
    // lines, read and written without partial lines), then the ghost slots in box
    // order; the region is rounded to 32 elements so that every block starts on a
    // line. The kernels index interior cells linearly (strides 1, s0, s0 s1) and
    // reach the few ghost slots they read (cross-level halos of block trees) by
    // the slot rule.

    // blocks, lattice occupancy, layout
    std::unordered_map<Key, int, KeyHash> lattice;
    lattice.reserve((size_t)nb * 2);
    P.off.assign(nb + 1, 0);
    P.ioff.assign(nb + 1, 0);
    P.dblocks.resize(nb);
    P.maxlevel = 0;
    P.ncell_interior = 0;
    for (int e = 0; e < 3; e++) P.smax[e] = 0;
    for (int64_t b = 0; b < nb; b++) {
        const bhac_block_desc &B = blocks[b];
        if (B.level < 0 || B.level > 16) { err = "block level out of range"; return BHAC_EINVAL; }
        for (int e = 0; e < 3; e++) {
            if (e >= p.ndim) {
                if (B.size[e] != 1 || B.origin[e] != 0) { err = "unused axis needs size 1, origin 0"; return BHAC_EINVAL; }
                continue;
            }
            const long long N = (long long)p.ncell0[e] << B.level;
            if (B.size[e] < p.nghost || B.size[e] > 1024) { err = "block size must be in [nghost, 1024]"; return BHAC_EINVAL; }
            if (N % B.size[e] != 0) { err = "block size must divide the level's cell count"; return BHAC_EINVAL; }
            if (B.origin[e] < 0 || B.origin[e] % B.size[e] != 0 || B.origin[e] + B.size[e] > N) {
                err = "block origin must lie on its size lattice inside the domain";
                return BHAC_EINVAL;
            }
        }
        Key k{B.level, B.size[0], B.size[1], B.size[2], B.origin[0] / B.size[0], B.origin[1] / B.size[1],
              B.origin[2] / B.size[2]};
        if (!lattice.emplace(k, (int)b).second) { err = "two blocks occupy one lattice slot"; return BHAC_EINVAL; }
        if (B.level > P.maxlevel) P.maxlevel = B.level;
        DevBlock &D = P.dblocks[b];
        for (int e = 0; e < 3; e++) {
            D.s[e] = B.size[e];
            D.o[e] = B.origin[e];
            if (B.size[e] > P.smax[e]) P.smax[e] = B.size[e];
        }
        D.n0 = B.size[0];
        D.n1 = B.size[1];
        const long long box =
            (long long)(B.size[0] + 2 * P.gd[0]) * (B.size[1] + 2 * P.gd[1]) * (B.size[2] + 2 * P.gd[2]);
        const long long ncell = (box + 31) / 32 * 32;
        D.level = B.level;
        D.off = P.off[b];
        D.ioff = P.ncell_interior;
        P.off[b + 1] = P.off[b] + ncell;
        P.ncell_interior += (long long)B.size[0] * B.size[1] * B.size[2];
        P.ioff[b + 1] = P.ncell_interior;
    }
    if (P.off[nb] >= (1ll << 31)) { err = "more than 2^31 padded cells"; return BHAC_EINVAL; }
    // block tree: one block size, even along every axis in use, no leaf inside the
    // region of another (no ancestor slot occupied)
    auto leaf_at = [&](int level, const long long c[3]) -> int {
        Key k{level, blocks[0].size[0], blocks[0].size[1], blocks[0].size[2], 0, 0, 0};
        for (int e = 0; e < 3; e++) {
            const long long N = e < p.ndim ? ((long long)p.ncell0[e] << level) : 1;
            if (level < 0 || c[e] < 0 || c[e] >= N) return -1;
        }
        k.c0 = (int)(c[0] / blocks[0].size[0]);
        k.c1 = (int)(c[1] / blocks[0].size[1]);
        k.c2 = (int)(c[2] / blocks[0].size[2]);
        auto it = lattice.find(k);
        return it == lattice.end() ? -1 : it->second;
    };
    if (p.ct && (p.fused || p.amr || p.entropy)) {
        err = "constrained transport needs the unfused substep (fused = 0) on independent patches (amr = 0) "
              "without the entropy field";
        return BHAC_EUNSUPPORTED;
    }
    if (p.entropy && (p.fused || p.amr)) {
        err = "the entropy field needs the unfused substep (fused = 0) on independent patches (amr = 0)";
        return BHAC_EUNSUPPORTED;
    }
    if (p.amr) {
        if (p.fused) { err = "the block-tiled substep does not support block trees (amr = 1)"; return BHAC_EUNSUPPORTED; }
        for (int64_t b = 0; b < nb; b++) {
            const bhac_block_desc &B = blocks[b];
            for (int e = 0; e < 3; e++) {
                if (B.size[e] != blocks[0].size[e]) { err = "a block tree needs one block size"; return BHAC_EINVAL; }
                if (e < p.ndim && (B.size[e] % 2 || B.size[e] < 2 * p.nghost)) {
                    // even, and deep enough that every ghost layer lies in an adjacent leaf
                    err = "a block tree needs even block sizes of at least 2 * nghost";
                    return BHAC_EINVAL;
                }
            }
            for (int l = 0; l < B.level; l++) {
                long long c[3];
                for (int e = 0; e < 3; e++) c[e] = e < p.ndim ? ((long long)B.origin[e] >> (B.level - l)) : 0;
                if (leaf_at(l, c) >= 0) { err = "block tree: a leaf lies inside a coarser leaf"; return BHAC_EINVAL; }
            }
        }
    }

    // levels
    P.levels.assign(P.maxlevel + 1, DevLevel{});
    for (int l = 0; l <= P.maxlevel; l++) {
        DevLevel &L = P.levels[l];
        for (int e = 0; e < 3; e++) {
            L.dx[e] = (p.x_hi[e] - p.x_lo[e]) / ((double)p.ncell0[e] * (double)(1 << l));
            L.inv_dx[e] = 1.0 / L.dx[e];
        }
        L.N0 = p.ncell0[0] << l;
        L.N1 = p.ncell0[1] << l;
    }

    // face offsets and work lists
    for (int d = 0; d < 3; d++) { P.wface[d].clear(); P.wmarch[d].clear(); P.nface[d] = 0; }
    P.wcell.clear();
    for (int64_t b = 0; b < nb; b++) {
        DevBlock &D = P.dblocks[b];
        const long long nc = (long long)D.s[0] * D.s[1] * D.s[2];
        for (long long st = 0; st < nc; st += WG) P.wcell.push_back({(int)b, (int)st});
        for (int d = 0; d < p.ndim; d++) {
            const long long nf = (long long)(D.s[0] + (d == 0)) * (D.s[1] + (d == 1)) * (D.s[2] + (d == 2));
            D.fofs[d] = P.nface[d];
            P.nface[d] += nf;
        }
        for (int d = p.ndim; d < 3; d++) D.fofs[d] = 0;
    }
    // face work of direction d walks the blocks in rows along d (level, size, the
    // other two lattice coordinates, then the coordinate along d), so the blocks
    // whose interiors a block's stencils reach are its neighbours in the list and,
    // after the XCD split below, mostly on the same XCD (one L2)
    const int march_faces = p.sched.set ? p.sched.march_faces
                                        : (p.precision == BHAC_PREC_MIXED ? MARCH_FACES_F32 : MARCH_FACES_F64);
    P.march_faces = march_faces;
    for (int d = 0; d < p.ndim; d++) {
        std::vector<int> ord(nb);
        for (int64_t b = 0; b < nb; b++) ord[b] = (int)b;
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        auto key = [&](int b) {
            const bhac_block_desc &B = blocks[b];
            return std::make_tuple(B.level, B.size[0], B.size[1], B.size[2], B.origin[e2] / B.size[e2],
                                   B.origin[e1] / B.size[e1], B.origin[d] / B.size[d]);
        };
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key(a) < key(b); });
        for (int b : ord) {
            const DevBlock &D = P.dblocks[b];
            const long long nf = (long long)(D.s[0] + (d == 0)) * (D.s[1] + (d == 1)) * (D.s[2] + (d == 2));
            for (long long st = 0; st < nf; st += WG) P.wface[d].push_back({b, (int)st});
            // lines along d: MWG per item, faces cut into nseg near-equal segments
            const int a = d == 0 ? 1 : 0, c = d == 2 ? 1 : 2;
            const int nline = D.s[a] * D.s[c], nfd = D.s[d] + 1;
            const int nseg = (nfd + march_faces - 1) / march_faces;
            for (int l0 = 0; l0 < nline; l0 += MWG)
                for (int q = 0; q < nseg; q++)
                    P.wmarch[d].push_back({b, l0, (int)((long long)nfd * q / nseg), (int)((long long)nfd * (q + 1) / nseg)});
        }
    }
    P.march_mask = (p.sched.set ? p.sched.march_mask : p.precision == BHAC_PREC_MIXED ? MARCH_MASK_F32 : MARCH_MASK_F64) &
                   ((1 << p.ndim) - 1);
    // staged x1 faces when every block's rows fit the LDS tile: a work-group's WG
    // consecutive faces touch at most ceil(WG / (s0 + 1)) + 1 rows of s0 + 6 cells
    {
        const int cap = p.precision == BHAC_PREC_MIXED ? x1s_max_cells<float>() : x1s_max_cells<double>();
        bool ok = !(P.march_mask & 1) && (!p.sched.set || p.sched.x1_staged);
        for (int64_t b = 0; b < nb && ok; b++) {
            const int s0 = P.dblocks[b].s[0];
            const int rows = (WG + s0) / (s0 + 1) + 1;
            ok = s0 >= 3 && rows * (s0 + 6) <= cap;
        }
        P.x1_staged = ok;
    }
    // x1 faces inside the update: independent patches without the entropy field,
    // x1 not marched, every block's rows fit the LDS tile
    {
        const int cap = p.precision == BHAC_PREC_MIXED ? x1s_max_cells<float>() : x1s_max_cells<double>();
        const int want = p.sched.set ? p.sched.x1_staged
                                     : (p.precision == BHAC_PREC_MIXED ? X1_IN_UPDATE_DEFAULT_F32 : X1_IN_UPDATE_DEFAULT_F64);
        bool ok = want == 2 && !p.amr && !p.entropy && !p.fused && !p.ct && !(P.march_mask & 1);
        for (int64_t b = 0; b < nb && ok; b++) {
            const int s0 = P.dblocks[b].s[0];
            ok = s0 >= 3 && x1u_rows(s0) >= 1 && x1u_rows(s0) * (s0 + 6) <= cap;
        }
        P.x1_in_update = ok;
        P.wupd1.clear();
        if (ok) {
            P.x1_staged = false;
            // blocks in rows along x1 (as the x1 face work): a work item's x1 halo
            // pieces are the end cells of its x1 neighbours' rows, which their own
            // work items read at about the same time on the same XCD (one L2)
            std::vector<int> ord(nb);
            for (int64_t b = 0; b < nb; b++) ord[b] = (int)b;
            auto key = [&](int b) {
                const bhac_block_desc &B = blocks[b];
                return std::make_tuple(B.level, B.size[0], B.size[1], B.size[2], B.origin[2] / B.size[2],
                                       B.origin[1] / B.size[1], B.origin[0] / B.size[0]);
            };
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key(a) < key(b); });
            for (int b : ord) {
                const DevBlock &D = P.dblocks[b];
                const int rpw = x1u_rows(D.s[0]), nrow = D.s[1] * D.s[2];
                for (int r = 0; r < nrow; r += rpw) P.wupd1.push_back({b, r});
            }
        }
    }

    // constrained transport: edges along K (every direction in 3-D, x3 only in 2-D)
    P.eofs.assign(p.ct ? (size_t)nb * 3 : 0, 0);
    for (int K = 0; K < 3; K++) {
        P.wedge[K].clear();
        P.nedge[K] = 0;
    }
    if (p.ct)
        for (int64_t b = 0; b < nb; b++)
            for (int K = p.ndim == 3 ? 0 : 2; K < 3; K++) {
                const DevBlock &D = P.dblocks[b];
                const long long ne = (long long)(D.s[0] + (K != 0)) * (D.s[1] + (K != 1)) * (D.s[2] + (K != 2));
                P.eofs[(size_t)b * 3 + K] = P.nedge[K];
                P.nedge[K] += ne;
                for (long long st = 0; st < ne; st += WG) P.wedge[K].push_back({(int)b, (int)st});
            }

    // XCD-aware order: work-group p runs on XCD p % NXCD, so item q is placed at
    // p = (q % per) * NXCD + q / per. Each XCD then walks a contiguous range of items
    // (neighbouring planes and blocks share its L2). Padding entries have block -1.
    auto xcd_order = [](auto &w, auto pad) {
        const size_t n = w.size(), per = (n + NXCD - 1) / NXCD;
        std::remove_reference_t<decltype(w)> out(per * NXCD, pad);
        for (size_t q = 0; q < n; q++) out[(q % per) * NXCD + q / per] = w[q];
        w.swap(out);
    };
    xcd_order(P.wcell, WorkItem{-1, 0});
    xcd_order(P.wupd1, WorkItem{-1, 0});
    for (int K = 0; K < 3; K++) xcd_order(P.wedge[K], WorkItem{-1, 0});
    for (int d = 0; d < p.ndim; d++) {
        xcd_order(P.wface[d], WorkItem{-1, 0});
        xcd_order(P.wmarch[d], MarchItem{-1, 0, 0, 0});
    }

    // halo sources per axis and neighbour slots (used by the gather map and the fused kernel)
    const int g = p.nghost;
    P.hmax = 0;
    for (int e = 0; e < 3; e++) P.hmax = std::max(P.hmax, P.smax[e] + 2 * P.gd[e]);
    P.halo.assign((size_t)nb * 3 * P.hmax, HaloAxis{0, 0, 0});
    P.nbr.assign((size_t)nb * 27, -1);
    for (int64_t b = 0; b < nb; b++) {
        const bhac_block_desc &B = blocks[b];
        int own[3], slot_of_dir[3][3];
        for (int e = 0; e < 3; e++) {
            own[e] = B.origin[e] / B.size[e];
            const long long N = e < p.ndim ? ((long long)p.ncell0[e] << B.level) : 1;
            const int ge = P.gd[e];
            for (int dd = 0; dd < 3; dd++) slot_of_dir[e][dd] = own[e];
            for (int l = -ge; l < B.size[e] + ge; l++) {
                long long G = B.origin[e] + l;
                if (G < 0 || G >= N) {
                    if (p.bc[e][G < 0 ? 0 : 1] == BHAC_BC_PERIODIC) G = ((G % N) + N) % N;
                    else G = G < 0 ? 0 : N - 1;
                }
                const int slot = (int)(G / B.size[e]);
                int dir = 0;
                if (slot != own[e]) dir = l < 0 ? -1 : 1;
                slot_of_dir[e][dir + 1] = slot;
                HaloAxis &h = P.halo[((size_t)b * 3 + e) * P.hmax + (l + ge)];
                h.dir = (signed char)dir;
                h.src = (short)(G - (long long)slot * B.size[e]);
            }
        }
        for (int d2 = 0; d2 < 3; d2++)
            for (int d1 = 0; d1 < 3; d1++)
                for (int d0 = 0; d0 < 3; d0++) {
                    Key k{B.level, B.size[0], B.size[1], B.size[2], slot_of_dir[0][d0], slot_of_dir[1][d1],
                          slot_of_dir[2][d2]};
                    auto it = lattice.find(k);
                    P.nbr[(size_t)b * 27 + d0 + 3 * d1 + 9 * d2] = it == lattice.end() ? -1 : it->second;
                }
    }

    // Block-tree helpers: the global level-L index of a block-local position after
    // the domain's periodic wrap / outflow clamp, the padded index of a cell given by
    // its global index, and the cross-level recipes.
    auto wrap_axis = [&](int level, int e, long long x) -> long long {
        if (e >= p.ndim) return 0;
        const long long N = (long long)p.ncell0[e] << level;
        if (x < 0 || x >= N) {
            if (p.bc[e][x < 0 ? 0 : 1] == BHAC_BC_PERIODIC) x = ((x % N) + N) % N;
            else x = x < 0 ? 0 : N - 1;
        }
        return x;
    };
    auto padded_global = [&](int blk, const long long g[3]) -> int32_t {
        const DevBlock &Q = P.dblocks[blk];
        int li[3];
        for (int e = 0; e < 3; e++) li[e] = (int)(g[e] - Q.o[e]);
        return (int32_t)slot_index(P, Q, li);
    };
    auto padded_local = [&](int blk, const int a[3]) -> int32_t {
        return (int32_t)slot_index(P, P.dblocks[blk], a);
    };
    const int nchild = p.ndim == 3 ? 8 : 4;
    // the 2^ndim cells of the level-(L+1) leaf fb under level-L cell Gi, z-outer
    auto push_children = [&](int fb, const long long Gi[3], std::vector<int32_t> &out) {
        for (int dz = 0; dz < (p.ndim == 3 ? 2 : 1); dz++)
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++) {
                    const long long f[3] = {2 * Gi[0] + dx, 2 * Gi[1] + dy, p.ndim == 3 ? 2 * Gi[2] + dz : 0};
                    out.push_back(padded_global(fb, f));
                }
    };
    // the value of block cb at local a (inside, or one cell outside along one axis)
    // as a list of cells to average: 1 cell, 2^ndim cells, or none where it would
    // need prolongation
    auto neighbour_ref = [&](int cb, const int a[3], std::vector<int32_t> &out) {
        const DevBlock &C = P.dblocks[cb];
        bool inside = true;
        for (int e = 0; e < 3; e++) inside = inside && a[e] >= 0 && a[e] < C.s[e];
        if (inside) { out.push_back(1); out.push_back(padded_local(cb, a)); return; }
        long long Ga[3];
        for (int e = 0; e < 3; e++) Ga[e] = wrap_axis(C.level, e, (long long)C.o[e] + a[e]);
        int q = leaf_at(C.level, Ga);
        if (q >= 0) { out.push_back(1); out.push_back(padded_global(q, Ga)); return; }
        const long long f[3] = {2 * Ga[0], 2 * Ga[1], p.ndim == 3 ? 2 * Ga[2] : 0};
        q = leaf_at(C.level + 1, f);
        if (q >= 0) { out.push_back(nchild); push_children(q, Ga, out); return; }
        if (C.level >= 1) {
            const long long c[3] = {Ga[0] >> 1, Ga[1] >> 1, Ga[2] >> 1};
            if (leaf_at(C.level - 1, c) >= 0) { out.push_back(0); return; }
        }
        int x[3];
        for (int e = 0; e < 3; e++) x[e] = std::min(std::max(a[e], 0), C.s[e] - 1);
        out.push_back(1);
        out.push_back(padded_local(cb, x));
    };
    // Cross-level case of ghost position l of block b when no same-level leaf holds
    // it. Returns 0 when no finer or coarser leaf does either (the zero-gradient copy
    // applies); 1 for a restriction, with rec = [0, dst, 2^ndim cells]; 2 for a
    // prolongation, with the coarse block and cell in cb, lc and the position's
    // upper-half bits in bits. Prolongations are grouped per (block, coarse cell):
    // the children of one coarse cell share its slopes, so a group's recipe is
    // [1, nchildren, coarse cell, the counts of the six neighbours (lower, upper per
    // axis; 0 = no slope), their cells, then (dst, bits) per child].
    auto cross_case = [&](int b, const int l[3], int32_t dst, std::vector<int32_t> &rec, int &cb, int lc[3],
                          int &bits) -> int {
        const DevBlock &B = P.dblocks[b];
        long long Gi[3];
        for (int e = 0; e < 3; e++) Gi[e] = wrap_axis(B.level, e, (long long)B.o[e] + l[e]);
        const long long f[3] = {2 * Gi[0], 2 * Gi[1], p.ndim == 3 ? 2 * Gi[2] : 0};
        const int fb = leaf_at(B.level + 1, f);
        if (fb >= 0) {
            rec.push_back(0);
            rec.push_back(dst);
            push_children(fb, Gi, rec);
            return 1;
        }
        if (B.level < 1) return 0;
        const long long c[3] = {Gi[0] >> 1, Gi[1] >> 1, Gi[2] >> 1};
        cb = leaf_at(B.level - 1, c);
        if (cb < 0) return 0;
        const DevBlock &C = P.dblocks[cb];
        bits = 0;
        for (int d = 0; d < p.ndim; d++) bits |= (int)(Gi[d] & 1) << d;
        for (int e = 0; e < 3; e++) lc[e] = (int)(c[e] - C.o[e]);
        return 2;
    };
    // coarse cell, the six neighbour counts (zero for unused axes), then the cells
    auto prolong_head = [&](int cb, const int lc[3], std::vector<int32_t> &out) {
        out.push_back(padded_local(cb, lc));
        std::vector<int32_t> refs;
        int32_t cnt[6] = {0, 0, 0, 0, 0, 0};
        for (int d = 0; d < p.ndim; d++)
            for (int sd = 0; sd < 2; sd++) {
                int a[3] = {lc[0], lc[1], lc[2]};
                a[d] += sd == 0 ? -1 : 1;
                std::vector<int32_t> one;
                neighbour_ref(cb, a, one);
                cnt[2 * d + sd] = one[0];
                refs.insert(refs.end(), one.begin() + 1, one.end());
            }
        out.insert(out.end(), cnt, cnt + 6);
        out.insert(out.end(), refs.begin(), refs.end());
    };

    // halo sides: for each block, axis and side, either the neighbour whose interior
    // continues the block (same size, so local index l maps to l +- s there) or the
    // zero-gradient clamp to the block's own edge cell. The unfused flux kernels read
    // their halo through these; the face part of the gather map below is checked
    // against them.
    for (int64_t b = 0; b < nb; b++) {
        DevBlock &D = P.dblocks[b];
        D.hclamp = 0;
        D.hxl = 0;
        for (int e = 0; e < 3; e++) {
            D.hshift[e][0] = D.hshift[e][1] = 0;
            if (e >= p.ndim) continue;
            const long long st = e == 0 ? 1 : (e == 1 ? (long long)D.n0 : (long long)D.n0 * D.n1);
            const int pw = e == 0 ? 1 : (e == 1 ? 3 : 9);
            for (int side = 0; side < 2; side++) {
                const int l = side == 0 ? -1 : D.s[e];
                const HaloAxis &h = P.halo[((size_t)b * 3 + e) * P.hmax + (l + P.gd[e])];
                const int nbk = P.nbr[(size_t)b * 27 + 13 + h.dir * pw];
                const int cont = side == 0 ? D.s[e] - 1 : 0;    // source index of a continuation
                std::vector<int32_t> probe;
                const int lp[3] = {e == 0 ? l : 0, e == 1 ? l : 0, e == 2 ? l : 0};
                int pcb, plc[3], pbits;
                if (nbk >= 0 && h.src == cont) {
                    D.hshift[e][side] = P.off[nbk] - P.off[b] + (side == 0 ? 1 : -1) * (long long)D.s[e] * st;
                } else if (p.amr && nbk < 0 && h.dir != 0 && cross_case((int)b, lp, 0, probe, pcb, plc, pbits)) {
                    // a coarser or finer leaf: the kernels read the block's own ghost
                    // slots (shift 0), which the cross-level fill refreshes
                    D.hshift[e][side] = 0;
                    D.hxl |= 1 << (2 * e + side);
                } else if (nbk < 0 || (h.dir == 0 && h.src == (side == 0 ? 0 : D.s[e] - 1))) {
                    D.hclamp |= 1 << (2 * e + side);
                } else {
                    err = "internal: unexpected halo source";
                    return BHAC_EINVAL;
                }
            }
        }
    }

    // same-level ghost gather map, one entry per ghost slot in padded order: the
    // slots with exactly one coordinate outside the block (the face slabs, which
    // are all a dimension-by-dimension stencil reads) first, then edges and corners
    P.gdst.clear();
    P.gsrc.clear();
    std::vector<int32_t> edst, esrc;
    // cross-level recipes (block trees), face slots first as for the gather map;
    // prolongation groups keyed by (block, coarse cell), per face/edge class
    std::vector<int32_t> xface, xedge;
    std::vector<int32_t> xface_off, xedge_off;
    struct PGroup { int cb; int lc[3]; std::vector<int32_t> kids; };
    std::vector<PGroup> pgroups[2];
    std::unordered_map<long long, size_t> pindex[2];
    for (int64_t b = 0; b < nb; b++) {
        const DevBlock &D = P.dblocks[b];
        for (int lk = -P.gd[2]; lk < D.s[2] + P.gd[2]; lk++)
            for (int lj = -P.gd[1]; lj < D.s[1] + P.gd[1]; lj++)
                for (int li = -P.gd[0]; li < D.s[0] + P.gd[0]; li++) {
                    const int l[3] = {li, lj, lk};
                    int nout = 0;
                    for (int e = 0; e < 3; e++) nout += (l[e] < 0 || l[e] >= D.s[e]);
                    if (nout == 0) continue;
                    int dir[3], src[3];
                    for (int e = 0; e < 3; e++) {
                        const HaloAxis &h = P.halo[((size_t)b * 3 + e) * P.hmax + (l[e] + P.gd[e])];
                        dir[e] = h.dir;
                        src[e] = h.src;
                    }
                    int sb = P.nbr[(size_t)b * 27 + (dir[0] + 1) + 3 * (dir[1] + 1) + 9 * (dir[2] + 1)];
                    const long long to = slot_index(P, D, l);
                    int fe = 0;                                  // axis outside (face slots)
                    while (nout == 1 && l[fe] >= 0 && l[fe] < D.s[fe]) fe++;
                    const int fside = nout == 1 && l[fe] >= D.s[fe] ? 1 : 0;
                    if (sb < 0 && p.amr) {
                        std::vector<int32_t> &xs = nout == 1 ? xface : xedge;
                        std::vector<int32_t> &xo = nout == 1 ? xface_off : xedge_off;
                        const size_t at = xs.size();
                        int ccb, clc[3], cbits;
                        const int kind = cross_case((int)b, l, (int32_t)to, xs, ccb, clc, cbits);
                        if (kind == 1) xo.push_back((int32_t)at);
                        if (kind == 2) {
                            const int cls = nout == 1 ? 0 : 1;
                            const long long key = ((long long)b << 32) | (long long)padded_local(ccb, clc);
                            auto it = pindex[cls].find(key);
                            if (it == pindex[cls].end()) {
                                it = pindex[cls].emplace(key, pgroups[cls].size()).first;
                                pgroups[cls].push_back(PGroup{ccb, {clc[0], clc[1], clc[2]}, {}});
                            }
                            pgroups[cls][it->second].kids.push_back((int32_t)to);
                            pgroups[cls][it->second].kids.push_back(cbits);
                        }
                        if (kind) {
                            if (nout == 1 && !(D.hxl >> (2 * fe + fside) & 1)) {
                                err = "block tree: a block face mixes levels (block " + std::to_string(b) + ", axis " +
                                      std::to_string(fe) + ", side " + std::to_string(fside) + ", local " +
                                      std::to_string(l[0]) + "," + std::to_string(l[1]) + "," + std::to_string(l[2]) + ", A)";
                                return BHAC_EINVAL;
                            }
                            continue;
                        }
                    }
                    if (nout == 1 && (D.hxl >> (2 * fe + fside) & 1)) {
                        err = "block tree: a block face mixes levels (block " + std::to_string(b) + ", axis " +
                              std::to_string(fe) + ", side " + std::to_string(fside) + ", local " +
                              std::to_string(l[0]) + "," + std::to_string(l[1]) + "," + std::to_string(l[2]) + ", B)";
                        return BHAC_EINVAL;
                    }
                    if (sb < 0) {
                        sb = (int)b;
                        for (int e = 0; e < 3; e++) src[e] = std::min(std::max(l[e], 0), D.s[e] - 1);
                    }
                    const DevBlock &S = P.dblocks[sb];
                    const long long from = slot_index(P, S, src);
                    if (nout == 1) {
                        // the halo-side rule must name the same source cell
                        int e = 0;
                        while (l[e] >= 0 && l[e] < D.s[e]) e++;
                        const int side = l[e] < 0 ? 0 : 1;
                        const long long st = e == 0 ? 1 : (e == 1 ? (long long)D.n0 : (long long)D.n0 * D.n1);
                        // the kernels address the halo from the linear index of l
                        const long long lin = linear_index(P, D, l);
                        long long expect;
                        if (D.hclamp >> (2 * e + side) & 1)
                            expect = lin + (long long)((side == 0 ? 0 : D.s[e] - 1) - l[e]) * st;
                        else
                            expect = lin + D.hshift[e][side];
                        if (expect != from) {
                            err = "internal: halo-side rule disagrees with the ghost gather map";
                            return BHAC_EINVAL;
                        }
                    }
                    std::vector<int32_t> &vd = nout == 1 ? P.gdst : edst;
                    std::vector<int32_t> &vs = nout == 1 ? P.gsrc : esrc;
                    vd.push_back((int32_t)to);
                    vs.push_back((int32_t)from);
                }
    }
    P.nface_slots = (long long)P.gdst.size();
    // flux correction of block trees: each face of a block whose far side lies in
    // finer leaves gets the mean of the fine faces covering it (second transverse
    // axis outer), applied between the face kernels and the update
    P.ffix.clear();
    if (p.amr) {
        for (int64_t b = 0; b < nb; b++) {
            const DevBlock &D = P.dblocks[b];
            for (int d = 0; d < p.ndim; d++) {
                const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
                const int fs0 = D.s[0] + (d == 0), fs1 = D.s[1] + (d == 1);
                for (int side = 0; side < 2; side++) {
                    if (!(D.hxl >> (2 * d + side) & 1)) continue;
                    for (int ib = 0; ib < D.s[tb]; ib++)
                        for (int ia = 0; ia < D.s[ta]; ia++) {
                            int l[3];
                            l[d] = side ? D.s[d] : -1;
                            l[ta] = ia;
                            l[tb] = ib;
                            long long Gi[3];
                            for (int e = 0; e < 3; e++) Gi[e] = wrap_axis(D.level, e, (long long)D.o[e] + l[e]);
                            const long long f[3] = {2 * Gi[0], 2 * Gi[1], p.ndim == 3 ? 2 * Gi[2] : 0};
                            const int fb = leaf_at(D.level + 1, f);
                            if (fb < 0) break;                // a coarser neighbour: nothing to correct
                            const DevBlock &F = P.dblocks[fb];
                            const int ffs0 = F.s[0] + (d == 0), ffs1 = F.s[1] + (d == 1);
                            int cl[3];
                            cl[d] = side ? D.s[d] : 0;
                            cl[ta] = ia;
                            cl[tb] = ib;
                            P.ffix.push_back(d);
                            P.ffix.push_back((int32_t)(D.fofs[d] + ((long long)cl[2] * fs1 + cl[1]) * fs0 + cl[0]));
                            for (int sb = 0; sb < 2; sb++)
                                for (int sa = 0; sa < 2; sa++) {
                                    if (p.ndim < 3 && sb > 0) { P.ffix.push_back(0); continue; }
                                    int fl[3];
                                    fl[d] = side ? (int)(f[d] - F.o[d]) : (int)(f[d] + 1 - F.o[d]) + 1;
                                    fl[ta] = (int)(f[ta] + sa - F.o[ta]);
                                    fl[tb] = tb < p.ndim ? (int)(f[tb] + sb - F.o[tb]) : 0;
                                    if (fl[d] != (side ? 0 : F.s[d]) || fl[ta] < 0 || fl[ta] >= F.s[ta] ||
                                        fl[tb] < 0 || fl[tb] >= F.s[tb]) {
                                        err = "internal: fine face of a flux correction outside its block";
                                        return BHAC_EINVAL;
                                    }
                                    P.ffix.push_back((int32_t)(F.fofs[d] + ((long long)fl[2] * ffs1 + fl[1]) * ffs0 + fl[0]));
                                }
                        }
                }
            }
        }
    }

    // prolongation groups after the restrictions of their class
    for (int cls = 0; cls < 2; cls++) {
        std::vector<int32_t> &xs = cls == 0 ? xface : xedge;
        std::vector<int32_t> &xo = cls == 0 ? xface_off : xedge_off;
        for (const PGroup &g : pgroups[cls]) {
            xo.push_back((int32_t)xs.size());
            xs.push_back(1);
            xs.push_back((int32_t)(g.kids.size() / 2));
            prolong_head(g.cb, g.lc, xs);
            xs.insert(xs.end(), g.kids.begin(), g.kids.end());
        }
    }
    // cross-level recipes: one stream, face recipes first, with offsets (n + 1)
    P.xdat = xface;
    P.xoff = xface_off;
    P.nxl_face = (long long)xface_off.size();
    for (int32_t o : xedge_off) P.xoff.push_back(o + (int32_t)xface.size());
    P.xdat.insert(P.xdat.end(), xedge.begin(), xedge.end());
    P.xoff.push_back((int32_t)P.xdat.size());
    P.gdst.insert(P.gdst.end(), edst.begin(), edst.end());
    P.gsrc.insert(P.gsrc.end(), esrc.begin(), esrc.end());
    (void)g;

    // metric tables
    P.nrec_c = P.nrec_f0 = P.nrec_f1 = 0;
    P.ctab.clear();
    P.f0tab.clear();
    P.f1tab.clear();
    P.ctab32.clear();
    P.f0tab32.clear();
    P.f1tab32.clear();
    if (tables && p.metric == BHAC_METRIC_KS_SPH_LOGR) {
        for (int l = 0; l <= P.maxlevel; l++) {
            DevLevel &L = P.levels[l];
            L.ctab = P.nrec_c;
            L.f0tab = P.nrec_f0;
            L.f1tab = P.nrec_f1;
            P.nrec_c += (long long)L.N0 * L.N1;
            P.nrec_f0 += (long long)(L.N0 + 1) * L.N1;
            P.nrec_f1 += (long long)L.N0 * (L.N1 + 1);
        }
        P.ctab.assign((size_t)P.nrec_c * C_NF, 0.0);
        P.f0tab.assign((size_t)P.nrec_f0 * C_FACE_NF, 0.0);
        P.f1tab.assign((size_t)P.nrec_f1 * C_FACE_NF, 0.0);
        double rec[C_NF];
        for (int l = 0; l <= P.maxlevel; l++) {
            const DevLevel &L = P.levels[l];
            for (int j = 0; j <= L.N1; j++)
                for (int i = 0; i <= L.N0; i++) {
                    const double xc1 = p.x_lo[0] + (i + 0.5) * L.dx[0], xc2 = p.x_lo[1] + (j + 0.5) * L.dx[1];
                    const double xf1 = p.x_lo[0] + i * L.dx[0], xf2 = p.x_lo[1] + j * L.dx[1];
                    if (i < L.N0 && j < L.N1) {
                        ks_record(p.spin, xc1, xc2, rec);
                        const long long r = L.ctab + (long long)j * L.N0 + i;
                        for (int f = 0; f < C_NF; f++) P.ctab[(size_t)f * P.nrec_c + r] = rec[f];
                    }
                    if (j < L.N1) {
                        ks_record(p.spin, xf1, xc2, rec);
                        const long long r = L.f0tab + (long long)j * (L.N0 + 1) + i;
                        for (int f = 0; f < C_FACE_NF; f++) P.f0tab[(size_t)f * P.nrec_f0 + r] = rec[f];
                    }
                    if (i < L.N0) {
                        ks_record(p.spin, xc1, xf2, rec);
                        const long long r = L.f1tab + (long long)j * L.N0 + i;
                        for (int f = 0; f < C_FACE_NF; f++) P.f1tab[(size_t)f * P.nrec_f1 + r] = rec[f];
                    }
                }
        }
    }
    if (!P.ctab.empty()) {
        P.ctab32.resize((size_t)P.nrec_c * C_FACE_NF);
        for (size_t q = 0; q < P.ctab32.size(); q++) P.ctab32[q] = (float)P.ctab[q];
        P.f0tab32.assign(P.f0tab.begin(), P.f0tab.end());
        P.f1tab32.assign(P.f1tab.begin(), P.f1tab.end());
    }
    return BHAC_OK;
}

}  // namespace bhac
