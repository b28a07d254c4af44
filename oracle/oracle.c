/*
 * oracle.c -- plain, slow, single-threaded FP64 CPU oracle for one Runge-Kutta
 * substep of the finite-volume GRMHD update on a list of blocks.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
 * this library: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no source, header, table or helper with the
 * HIP library; the two meet only in the data contract (structure-of-arrays
 * [9][padded cells], blocks stored one after another, x fastest).
 *
 * What it computes. The paper (Section 2, "Code overview") names the method's
 * ingredients: GRMHD in a covariant coordinate system, a high-resolution
 * shock-capturing finite-volume scheme, second-order time stepping, second- or
 * third-order (PPM) reconstruction, and a Newton-Raphson conserved-to-primitive
 * inversion with backups, on blocks of cells with ghost layers (Section 4.3 names
 * the same-level ghost fill, Section 5.1 the ghost-cell exchange). It prints no
 * equation, so every formula below is the standard 3+1 ("Valencia") form of
 * ideal GRMHD that the code family uses; each function says which reading it
 * implements. Build: gcc -O2 -ffp-contract=off, no fast-math.
 *
 * Parity pins: every function here is checked in tests/ against something other
 * than itself (closed forms, invariants, brute force, covariant re-derivations).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define NV 9
#define NVE 10                         /* with the entropy field */

/* Op-count regions. The plain build leaves OC_SCOPE empty. The op-count build
 * (opcount.cpp) compiles this file with a counting arithmetic type and defines
 * OC_SCOPE to attribute the arithmetic of the enclosing block to a region, so that
 * the algorithmic operations per zone and substep can be read per part of the
 * method. */
#ifndef OC_SCOPE
#define OC_SCOPE(region)
#endif
enum { IRHO = 0, IU1 = 1, IP = 4, IB1 = 5, IPSI = 8, IENT = 9 };
enum { ID = 0, IS1 = 1, ITAU = 4 };

/* ---------------------------------------------------------------------------------
 * Parameters (the oracle's own definition; same meaning as the library's struct).
 * ------------------------------------------------------------------------------- */
typedef struct {
    int ndim, nghost, metric;          /* metric: 0 Minkowski Cartesian, 1 Kerr-Schild (ln r, theta, phi) */
    double spin, gamma_ad;
    double x_lo[3], x_hi[3];
    int ncell0[3];
    int bc[3][2];                      /* 0 periodic, 1 outflow */
    int recon, flux;                   /* recon: 0 MC, 1 PPM; flux: 0 HLL, 1 TVDLF */
    double cfl, rho_floor, p_floor, w_max, glm_alpha, c2p_tol;
    int c2p_maxit;
    int amr;                           /* 0 independent same-level patches, 1 2:1 block tree */
    int entropy;                       /* 1: carry the entropy field (P[9] = K, U[9] = U[0] K) */
    int c2p_2d;                        /* 1: a failed inversion tries the two-unknown Newton backup */
    int ct;                            /* 1: staggered constrained transport instead of GLM cleaning */
} orc_params;

/* rows of P and U: the nine GRMHD variables, plus the entropy field if carried */
static int nvar(const orc_params *p) { return p->entropy ? NVE : NV; }

typedef struct { int level, size[3], origin[3]; } orc_block;

typedef struct {
    double dt_next, dt, ch, kappa;
    double lam[3];
    double dt_fixed;                   /* > 0: every step uses this dt */
    int have_dt;
    int64_t c2p_fail, floor_hits;
    int max_iter;
    int64_t c2p_backup;                /* cells whose inversion came from the entropy backup */
} orc_state;

/* Inversion counters of one block (merged into orc_state after the block). */
typedef struct { int64_t fail, floors, backup; int max_iter; } ocount;

static void ocount_merge(orc_state *st, const ocount *c)
{
    st->c2p_fail += c->fail;
    st->floor_hits += c->floors;
    st->c2p_backup += c->backup;
    if (c->max_iter > st->max_iter) st->max_iter = c->max_iter;
}

/* Threads of the block loops (default 1: the oracle runs single-threaded unless a
 * caller asks for more). Blocks are independent within every call, each block's
 * arithmetic is the same whichever thread runs it, and the only cross-block
 * results are exact (integer counts and maxima), so any thread count gives
 * bit-identical results. */
static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return g_threads; }

/* ---------------------------------------------------------------------------------
 * Spacetime metric (reading: stationary Kerr-Schild in spherical coordinates with
 * x1 = ln r, x2 = theta, x3 = phi, M = 1; or flat Cartesian). Section 2 allows any
 * covariant coordinate system; the metric is analytic and evaluated pointwise.
 * ------------------------------------------------------------------------------- */
typedef struct {
    double alpha, beta[3], g[3][3], gi[3][3], sqrtg;
    double da[3];          /* d_j alpha */
    double db[3][3];       /* db[j][i] = d_j beta^i */
    double dg[3][3][3];    /* dg[j][i][k] = d_j gamma_ik */
} ometric;

static void metric_at(const orc_params *p, double x1, double x2, ometric *m)
{
    OC_SCOPE(OC_METRIC);
    memset(m, 0, sizeof *m);
    if (p->metric == 0) {
        m->alpha = 1.0;
        m->sqrtg = 1.0;
        for (int i = 0; i < 3; i++) { m->g[i][i] = 1.0; m->gi[i][i] = 1.0; }
        return;
    }
    const double a = p->spin;
    const double r = exp(x1), st = sin(x2), ct = cos(x2);
    const double sig = r * r + a * a * ct * ct;
    const double z = 2.0 * r / sig;
    const double opz = 1.0 + z;

    m->alpha = 1.0 / sqrt(opz);
    m->beta[0] = z / (r * opz);
    m->g[0][0] = r * r * opz;
    m->g[0][2] = m->g[2][0] = -a * r * st * st * opz;
    m->g[1][1] = sig;
    m->g[2][2] = st * st * (sig + a * a * st * st * opz);
    m->sqrtg = r * sig * st * sqrt(opz);
    const double det13 = m->g[0][0] * m->g[2][2] - m->g[0][2] * m->g[0][2];
    m->gi[0][0] = m->g[2][2] / det13;
    m->gi[2][2] = m->g[0][0] / det13;
    m->gi[0][2] = m->gi[2][0] = -m->g[0][2] / det13;
    m->gi[1][1] = 1.0 / sig;

    /* derivatives with respect to r and theta, then d/dx1 = r d/dr */
    const double dsig_r = 2.0 * r, dsig_t = -2.0 * a * a * st * ct;
    const double dz_r = 2.0 / sig - 2.0 * r * dsig_r / (sig * sig);
    const double dz_t = -2.0 * r * dsig_t / (sig * sig);
    const double dz[2] = { dz_r, dz_t };
    double dal[2], db1[2], dg11[2], dg13[2], dg22[2], dg33[2];
    for (int q = 0; q < 2; q++) dal[q] = -0.5 * pow(opz, -1.5) * dz[q];
    db1[0] = (r * dz_r - z * opz) / (r * r * opz * opz);
    db1[1] = dz_t / (r * opz * opz);
    dg11[0] = 2.0 * r * opz + r * r * dz_r;
    dg11[1] = r * r * dz_t;
    dg13[0] = -a * st * st * opz - a * r * st * st * dz_r;
    dg13[1] = -a * r * (2.0 * st * ct * opz + st * st * dz_t);
    dg22[0] = dsig_r;
    dg22[1] = dsig_t;
    dg33[0] = st * st * dsig_r + a * a * st * st * st * st * dz_r;
    dg33[1] = 2.0 * st * ct * sig + st * st * dsig_t
              + a * a * (4.0 * st * st * st * ct * opz + st * st * st * st * dz_t);
    const double fac[2] = { r, 1.0 };          /* chain rule for x1 = ln r */
    for (int j = 0; j < 2; j++) {
        m->da[j] = fac[j] * dal[j];
        m->db[j][0] = fac[j] * db1[j];
        m->dg[j][0][0] = fac[j] * dg11[j];
        m->dg[j][0][2] = m->dg[j][2][0] = fac[j] * dg13[j];
        m->dg[j][1][1] = fac[j] * dg22[j];
        m->dg[j][2][2] = fac[j] * dg33[j];
    }
}

/* ---------------------------------------------------------------------------------
 * Primitive -> conserved (reading: Valencia 3+1 variables with an ideal-gas EOS).
 * P = (rho, u~^i = W v^i, p, B^i, psi); U = sqrt(gamma) (D, S_i, tau, B^i), psi.
 * ------------------------------------------------------------------------------- */
typedef struct {
    double rho, p, W, v[3], vl[3], B[3], Bl[3], B2, Bv, v2, h, xi, D, S[3], tau;
} ostate;

static void state_from_prim(const orc_params *p, const ometric *m, const double *P, ostate *s)
{
    const double gam = p->gamma_ad;
    s->rho = P[IRHO];
    s->p = P[IP];
    double ul[3], u2 = 0.0;
    for (int i = 0; i < 3; i++) {
        ul[i] = 0.0;
        for (int j = 0; j < 3; j++) ul[i] += m->g[i][j] * P[IU1 + j];
    }
    for (int i = 0; i < 3; i++) u2 += P[IU1 + i] * ul[i];
    s->W = sqrt(1.0 + u2);
    for (int i = 0; i < 3; i++) { s->v[i] = P[IU1 + i] / s->W; s->vl[i] = ul[i] / s->W; }
    s->v2 = 0.0;
    for (int i = 0; i < 3; i++) s->v2 += s->v[i] * s->vl[i];
    for (int i = 0; i < 3; i++) s->B[i] = P[IB1 + i];
    for (int i = 0; i < 3; i++) {
        s->Bl[i] = 0.0;
        for (int j = 0; j < 3; j++) s->Bl[i] += m->g[i][j] * s->B[j];
    }
    s->B2 = 0.0;
    s->Bv = 0.0;
    for (int i = 0; i < 3; i++) { s->B2 += s->B[i] * s->Bl[i]; s->Bv += s->B[i] * s->vl[i]; }
    s->h = 1.0 + gam / (gam - 1.0) * s->p / s->rho;
    s->xi = s->rho * s->h * s->W * s->W;
    s->D = s->rho * s->W;
    for (int i = 0; i < 3; i++) s->S[i] = (s->xi + s->B2) * s->vl[i] - s->Bv * s->Bl[i];
    s->tau = s->xi + s->B2 - s->p - 0.5 * (s->Bv * s->Bv + s->B2 / (s->W * s->W)) - s->D;
}

static void p2c_point(const orc_params *p, const ometric *m, const double *P, double *U)
{
    OC_SCOPE(OC_P2C);
    ostate s;
    state_from_prim(p, m, P, &s);
    U[ID] = m->sqrtg * s.D;
    for (int i = 0; i < 3; i++) U[IS1 + i] = m->sqrtg * s.S[i];
    U[ITAU] = m->sqrtg * s.tau;
    for (int i = 0; i < 3; i++) U[IB1 + i] = m->sqrtg * s.B[i];
    U[IPSI] = P[IPSI];
    if (p->entropy) U[IENT] = U[ID] * P[IENT];
}

/* ---------------------------------------------------------------------------------
 * Physical flux along direction d and the fast-speed bounds (reading: 3+1 fluxes;
 * isotropic fast-magnetosonic bound c_e^2 = c_s^2 + c_a^2 - c_s^2 c_a^2).
 * The normal-field flux and the psi flux are left zero: the GLM solve sets them.
 * ------------------------------------------------------------------------------- */
static void phys_flux(const orc_params *p, const ometric *m, const double *P, int d,
                      double *U, double *F, double *lminus, double *lplus)
{
    OC_SCOPE(OC_FACE_STATE);
    const double gam = p->gamma_ad;
    ostate s;
    state_from_prim(p, m, P, &s);
    const double W2 = s.W * s.W;
    const double b2 = s.B2 / W2 + s.Bv * s.Bv;
    const double pt = s.p + 0.5 * b2;
    double Sd = 0.0;
    for (int k = 0; k < 3; k++) Sd += m->gi[d][k] * s.S[k];
    const double sg = m->sqrtg, al = m->alpha;
    const double vd = s.v[d], bd = m->beta[d];

    U[ID] = sg * s.D;
    for (int i = 0; i < 3; i++) U[IS1 + i] = sg * s.S[i];
    U[ITAU] = sg * s.tau;
    for (int i = 0; i < 3; i++) U[IB1 + i] = sg * s.B[i];
    U[IPSI] = P[IPSI];

    F[ID] = sg * s.D * (al * vd - bd);
    for (int j = 0; j < 3; j++) {
        double Wdj = Sd * s.vl[j] + (j == d ? pt : 0.0) - (s.B[d] / W2 + s.Bv * vd) * s.Bl[j];
        F[IS1 + j] = sg * (al * Wdj - bd * s.S[j]);
    }
    F[ITAU] = sg * (al * (Sd - s.D * vd) - bd * s.tau);
    for (int j = 0; j < 3; j++) {
        if (j == d) { F[IB1 + j] = 0.0; continue; }
        F[IB1 + j] = sg * ((al * vd - bd) * s.B[j] - (al * s.v[j] - m->beta[j]) * s.B[d]);
    }
    F[IPSI] = 0.0;

    const double rhoh = s.rho * s.h;
    const double cs2 = gam * s.p / rhoh;
    const double ca2 = b2 / (rhoh + b2);
    const double ce2 = cs2 + ca2 - cs2 * ca2;
    const double v2 = s.v2;
    double disc = ce2 * (1.0 - v2) * (m->gi[d][d] * (1.0 - v2 * ce2) - vd * vd * (1.0 - ce2));
    if (disc < 0.0) disc = 0.0;
    const double sq = sqrt(disc);
    const double pre = al / (1.0 - v2 * ce2);
    *lplus = pre * (vd * (1.0 - ce2) + sq) - bd;
    *lminus = pre * (vd * (1.0 - ce2) - sq) - bd;
}

/* ---------------------------------------------------------------------------------
 * Face flux: exact solve of the (B~^d, psi) GLM subsystem, then HLL or TVDLF on
 * the other variables (reading: Dedner mixed GLM in coordinate space).
 * ------------------------------------------------------------------------------- */
/* HLL or TVDLF combination of the two face states' fluxes for every variable except
 * the normal field and psi (their fluxes come from the GLM solve, or vanish under
 * constrained transport); returns the largest |lambda| of both states. */
static double hll_combine(const orc_params *p, int d, const double *UL, const double *UR, const double *FL,
                          const double *FR, double lml, double lpl, double lmr, double lpr, double *F)
{
    for (int v = 0; v < NV; v++) {
        if (v == IB1 + d || v == IPSI) continue;
        if (p->flux == 0) {
            double sr = 0.0, sl = 0.0;
            if (lpl > sr) sr = lpl;
            if (lpr > sr) sr = lpr;
            if (lml < sl) sl = lml;
            if (lmr < sl) sl = lmr;
            if (sr == sl) F[v] = 0.5 * (FL[v] + FR[v]);
            else F[v] = (sr * FL[v] - sl * FR[v] + sr * sl * (UR[v] - UL[v])) / (sr - sl);
        } else {
            double c = fabs(lml);
            if (fabs(lpl) > c) c = fabs(lpl);
            if (fabs(lmr) > c) c = fabs(lmr);
            if (fabs(lpr) > c) c = fabs(lpr);
            F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * c * (UR[v] - UL[v]);
        }
    }
    double lam = fabs(lml);
    if (fabs(lpl) > lam) lam = fabs(lpl);
    if (fabs(lmr) > lam) lam = fabs(lmr);
    if (fabs(lpr) > lam) lam = fabs(lpr);
    return lam;
}

static double riemann(const orc_params *p, const ometric *mf, int d, const double *PL,
                      const double *PR, double ch, double *F)
{
    OC_SCOPE(OC_RIEMANN);
    const double sg = mf->sqrtg;
    const double btl = sg * PL[IB1 + d], btr = sg * PR[IB1 + d];
    const double psl = PL[IPSI], psr = PR[IPSI];
    const double bstar = 0.5 * (btl + btr) - (psr - psl) / (2.0 * ch);
    const double psistar = 0.5 * (psl + psr) - 0.5 * ch * (btr - btl);
    double ql[NV], qr[NV];
    memcpy(ql, PL, sizeof ql);
    memcpy(qr, PR, sizeof qr);
    ql[IB1 + d] = bstar / sg;
    qr[IB1 + d] = bstar / sg;
    double UL[NV], UR[NV], FL[NV], FR[NV], lml, lpl, lmr, lpr;
    phys_flux(p, mf, ql, d, UL, FL, &lml, &lpl);
    phys_flux(p, mf, qr, d, UR, FR, &lmr, &lpr);
    const double lam = hll_combine(p, d, UL, UR, FL, FR, lml, lpl, lmr, lpr, F);
    F[IB1 + d] = psistar;
    F[IPSI] = ch * ch * bstar;
    return lam;
}

/* Face flux under constrained transport (reading): the normal field of the face is
 * the staggered face field phi = sqrt(gamma) B^d there, the same for both states;
 * no GLM solve: the normal-field and psi fluxes vanish (the face field is advanced by
 * the edge electric fields instead). */
static double riemann_ct(const orc_params *p, const ometric *mf, int d, const double *PL, const double *PR,
                         double phi, double *F)
{
    OC_SCOPE(OC_RIEMANN);
    double ql[NV], qr[NV];
    memcpy(ql, PL, sizeof ql);
    memcpy(qr, PR, sizeof qr);
    ql[IB1 + d] = phi / mf->sqrtg;
    qr[IB1 + d] = phi / mf->sqrtg;
    double UL[NV], UR[NV], FL[NV], FR[NV], lml, lpl, lmr, lpr;
    phys_flux(p, mf, ql, d, UL, FL, &lml, &lpl);
    phys_flux(p, mf, qr, d, UR, FR, &lmr, &lpr);
    const double lam = hll_combine(p, d, UL, UR, FL, FR, lml, lpl, lmr, lpr, F);
    F[IB1 + d] = 0.0;
    F[IPSI] = 0.0;
    return lam;
}

/* ---------------------------------------------------------------------------------
 * Reconstruction (Section 2: second order, or third order PPM).
 * MC: monotonised-central limited slope. PPM: Colella-Woodward interface values
 * from MC slopes, then the two monotonicity constraints, no flattening.
 * ------------------------------------------------------------------------------- */
static double mc_slope(double qm, double q0, double qp)
{
    OC_SCOPE(OC_SLOPE);
    const double dm = q0 - qm, dp = qp - q0;
    if (dm * dp <= 0.0) return 0.0;
    double s = 2.0 * fabs(dm);
    if (2.0 * fabs(dp) < s) s = 2.0 * fabs(dp);
    if (0.5 * fabs(dm + dp) < s) s = 0.5 * fabs(dm + dp);
    return dp > 0.0 ? s : -s;
}

/* q[0..4] = cells c-2..c+2; returns the values at the cell's lower and upper faces */
static void ppm_cell(const double *q, double *qminus, double *qplus)
{
    const double sm = mc_slope(q[0], q[1], q[2]);
    const double s0 = mc_slope(q[1], q[2], q[3]);
    const double sp = mc_slope(q[2], q[3], q[4]);
    double ql, qr;
    {
        OC_SCOPE(OC_PPM_IFACE);
        ql = 0.5 * (q[1] + q[2]) - (s0 - sm) / 6.0;
        qr = 0.5 * (q[2] + q[3]) - (sp - s0) / 6.0;
    }
    OC_SCOPE(OC_PPM_LIMIT);
    const double qi = q[2];
    if ((qr - qi) * (qi - ql) <= 0.0) {
        ql = qi;
        qr = qi;
    } else if ((qr - ql) * (qi - 0.5 * (ql + qr)) > (qr - ql) * (qr - ql) / 6.0) {
        ql = 3.0 * qi - 2.0 * qr;
    } else if (-(qr - ql) * (qr - ql) / 6.0 > (qr - ql) * (qi - 0.5 * (ql + qr))) {
        qr = 3.0 * qi - 2.0 * ql;
    }
    *qminus = ql;
    *qplus = qr;
}

/* q[0..5] = cells i-3..i+2 around face i-1/2; left and right face states */
static void recon_face(int method, const double *q, double *qL, double *qR)
{
    if (method == 0) {
        const double sl = mc_slope(q[1], q[2], q[3]), sr = mc_slope(q[2], q[3], q[4]);
        OC_SCOPE(OC_MC_FACE);
        *qL = q[2] + 0.5 * sl;
        *qR = q[3] - 0.5 * sr;
    } else {
        double a, b;
        ppm_cell(q + 0, &a, qL);      /* cell i-1 uses i-3..i+1 */
        ppm_cell(q + 1, qR, &b);      /* cell i uses i-2..i+2 */
    }
}

/* ---------------------------------------------------------------------------------
 * Geometric sources (reading: stationary metric, extrinsic curvature eliminated,
 * written with metric derivatives; equal to the Christoffel-symbol form).
 * Conserved D, S_j, tau from U_stage; the rest from P_stage. GLM damping on psi.
 * ------------------------------------------------------------------------------- */
static void sources_point(const orc_params *p, const ometric *m, const double *P, const double *U,
                          double kappa, double *S)
{
    OC_SCOPE(OC_SOURCES);
    ostate s;
    state_from_prim(p, m, P, &s);
    const double sg = m->sqrtg;
    const double D = U[ID] / sg, tau = U[ITAU] / sg;
    double Sl[3], Su[3];
    for (int i = 0; i < 3; i++) Sl[i] = U[IS1 + i] / sg;
    for (int i = 0; i < 3; i++) {
        Su[i] = 0.0;
        for (int k = 0; k < 3; k++) Su[i] += m->gi[i][k] * Sl[k];
    }
    const double W2 = s.W * s.W;
    const double b2 = s.B2 / W2 + s.Bv * s.Bv;
    const double pt = s.p + 0.5 * b2;
    double Wuu[3][3], Wud[3][3];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++)
            Wuu[i][k] = Su[i] * s.v[k] + pt * m->gi[i][k] - (s.B[i] / W2 + s.Bv * s.v[i]) * s.B[k];
    for (int j = 0; j < 3; j++)
        for (int i = 0; i < 3; i++) {
            Wud[j][i] = 0.0;
            for (int k = 0; k < 3; k++) Wud[j][i] += Wuu[j][k] * m->g[k][i];
        }
    for (int v = 0; v < NV; v++) S[v] = 0.0;
    for (int j = 0; j < 3; j++) {
        double t = 0.0;
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) t += 0.5 * m->alpha * Wuu[i][k] * m->dg[j][i][k];
        for (int i = 0; i < 3; i++) t += Sl[i] * m->db[j][i];
        t -= (tau + D) * m->da[j];
        S[IS1 + j] = sg * t;
    }
    double te = 0.0;
    for (int j = 0; j < 3; j++) {
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) te += 0.5 * Wuu[i][k] * m->beta[j] * m->dg[j][i][k];
        for (int i = 0; i < 3; i++) te += Wud[j][i] * m->db[j][i];
        te -= Su[j] * m->da[j];
    }
    S[ITAU] = sg * te;
    S[IPSI] = -kappa * U[IPSI];
}

/* ---------------------------------------------------------------------------------
 * Conserved -> primitive (Section 2: Newton-Raphson with a backup). Reading: 1-D
 * Newton on xi = rho h W^2, safeguarded by bisection towards the previous iterate,
 * stop at |dxi| <= tol xi plus one more step; floors after success; on failure the
 * cell keeps its stage primitives (the backup) and is flagged.
 * Returns 0 on success, 1 on failure. *nit = Newton steps taken.
 * ------------------------------------------------------------------------------- */
typedef struct { double D, Ut, S2, B2, SB, gam; } c2p_sys;

static double c2p_v2(const c2p_sys *c, double xi)
{
    const double xb = xi + c->B2;
    return (xi * xi * c->S2 + c->SB * c->SB * (c->B2 + 2.0 * xi)) / (xi * xi * xb * xb);
}

static void c2p_fdf(const c2p_sys *c, double xi, double *f, double *df)
{
    const double v2 = c2p_v2(c, xi);
    const double w2inv = 1.0 - v2;
    const double W = 1.0 / sqrt(w2inv);
    const double rho = c->D / W;
    const double gfac = (c->gam - 1.0) / c->gam;
    const double p = gfac * (xi * w2inv - rho);
    *f = xi - p + c->B2 - 0.5 * (c->B2 * w2inv + c->SB * c->SB / (xi * xi)) - c->Ut;
    const double xb = xi + c->B2;
    const double dv2 = -2.0 * c->S2 / (xb * xb * xb)
                       - 2.0 * c->SB * c->SB * (3.0 * xi * xi + 3.0 * xi * c->B2 + c->B2 * c->B2)
                             / (xi * xi * xi * xb * xb * xb);
    const double dp = gfac * (w2inv + (0.5 * c->D * W - xi) * dv2);
    *df = 1.0 - dp + 0.5 * c->B2 * dv2 + c->SB * c->SB / (xi * xi * xi);
}

static double c2p_step(const c2p_sys *c, double xi)
{
    double f, df;
    c2p_fdf(c, xi, &f, &df);
    double xn = xi - f / df;
    int nh = 0;
    while ((xn <= 0.0 || c2p_v2(c, xn) >= 1.0) && nh < 64) {
        xn = 0.5 * (xn + xi);
        nh++;
    }
    if (xn <= 0.0 || c2p_v2(c, xn) >= 1.0) return NAN;
    return xn;
}

/* ---------------------------------------------------------------------------------
 * Two-unknown Newton backup (Section 2 lists multi-dimensional Newton solvers among
 * the inversion's strategies). Reading: unknowns xi = rho h W^2 and q = W^2 - 1 (so
 * v^2 = q / (1 + q) and the iteration never meets the wall v^2 = 1), with the
 * momentum relation (the v^2(xi) identity multiplied out)
 *   F1 = (xi + B^2)^2 q / (1 + q) - (S.B)^2 (2 xi + B^2) / xi^2 - S^2 = 0
 * and the energy relation
 *   F2 = xi - p + B^2 - (B^2 / (1 + q) + (S.B)^2 / xi^2) / 2 - (tau + D) = 0,
 *   p = (Gamma - 1) / Gamma (xi / (1 + q) - D / sqrt(1 + q)),
 * solved together: Newton steps with the analytic Jacobian, each step halved while
 * it would leave xi > 0, q >= 0; stop when |dxi| <= tol xi and |dq| <= tol (1 + q),
 * then one more step; at most maxit steps.
 * ------------------------------------------------------------------------------- */
static void c2p2_fj(const c2p_sys *c, double xi, double q, double F[2], double J[2][2])
{
    const double gi = (c->gam - 1.0) / c->gam;
    const double sb2 = c->SB * c->SB, xb = xi + c->B2, w2inv = 1.0 / (1.0 + q), iw = sqrt(w2inv);
    const double p = gi * (xi * w2inv - c->D * iw);
    F[0] = xb * xb * q * w2inv - sb2 * (2.0 * xi + c->B2) / (xi * xi) - c->S2;
    F[1] = xi - p + c->B2 - 0.5 * (c->B2 * w2inv + sb2 / (xi * xi)) - c->Ut;
    const double dw2inv = -w2inv * w2inv;                 /* d(1/(1+q))/dq */
    const double dp_dxi = gi * w2inv;
    const double dp_dq = gi * (xi * dw2inv + 0.5 * c->D * iw * w2inv);
    J[0][0] = 2.0 * xb * q * w2inv + 2.0 * sb2 * xb / (xi * xi * xi);
    J[0][1] = xb * xb * w2inv * w2inv;
    J[1][0] = 1.0 - dp_dxi + sb2 / (xi * xi * xi);
    J[1][1] = -dp_dq - 0.5 * c->B2 * dw2inv;
}

/* one safeguarded Newton step of the pair; returns 1 where it cannot be taken */
static int c2p2_step(const c2p_sys *c, double *xi, double *q, double tol, int *small)
{
    double F[2], J[2][2];
    c2p2_fj(c, *xi, *q, F, J);
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (!isfinite(det) || det == 0.0 || !isfinite(F[0]) || !isfinite(F[1])) return 1;
    double dxi = -(J[1][1] * F[0] - J[0][1] * F[1]) / det;
    double dq = -(J[0][0] * F[1] - J[1][0] * F[0]) / det;
    int nh = 0;
    while ((*xi + dxi <= 0.0 || *q + dq < 0.0) && nh < 64) {
        dxi *= 0.5;
        dq *= 0.5;
        nh++;
    }
    if (*xi + dxi <= 0.0 || *q + dq < 0.0) return 1;
    *xi += dxi;
    *q += dq;
    *small = fabs(dxi) <= tol * *xi && fabs(dq) <= tol * (1.0 + *q);
    return 0;
}

/* from (xi, q) to a root (xi, q); returns 0 on convergence */
static int c2p_newton2(const c2p_sys *c, double xi, double q, double tol, int maxit, double *xi_out, double *q_out,
                       int *nit)
{
    int it = 0, conv = 0, small = 0;
    while (it < maxit) {
        if (c2p2_step(c, &xi, &q, tol, &small)) { *nit = it; return 1; }
        it++;
        if (small) { conv = 1; break; }
    }
    if (conv) {
        if (c2p2_step(c, &xi, &q, tol, &small)) conv = 0;     /* one more step after the stopping test */
        it++;
    }
    *nit = it;
    *xi_out = xi;
    *q_out = q;
    return conv && isfinite(xi) && isfinite(q) ? 0 : 1;
}

/* ---------------------------------------------------------------------------------
 * Entropy backup of the inversion (Section 2 names backups; reading 19). The
 * entropy function K = p / rho^gamma is carried as its own field, so where the
 * energy relation cannot be inverted the pressure is p = K rho^gamma instead, and
 * with rho = D / W the enthalpy density xi = rho h W^2 becomes a function of W
 * alone:  xi(W) = D W + gamma/(gamma-1) K D^gamma W^(2-gamma).  What is left is
 * the momentum relation
 *     f(W) = (xi + B^2)^2 (1 - 1/W^2) - (S.B)^2 (2 xi + B^2) / xi^2 - S^2 = 0.
 * For gamma <= 2 every term of f grows with W and f(1) <= 0, so f has one root
 * in [1, inf). It is found by Newton steps in W kept inside a bracket [lo, hi]
 * (a step leaving the bracket is replaced by its midpoint; every evaluation
 * moves one end), stopping at |dW| <= tol W.
 * ------------------------------------------------------------------------------- */
#define ENT_MAXIT 100

static void ent_fdf(const c2p_sys *c, double K, double W, double *xi, double *f, double *df)
{
    const double g = c->gam, a = g / (g - 1.0);
    const double KDg = a * K * pow(c->D, g);
    *xi = c->D * W + KDg * pow(W, 2.0 - g);
    const double dxi = c->D + KDg * (2.0 - g) * pow(W, 1.0 - g);
    const double x = *xi, xb = x + c->B2, w2i = 1.0 / (W * W), sb2 = c->SB * c->SB;
    *f = xb * xb * (1.0 - w2i) - sb2 * (2.0 * x + c->B2) / (x * x) - c->S2;
    *df = 2.0 * xb * dxi * (1.0 - w2i) + 2.0 * xb * xb * w2i / W + sb2 * dxi * (2.0 / (x * x) + 2.0 * c->B2 / (x * x * x));
}

/* Returns 0 with the root W and xi(W), or 1 if no root was found. Wg: start value. */
static int c2p_entropy(const c2p_sys *c, double K, double Wg, double tol, double *Wout, double *xiout)
{
    double xi, f, df;
    double lo = 1.0, hi = 2.0;
    ent_fdf(c, K, hi, &xi, &f, &df);
    int nd = 0;
    while (f < 0.0 && nd < 60) {
        lo = hi;
        hi *= 2.0;
        ent_fdf(c, K, hi, &xi, &f, &df);
        nd++;
    }
    if (!(f >= 0.0)) return 1;
    double W = (Wg > lo && Wg < hi) ? Wg : 0.5 * (lo + hi);
    for (int it = 0; it < ENT_MAXIT; it++) {
        ent_fdf(c, K, W, &xi, &f, &df);
        if (!isfinite(f) || !isfinite(df)) return 1;
        if (f == 0.0) { *Wout = W; *xiout = xi; return 0; }
        if (f < 0.0) lo = W; else hi = W;
        double Wn = W - f / df;
        if (!(Wn > lo && Wn < hi)) Wn = 0.5 * (lo + hi);
        const int done = fabs(Wn - W) <= tol * Wn;
        W = Wn;
        if (done) {
            ent_fdf(c, K, W, &xi, &f, &df);
            *Wout = W;
            *xiout = xi;
            return 0;
        }
    }
    return 1;
}

static int c2p_point(const orc_params *p, const ometric *m, const double *U, const double *Pg,
                     double *Pout, int *nit, int *floored, int *backup)
{
    OC_SCOPE(OC_C2P);
    const double sg = m->sqrtg;
    *nit = 0;
    *floored = 0;
    *backup = 0;
    c2p_sys c;
    c.gam = p->gamma_ad;
    c.D = U[ID] / sg;
    const double tau = U[ITAU] / sg;
    double Sl[3], B[3], Bl[3];
    for (int i = 0; i < 3; i++) { Sl[i] = U[IS1 + i] / sg; B[i] = U[IB1 + i] / sg; }
    c.Ut = tau + c.D;
    c.S2 = 0.0;
    c.B2 = 0.0;
    c.SB = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) c.S2 += m->gi[i][j] * Sl[i] * Sl[j];
    for (int i = 0; i < 3; i++) {
        Bl[i] = 0.0;
        for (int j = 0; j < 3; j++) Bl[i] += m->g[i][j] * B[j];
    }
    for (int i = 0; i < 3; i++) { c.B2 += B[i] * Bl[i]; c.SB += Sl[i] * B[i]; }

    int fail = 0;
    double xi = 0.0;
    if (!(c.D > 0.0) || !isfinite(c.Ut) || !isfinite(c.S2) || !isfinite(c.B2)) fail = 1;
    if (!fail) {
        ostate g;
        state_from_prim(p, m, Pg, &g);
        xi = g.xi;
        if (!(xi > 0.0) || !isfinite(xi)) xi = c.Ut > c.D ? c.Ut : c.D;
        int nrep = 0;
        while (c2p_v2(&c, xi) >= 1.0 && nrep < 200) { xi *= 2.0; nrep++; }
        if (!(c2p_v2(&c, xi) < 1.0)) fail = 1;
    }
    if (!fail) {
        int conv = 0, it = 0;
        while (it < p->c2p_maxit) {
            const double xn = c2p_step(&c, xi);
            it++;
            if (!isfinite(xn)) { fail = 1; break; }
            const int done = fabs(xn - xi) <= p->c2p_tol * xn;
            xi = xn;
            if (done) { conv = 1; break; }
        }
        if (!fail && !conv) fail = 1;
        if (!fail) {
            xi = c2p_step(&c, xi);      /* one more step after the stopping test */
            it++;
            if (!isfinite(xi)) fail = 1;
        }
        *nit = it;
    }
    double rho = 0.0, prs = 0.0, W = 1.0, ut[3] = { 0.0, 0.0, 0.0 };
    if (!fail) {
        const double v2 = c2p_v2(&c, xi);
        if (!(v2 < 1.0)) fail = 1;
        else {
            W = 1.0 / sqrt(1.0 - v2);
            rho = c.D / W;
            prs = (c.gam - 1.0) / c.gam * (xi / (W * W) - rho);
            if (!(rho > 0.0) || !(prs >= 0.0) || !isfinite(rho) || !isfinite(prs)) fail = 1;
        }
    }
    if (fail && p->c2p_2d && c.D > 0.0 && isfinite(c.Ut) && isfinite(c.S2) && isfinite(c.B2)) {
        ostate g;
        state_from_prim(p, m, Pg, &g);
        const double xi0 = g.xi > 0.0 && isfinite(g.xi) ? g.xi : (c.Ut > c.D ? c.Ut : c.D);
        const double q0 = isfinite(g.W) ? g.W * g.W - 1.0 : 0.0;
        double xb, qb;
        int n2;
        if (c2p_newton2(&c, xi0, q0 > 0.0 ? q0 : 0.0, p->c2p_tol, p->c2p_maxit, &xb, &qb, &n2) == 0) {
            const double Wb = sqrt(1.0 + qb), rb = c.D / Wb;
            const double pb = (c.gam - 1.0) / c.gam * (xb / (Wb * Wb) - rb);
            if (rb > 0.0 && pb >= 0.0 && isfinite(rb) && isfinite(pb)) {
                W = Wb;
                xi = xb;
                rho = rb;
                prs = pb;
                fail = 0;
                *backup = 1;
            }
        }
    }
    if (fail && p->entropy) {
        const double K = U[IENT] / U[ID];
        if (c.D > 0.0 && K > 0.0 && isfinite(K) && isfinite(c.S2) && isfinite(c.B2)) {
            ostate g;
            state_from_prim(p, m, Pg, &g);
            double Wb, xib;
            if (c2p_entropy(&c, K, g.W, p->c2p_tol, &Wb, &xib) == 0) {
                const double rb = c.D / Wb, pb = K * pow(rb, c.gam);
                if (rb > 0.0 && pb >= 0.0 && isfinite(rb) && isfinite(pb) && xib > 0.0) {
                    W = Wb;
                    xi = xib;
                    rho = rb;
                    prs = pb;
                    fail = 0;
                    *backup = 1;
                }
            }
        }
    }
    if (fail) {
        memcpy(Pout, Pg, nvar(p) * sizeof(double));
        return 1;
    }
    double vl[3];
    for (int i = 0; i < 3; i++) vl[i] = (Sl[i] + c.SB * Bl[i] / xi) / (xi + c.B2);
    for (int i = 0; i < 3; i++) {
        double vu = 0.0;
        for (int j = 0; j < 3; j++) vu += m->gi[i][j] * vl[j];
        ut[i] = W * vu;
    }
    if (rho < p->rho_floor) { rho = p->rho_floor; *floored = 1; }
    if (prs < p->p_floor) { prs = p->p_floor; *floored = 1; }
    if (W > p->w_max) {
        const double f = sqrt(p->w_max * p->w_max - 1.0) / sqrt(W * W - 1.0);
        for (int i = 0; i < 3; i++) ut[i] *= f;
        *floored = 1;
    }
    Pout[IRHO] = rho;
    for (int i = 0; i < 3; i++) Pout[IU1 + i] = ut[i];
    Pout[IP] = prs;
    for (int i = 0; i < 3; i++) Pout[IB1 + i] = B[i];
    Pout[IPSI] = U[IPSI];
    if (p->entropy) Pout[IENT] = U[IENT] / U[ID];
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Grid: block list, padded layout and same-level ghost fill (Section 4.3).
 * ------------------------------------------------------------------------------- */
typedef struct {
    int level, size[3];
    int nslot[3];
    int *occ;            /* block id per slot, -1 if free */
} ogroup;

typedef struct {
    orc_params p;
    int64_t nb;
    orc_block *blk;
    int64_t *off;         /* padded offset, nb+1 */
    int64_t *ioff;        /* interior offset, nb+1 */
    int *grp;             /* group of each block */
    int ngroup;
    ogroup *groups;
    int gz;               /* ghost layers per axis */
    int gd[3];
    int maxlevel;
    int64_t *foff[3];     /* staggered face field: first face of each block per direction, nb+1 */
} orc_grid;

/* Where a block's cells and ghost slots sit in P (data contract shared with the
 * library): the block's interior cells first (x fastest), then the ghost slots of
 * its (size + 2g) box in box order with the interior skipped, the region rounded
 * up to 32 slots (the rest is padding). */
static int64_t ncell_axis(const orc_grid *G, int b, int e)
{
    return G->blk[b].size[e] + 2 * G->gd[e];
}

/* slots of block b's region */
static int64_t region_size(const orc_grid *G, int b)
{
    const int64_t box = ncell_axis(G, b, 0) * ncell_axis(G, b, 1) * ncell_axis(G, b, 2);
    return (box + 31) / 32 * 32;
}

static int64_t pad_index(const orc_grid *G, int b, int i, int j, int k)
{
    /* i, j, k: local indices, interior is [0, size) */
    const orc_block *B = &G->blk[b];
    const int s0 = B->size[0], s1 = B->size[1], s2 = B->size[2];
    if (i >= 0 && i < s0 && j >= 0 && j < s1 && k >= 0 && k < s2)
        return G->off[b] + ((int64_t)k * s1 + j) * s0 + i;
    /* a ghost slot: count the ghost slots that come before it in box order (whole
     * planes, then whole rows of its plane, then slots of its row) */
    const int g0 = G->gd[0], g1 = G->gd[1], g2 = G->gd[2];
    const int64_t w0 = s0 + 2 * g0, w1 = s1 + 2 * g1;
    const int64_t bx = i + g0, by = j + g1, bz = k + g2;
    const int64_t zin = bz - g2 < 0 ? 0 : (bz - g2 > s2 ? s2 : bz - g2);     /* interior planes before */
    int64_t before = bz * w0 * w1 - zin * s0 * s1;
    if (bz < g2 || bz >= s2 + g2) {
        before += by * w0 + bx;
    } else {
        const int64_t yin = by - g1 < 0 ? 0 : (by - g1 > s1 ? s1 : by - g1);  /* interior rows before */
        before += by * w0 - yin * s0;
        before += (by < g1 || by >= s1 + g1 || bx < g0) ? bx : bx - s0;
    }
    return G->off[b] + (int64_t)s0 * s1 * s2 + before;
}

static double level_dx(const orc_grid *G, int level, int e)
{
    OC_SCOPE(OC_OTHER);
    return (G->p.x_hi[e] - G->p.x_lo[e]) / ((double)G->p.ncell0[e] * (double)(1 << level));
}

void orc_grid_free(orc_grid *G)
{
    if (!G) return;
    for (int q = 0; q < G->ngroup; q++) free(G->groups[q].occ);
    free(G->groups);
    free(G->grp);
    free(G->off);
    free(G->ioff);
    for (int d = 0; d < 3; d++) free(G->foff[d]);
    free(G->blk);
    free(G);
}

/* Block of the given level whose region holds level-`level` cell c (each axis in
 * [0, N_level)), among blocks of the first block's size; -1 if none. Used by the
 * block-tree ghost rule, where all blocks share one size. */
static int leaf_at(const orc_grid *G, int level, const int64_t c[3])
{
    const orc_block *B0 = &G->blk[0];
    for (int q = 0; q < G->ngroup; q++) {
        const ogroup *g = &G->groups[q];
        if (g->level != level || g->size[0] != B0->size[0] || g->size[1] != B0->size[1]
            || g->size[2] != B0->size[2]) continue;
        int64_t sl[3];
        for (int e = 0; e < 3; e++) {
            sl[e] = c[e] / g->size[e];
            if (c[e] < 0 || sl[e] >= g->nslot[e]) return -1;
        }
        return g->occ[(sl[2] * g->nslot[1] + sl[1]) * g->nslot[0] + sl[0]];
    }
    return -1;
}

/* returns NULL on invalid input */
orc_grid *orc_grid_new(const orc_params *p, const orc_block *blocks, int64_t nb)
{
    if (nb <= 0 || p->ndim < 2 || p->ndim > 3 || p->nghost < 1) return NULL;
    orc_grid *G = calloc(1, sizeof *G);
    G->p = *p;
    G->nb = nb;
    G->blk = malloc(nb * sizeof(orc_block));
    memcpy(G->blk, blocks, nb * sizeof(orc_block));
    for (int e = 0; e < 3; e++) G->gd[e] = e < p->ndim ? p->nghost : 0;
    G->off = malloc((nb + 1) * sizeof(int64_t));
    G->ioff = malloc((nb + 1) * sizeof(int64_t));
    G->grp = malloc(nb * sizeof(int));
    G->off[0] = 0;
    G->ioff[0] = 0;
    G->maxlevel = 0;
    for (int64_t b = 0; b < nb; b++) {
        const orc_block *B = &G->blk[b];
        if (B->level < 0 || B->level > 20) goto bad;
        if (B->level > G->maxlevel) G->maxlevel = B->level;
        for (int e = 0; e < 3; e++) {
            if (e >= p->ndim) {
                if (B->size[e] != 1 || B->origin[e] != 0 || p->ncell0[e] != 1) goto bad;
                continue;
            }
            const int64_t N = (int64_t)p->ncell0[e] << B->level;
            if (B->size[e] < p->nghost || B->origin[e] < 0 || B->origin[e] % B->size[e] != 0) goto bad;
            if (B->origin[e] + B->size[e] > N || N % B->size[e] != 0) goto bad;
        }
        G->off[b + 1] = G->off[b] + region_size(G, (int)b);
        G->ioff[b + 1] = G->ioff[b] + (int64_t)B->size[0] * B->size[1] * B->size[2];
    }
    /* same (level, size) lattices with their occupancy */
    G->groups = NULL;
    G->ngroup = 0;
    for (int64_t b = 0; b < nb; b++) {
        const orc_block *B = &G->blk[b];
        int q;
        for (q = 0; q < G->ngroup; q++) {
            ogroup *g = &G->groups[q];
            if (g->level == B->level && g->size[0] == B->size[0] && g->size[1] == B->size[1]
                && g->size[2] == B->size[2]) break;
        }
        if (q == G->ngroup) {
            G->groups = realloc(G->groups, (G->ngroup + 1) * sizeof(ogroup));
            ogroup *g = &G->groups[G->ngroup++];
            g->level = B->level;
            int64_t tot = 1;
            for (int e = 0; e < 3; e++) {
                g->size[e] = B->size[e];
                g->nslot[e] = e < p->ndim ? (int)(((int64_t)p->ncell0[e] << B->level) / B->size[e]) : 1;
                tot *= g->nslot[e];
            }
            g->occ = malloc(tot * sizeof(int));
            for (int64_t t = 0; t < tot; t++) g->occ[t] = -1;
        }
        ogroup *g = &G->groups[q];
        G->grp[b] = q;
        const int64_t s = ((int64_t)(B->origin[2] / B->size[2]) * g->nslot[1] + B->origin[1] / B->size[1])
                          * g->nslot[0] + B->origin[0] / B->size[0];
        if (g->occ[s] != -1) goto bad;   /* two blocks in one slot */
        g->occ[s] = (int)b;
    }
    /* the entropy field: same-level patches only, gamma <= 2 (its inversion needs it) */
    if (p->entropy && (p->entropy != 1 || p->amr || !(p->gamma_ad <= 2.0))) goto bad;
    /* constrained transport: same-level patches without the entropy field */
    if (p->ct && (p->ct != 1 || p->amr || p->entropy)) goto bad;
    /* face layout of the staggered field (every block holds all faces of its cells,
     * both boundary faces included; blocks one after another, x fastest) */
    for (int d = 0; d < 3; d++) {
        G->foff[d] = malloc((nb + 1) * sizeof(int64_t));
        G->foff[d][0] = 0;
        for (int64_t b = 0; b < nb; b++) {
            const orc_block *B = &G->blk[b];
            const int64_t nf = d < p->ndim ? (int64_t)(B->size[0] + (d == 0)) * (B->size[1] + (d == 1))
                                                 * (B->size[2] + (d == 2))
                                           : 0;
            G->foff[d][b + 1] = G->foff[d][b] + nf;
        }
    }
    if (p->amr) {
        /* block tree: one block size, even and at least twice the ghost depth along
         * every axis in use (so every ghost layer lies in a leaf adjacent to the
         * block), and no leaf inside another leaf's region (no ancestor slot
         * occupied) */
        for (int64_t b = 0; b < nb; b++) {
            const orc_block *B = &G->blk[b];
            for (int e = 0; e < 3; e++) {
                if (B->size[e] != G->blk[0].size[e]) goto bad;
                if (e < p->ndim && (B->size[e] % 2 != 0 || B->size[e] < 2 * p->nghost)) goto bad;
            }
            for (int l = 0; l < B->level; l++) {
                int64_t c[3];
                for (int e = 0; e < 3; e++) c[e] = e < p->ndim ? (int64_t)B->origin[e] >> (B->level - l) : 0;
                if (leaf_at(G, l, c) >= 0) goto bad;
            }
        }
    }
    return G;
bad:
    orc_grid_free(G);
    return NULL;
}

void orc_grid_layout(const orc_grid *G, int64_t *off, int64_t *ioff)
{
    memcpy(off, G->off, (G->nb + 1) * sizeof(int64_t));
    memcpy(ioff, G->ioff, (G->nb + 1) * sizeof(int64_t));
}

/* Source of one ghost slot of block b at local (l0,l1,l2): (block, local index). */
static void ghost_source(const orc_grid *G, int b, const int l[3], int *sb, int src[3])
{
    const orc_block *B = &G->blk[b];
    const ogroup *g = &G->groups[G->grp[b]];
    int64_t Gi[3];
    int slot[3];
    for (int e = 0; e < 3; e++) {
        if (e >= G->p.ndim) { Gi[e] = 0; slot[e] = 0; continue; }
        const int64_t N = (int64_t)G->p.ncell0[e] << B->level;
        int64_t x = B->origin[e] + l[e];
        if (x < 0 || x >= N) {
            const int side = x < 0 ? 0 : 1;
            if (G->p.bc[e][side] == 0) x = ((x % N) + N) % N;        /* periodic wrap */
            else x = x < 0 ? 0 : N - 1;                              /* outflow clamp */
        }
        Gi[e] = x;
        slot[e] = (int)(x / B->size[e]);
    }
    const int64_t s = ((int64_t)slot[2] * g->nslot[1] + slot[1]) * g->nslot[0] + slot[0];
    const int nbk = g->occ[s];
    if (nbk >= 0) {
        *sb = nbk;
        for (int e = 0; e < 3; e++) src[e] = (int)(Gi[e] - (int64_t)slot[e] * B->size[e]);
    } else {
        *sb = b;                        /* no same-level block there: copy own edge cell */
        for (int e = 0; e < 3; e++) {
            int x = l[e];
            if (x < 0) x = 0;
            if (x > B->size[e] - 1) x = B->size[e] - 1;
            src[e] = x;
        }
    }
}

/* ---------------------------------------------------------------------------------
 * Block-tree ghost rule (amr = 1): the leaves of a 2:1-balanced tree of equal-size
 * blocks (Section 2's block-based adaptive mesh). A ghost position of a level-l
 * block is, after the domain's periodic wrap or outflow clamp at level l:
 *   held by a level-l leaf    -> that cell, copied;
 *   held by level-(l+1) leaves -> restriction: the mean of the 2^ndim fine cells
 *                                 covering it, summed z-outer, x-inner;
 *   held by a level-(l-1) leaf -> prolongation: coarse value q plus, per axis d,
 *                                 (+1/4 for the upper, -1/4 for the lower half of
 *                                 the coarse cell) times minmod(q - q_lo, q_hi - q),
 *                                 added in axis order; q_lo, q_hi are the coarse
 *                                 block's neighbour cells, taken from its interior
 *                                 or, outside it, by this rule without the
 *                                 prolongation case (a neighbour that would need it
 *                                 gives a zero slope on that axis);
 *   held by no leaf           -> the block's own nearest interior cell.
 * Every case reads interior cells only, so the fill is one pass in any order.
 * ------------------------------------------------------------------------------- */
static void ghost_global(const orc_grid *G, int b, const int l[3], int64_t Gi[3])
{
    const orc_block *B = &G->blk[b];
    for (int e = 0; e < 3; e++) {
        if (e >= G->p.ndim) { Gi[e] = 0; continue; }
        const int64_t N = (int64_t)G->p.ncell0[e] << B->level;
        int64_t x = B->origin[e] + l[e];
        if (x < 0 || x >= N) {
            if (G->p.bc[e][x < 0 ? 0 : 1] == 0) x = ((x % N) + N) % N;
            else x = x < 0 ? 0 : N - 1;
        }
        Gi[e] = x;
    }
}

static double minmod2(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}

static void copy_cell(const orc_grid *G, const double *P, int64_t ncp, int b, const int64_t Gi[3], double *out)
{
    const orc_block *B = &G->blk[b];
    const int64_t i = pad_index(G, b, (int)(Gi[0] - B->origin[0]), (int)(Gi[1] - B->origin[1]),
                                (int)(Gi[2] - B->origin[2]));
    for (int v = 0; v < NV; v++) out[v] = P[v * ncp + i];
}

static int tree_value(const orc_grid *G, const double *P, int64_t ncp, int b, const int l[3], int allow_prolong,
                      double *out);

/* value of coarse block cb at local position a (interior, or one cell outside along
 * one axis); 0 if that position would need prolongation */
static int coarse_neighbour(const orc_grid *G, const double *P, int64_t ncp, int cb, const int a[3], double *out)
{
    const orc_block *C = &G->blk[cb];
    int inside = 1;
    for (int e = 0; e < 3; e++) inside = inside && a[e] >= 0 && a[e] < C->size[e];
    if (inside) {
        const int64_t i = pad_index(G, cb, a[0], a[1], a[2]);
        for (int v = 0; v < NV; v++) out[v] = P[v * ncp + i];
        return 1;
    }
    return tree_value(G, P, ncp, cb, a, 0, out);
}

static void prolong(const orc_grid *G, const double *P, int64_t ncp, int cb, const int64_t c[3],
                    const int64_t Gi[3], double *out)
{
    const orc_block *C = &G->blk[cb];
    const int nd = G->p.ndim;
    const int lc[3] = { (int)(c[0] - C->origin[0]), (int)(c[1] - C->origin[1]), (int)(c[2] - C->origin[2]) };
    const int64_t ic = pad_index(G, cb, lc[0], lc[1], lc[2]);
    double lo[3][NV], hi[3][NV];
    int ok[3] = { 0, 0, 0 };
    for (int d = 0; d < nd; d++) {
        int a[3] = { lc[0], lc[1], lc[2] };
        a[d] = lc[d] - 1;
        const int okl = coarse_neighbour(G, P, ncp, cb, a, lo[d]);
        a[d] = lc[d] + 1;
        const int okh = coarse_neighbour(G, P, ncp, cb, a, hi[d]);
        ok[d] = okl && okh;
    }
    for (int v = 0; v < NV; v++) {
        const double q = P[v * ncp + ic];
        double val = q;
        for (int d = 0; d < nd; d++) {
            const double sl = ok[d] ? minmod2(q - lo[d][v], hi[d][v] - q) : 0.0;
            val += ((Gi[d] & 1) ? 0.25 : -0.25) * sl;
        }
        out[v] = val;
    }
}

static int tree_value(const orc_grid *G, const double *P, int64_t ncp, int b, const int l[3], int allow_prolong,
                      double *out)
{
    const orc_block *B = &G->blk[b];
    const int nd = G->p.ndim;
    int64_t Gi[3];
    ghost_global(G, b, l, Gi);
    int nbk = leaf_at(G, B->level, Gi);
    if (nbk >= 0) {
        copy_cell(G, P, ncp, nbk, Gi, out);
        return 1;
    }
    const int64_t f[3] = { 2 * Gi[0], nd > 1 ? 2 * Gi[1] : 0, nd > 2 ? 2 * Gi[2] : 0 };
    nbk = leaf_at(G, B->level + 1, f);
    if (nbk >= 0) {
        const orc_block *F = &G->blk[nbk];
        double sum[NV];
        for (int v = 0; v < NV; v++) sum[v] = 0.0;
        for (int dz = 0; dz < (nd > 2 ? 2 : 1); dz++)
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++) {
                    const int64_t i = pad_index(G, nbk, (int)(f[0] + dx - F->origin[0]), (int)(f[1] + dy - F->origin[1]),
                                                (int)(f[2] + dz - F->origin[2]));
                    for (int v = 0; v < NV; v++) sum[v] += P[v * ncp + i];
                }
        const double w = nd > 2 ? 0.125 : 0.25;
        for (int v = 0; v < NV; v++) out[v] = sum[v] * w;
        return 1;
    }
    if (B->level >= 1) {
        const int64_t c[3] = { Gi[0] >> 1, nd > 1 ? Gi[1] >> 1 : 0, nd > 2 ? Gi[2] >> 1 : 0 };
        nbk = leaf_at(G, B->level - 1, c);
        if (nbk >= 0) {
            if (!allow_prolong) return 0;
            prolong(G, P, ncp, nbk, c, Gi, out);
            return 1;
        }
    }
    int x[3];
    for (int e = 0; e < 3; e++) {
        x[e] = l[e] < 0 ? 0 : (l[e] > B->size[e] - 1 ? B->size[e] - 1 : l[e]);
    }
    const int64_t i = pad_index(G, b, x[0], x[1], x[2]);
    for (int v = 0; v < NV; v++) out[v] = P[v * ncp + i];
    return 1;
}

static void fill_block(const orc_grid *G, int b, double *P, int64_t ncp)
{
    const orc_block *B = &G->blk[b];
    const int g0 = G->gd[0], g1 = G->gd[1], g2 = G->gd[2];
    for (int k = -g2; k < B->size[2] + g2; k++)
        for (int j = -g1; j < B->size[1] + g1; j++)
            for (int i = -g0; i < B->size[0] + g0; i++) {
                const int inside = i >= 0 && i < B->size[0] && j >= 0 && j < B->size[1] && k >= 0
                                   && k < B->size[2];
                if (inside) continue;
                const int l[3] = { i, j, k };
                const int64_t dst = pad_index(G, b, i, j, k);
                if (G->p.amr) {
                    double val[NV];
                    tree_value(G, P, ncp, b, l, 1, val);
                    for (int v = 0; v < NV; v++) P[v * ncp + dst] = val[v];
                    continue;
                }
                int sb, src[3];
                ghost_source(G, b, l, &sb, src);
                const int64_t from = pad_index(G, sb, src[0], src[1], src[2]);
                for (int v = 0; v < nvar(&G->p); v++) P[v * ncp + dst] = P[v * ncp + from];
            }
}

/* blocks: subset of block ids (NULL = all) */
void orc_fill_ghosts(const orc_grid *G, double *P, const int64_t *blocks, int64_t nsel)
{
    const int64_t ncp = G->off[G->nb];
    const int64_t n = blocks ? nsel : G->nb;
    /* each block writes its own ghost slots from interior cells only */
#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int64_t q = 0; q < n; q++) fill_block(G, (int)(blocks ? blocks[q] : q), P, ncp);
}

static void cell_center(const orc_grid *G, int b, int i, int j, double *x1, double *x2)
{
    OC_SCOPE(OC_OTHER);
    const orc_block *B = &G->blk[b];
    *x1 = G->p.x_lo[0] + (B->origin[0] + i + 0.5) * level_dx(G, B->level, 0);
    *x2 = G->p.x_lo[1] + (B->origin[1] + j + 0.5) * level_dx(G, B->level, 1);
}

void orc_prim2con(const orc_grid *G, const double *P, double *U, const int64_t *blocks, int64_t nsel)
{
    const int64_t ncp = G->off[G->nb];
    const int64_t n = blocks ? nsel : G->nb;
#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int64_t q = 0; q < n; q++) {
        const int b = (int)(blocks ? blocks[q] : q);
        const orc_block *B = &G->blk[b];
        for (int k = 0; k < B->size[2]; k++)
            for (int j = 0; j < B->size[1]; j++)
                for (int i = 0; i < B->size[0]; i++) {
                    double x1, x2, Pc[NVE], Uc[NVE];
                    ometric m;
                    cell_center(G, b, i, j, &x1, &x2);
                    metric_at(&G->p, x1, x2, &m);
                    const int64_t c = pad_index(G, b, i, j, k);
                    for (int v = 0; v < nvar(&G->p); v++) Pc[v] = P[v * ncp + c];
                    p2c_point(&G->p, &m, Pc, Uc);
                    for (int v = 0; v < nvar(&G->p); v++) U[v * ncp + c] = Uc[v];
                }
    }
}

/* Standalone inversion: P_inout holds the guess on entry. fail: int8 per padded cell (nullable). */
void orc_con2prim(const orc_grid *G, const double *U, double *P, int8_t *fail, orc_state *st,
                  const int64_t *blocks, int64_t nsel)
{
    const int64_t ncp = G->off[G->nb];
    const int64_t n = blocks ? nsel : G->nb;
#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int64_t q = 0; q < n; q++) {
        const int b = (int)(blocks ? blocks[q] : q);
        const orc_block *B = &G->blk[b];
        ocount cnt = { 0, 0, 0, 0 };
        for (int k = 0; k < B->size[2]; k++)
            for (int j = 0; j < B->size[1]; j++)
                for (int i = 0; i < B->size[0]; i++) {
                    double x1, x2, Pg[NVE], Uc[NVE], Po[NVE];
                    ometric m;
                    cell_center(G, b, i, j, &x1, &x2);
                    metric_at(&G->p, x1, x2, &m);
                    const int64_t c = pad_index(G, b, i, j, k);
                    for (int v = 0; v < nvar(&G->p); v++) { Pg[v] = P[v * ncp + c]; Uc[v] = U[v * ncp + c]; }
                    int nit, fl, bk;
                    const int f = c2p_point(&G->p, &m, Uc, Pg, Po, &nit, &fl, &bk);
                    for (int v = 0; v < nvar(&G->p); v++) P[v * ncp + c] = Po[v];
                    if (fail) fail[c] = (int8_t)f;
                    cnt.fail += f;
                    cnt.backup += bk;
                    cnt.floors += (!f && fl);
                    if (nit > cnt.max_iter) cnt.max_iter = nit;
                }
        if (st) {
#pragma omp critical(oracle_counts)
            ocount_merge(st, &cnt);
        }
    }
}

/* ---------------------------------------------------------------------------------
 * Time step (reading): per-direction maximum |lambda| over faces of the last
 * substep, dt = C / sum_d(lam_d / dx_d) on the finest level present,
 * c_h = C / (dt sum_d 1/dx_d), kappa = alpha_glm c_h / min_d dx_d.
 * ------------------------------------------------------------------------------- */
static double dt_from_lam(const orc_grid *G, const double *lam)
{
    double s = 0.0;
    for (int d = 0; d < G->p.ndim; d++) s += lam[d] / level_dx(G, G->maxlevel, d);
    return G->p.cfl / s;
}

void orc_compute_dt(const orc_grid *G, const double *P, orc_state *st)
{
    const int64_t ncp = G->off[G->nb];
    double lam[3] = { 0.0, 0.0, 0.0 };
    /* maxima are exact, so the order in which blocks are visited does not matter */
#pragma omp parallel for schedule(dynamic) num_threads(g_threads) reduction(max : lam[:3])
    for (int64_t b = 0; b < G->nb; b++) {
        const orc_block *B = &G->blk[b];
        for (int k = 0; k < B->size[2]; k++)
            for (int j = 0; j < B->size[1]; j++)
                for (int i = 0; i < B->size[0]; i++) {
                    double x1, x2, Pc[NV], U[NV], F[NV], lm, lp;
                    ometric m;
                    cell_center(G, (int)b, i, j, &x1, &x2);
                    metric_at(&G->p, x1, x2, &m);
                    const int64_t c = pad_index(G, (int)b, i, j, k);
                    for (int v = 0; v < NV; v++) Pc[v] = P[v * ncp + c];
                    for (int d = 0; d < G->p.ndim; d++) {
                        phys_flux(&G->p, &m, Pc, d, U, F, &lm, &lp);
                        if (fabs(lm) > lam[d]) lam[d] = fabs(lm);
                        if (fabs(lp) > lam[d]) lam[d] = fabs(lp);
                    }
                }
    }
    st->dt_next = dt_from_lam(G, lam);
    st->have_dt = 1;
}

void orc_set_dt(orc_state *st, double dt)
{
    st->dt_fixed = dt;
    if (dt > 0.0) { st->dt_next = dt; st->have_dt = 1; }
}

/* ---------------------------------------------------------------------------------
 * One Runge-Kutta substep (Section 2: second-order explicit stepping; Section 4.2
 * counts each substep times the number of cells as the unit of work):
 *   U_out = a U_base + b (U_stage + dt L(U_stage)),
 *   L = -sum_d (F_{+1/2} - F_{-1/2}) / dx_d + S,
 * then the inversion of U_out with P_stage as the initial guess.
 * A substep with a == 0 starts a step and latches dt from the previous substep's
 * wave speeds. P_stage ghost slots must be filled. blocks: subset (NULL = all).
 * ------------------------------------------------------------------------------- */
/* Index of block b's face (i, j, k) of direction d in the staggered field array:
 * the directions' face arrays one after another, each block's faces x fastest. */
static int64_t phi_index(const orc_grid *G, int d, int b, int i, int j, int k)
{
    int64_t base = 0;
    for (int e = 0; e < d; e++) base += G->foff[e][G->nb];
    const orc_block *B = &G->blk[b];
    const int fs0 = B->size[0] + (d == 0), fs1 = B->size[1] + (d == 1);
    return base + G->foff[d][b] + ((int64_t)k * fs1 + j) * fs0 + i;
}

/* Face fluxes of block bk along every direction (F[d]: [9][faces], x fastest);
 * raises lam[d] to the largest |lambda| seen. Under constrained transport (Phi not
 * NULL) the normal field of each face is the staggered face field. */
static void block_fluxes(const orc_grid *G, int bk, const double *Ps, double ch, double *F[3], double *lam,
                         const double *Phi)
{
    const orc_params *p = &G->p;
    const int64_t ncp = G->off[G->nb];
    const orc_block *B = &G->blk[bk];
    for (int d = 0; d < p->ndim; d++) {
        int fs[3];
        for (int e = 0; e < 3; e++) fs[e] = B->size[e] + (e == d);
        const int64_t nf = (int64_t)fs[0] * fs[1] * fs[2];
        const double dx = level_dx(G, B->level, d);
        for (int k = 0; k < fs[2]; k++)
            for (int j = 0; j < fs[1]; j++)
                for (int i = 0; i < fs[0]; i++) {
                    /* face between the cell at (i,j,k) - e_d and the cell at (i,j,k) */
                    int c[3] = { i, j, k };
                    double qv[6], PL[NV], PR[NV];
                    /* MC reads cells i-2..i+1, PPM reads i-3..i+2 */
                    const int t0 = p->recon == 0 ? 1 : 0, t1 = p->recon == 0 ? 5 : 6;
                    for (int t = 0; t < 6; t++) qv[t] = 0.0;
                    for (int v = 0; v < NV; v++) {
                        for (int t = t0; t < t1; t++) {
                            int cc[3] = { c[0], c[1], c[2] };
                            cc[d] += t - 3;
                            qv[t] = Ps[v * ncp + pad_index(G, bk, cc[0], cc[1], cc[2])];
                        }
                        recon_face(p->recon, qv, &PL[v], &PR[v]);
                    }
                    double x1, x2;
                    cell_center(G, bk, i, j, &x1, &x2);
                    if (d == 0) x1 = p->x_lo[0] + (B->origin[0] + i) * dx;
                    if (d == 1) x2 = p->x_lo[1] + (B->origin[1] + j) * dx;
                    ometric mf;
                    metric_at(p, x1, x2, &mf);
                    double Ff[NVE];
                    const double l = Phi ? riemann_ct(p, &mf, d, PL, PR, Phi[phi_index(G, d, bk, i, j, k)], Ff)
                                         : riemann(p, &mf, d, PL, PR, ch, Ff);
                    if (l > lam[d]) lam[d] = l;
                    if (p->entropy) {
                        /* entropy field (reading 19): reconstructed like the others and
                         * carried by the mass flux from its upwind side */
                        double KL, KR;
                        for (int t = t0; t < t1; t++) {
                            int cc[3] = { c[0], c[1], c[2] };
                            cc[d] += t - 3;
                            qv[t] = Ps[IENT * ncp + pad_index(G, bk, cc[0], cc[1], cc[2])];
                        }
                        recon_face(p->recon, qv, &KL, &KR);
                        Ff[IENT] = Ff[ID] * (Ff[ID] >= 0.0 ? KL : KR);
                    }
                    const int64_t fi = ((int64_t)k * fs[1] + j) * fs[0] + i;
                    for (int v = 0; v < nvar(p); v++) F[d][v * nf + fi] = Ff[v];
                }
    }
}

/* Flux divergence, sources, RK combine and inversion of block bk. */
static void block_update(const orc_grid *G, int bk, double *F[3], const double *Ub, const double *Us,
                         const double *Ps, double *Uo, double *Po, double a, double b, const orc_state *st,
                         ocount *cnt, const double *Phio)
{
    const orc_params *p = &G->p;
    const int64_t ncp = G->off[G->nb];
    const orc_block *B = &G->blk[bk];
    for (int k = 0; k < B->size[2]; k++)
        for (int j = 0; j < B->size[1]; j++)
            for (int i = 0; i < B->size[0]; i++) {
                OC_SCOPE(OC_UPDATE);
                const int64_t c = pad_index(G, bk, i, j, k);
                const int nv = nvar(p);
                double x1, x2, Pc[NVE], Uc[NVE], Sv[NVE], L[NVE], Un[NVE], Pn[NVE];
                ometric m;
                cell_center(G, bk, i, j, &x1, &x2);
                metric_at(p, x1, x2, &m);
                for (int v = 0; v < nv; v++) { Pc[v] = Ps[v * ncp + c]; Uc[v] = Us[v * ncp + c]; }
                sources_point(p, &m, Pc, Uc, st->kappa, Sv);
                Sv[IENT] = 0.0;                     /* the entropy field has no source */
                for (int v = 0; v < nv; v++) L[v] = 0.0;
                for (int d = 0; d < p->ndim; d++) {
                    int fs[3];
                    for (int e = 0; e < 3; e++) fs[e] = B->size[e] + (e == d);
                    const double dx = level_dx(G, B->level, d);
                    const int64_t nf = (int64_t)fs[0] * fs[1] * fs[2];
                    int hi[3] = { i, j, k };
                    hi[d] += 1;
                    const int64_t flo = ((int64_t)k * fs[1] + j) * fs[0] + i;
                    const int64_t fhi = ((int64_t)hi[2] * fs[1] + hi[1]) * fs[0] + hi[0];
                    for (int v = 0; v < nv; v++) L[v] -= (F[d][v * nf + fhi] - F[d][v * nf + flo]) / dx;
                }
                for (int v = 0; v < nv; v++) {
                    L[v] += Sv[v];
                    Un[v] = a * Ub[v * ncp + c] + b * (Uc[v] + st->dt * L[v]);
                }
                if (Phio) {
                    /* constrained transport: the cell's densitised field is the mean of
                     * its two updated face fields along each resolved direction */
                    for (int d = 0; d < p->ndim; d++) {
                        int hi[3] = { i, j, k };
                        hi[d] += 1;
                        Un[IB1 + d] = 0.5 * (Phio[phi_index(G, d, bk, i, j, k)]
                                             + Phio[phi_index(G, d, bk, hi[0], hi[1], hi[2])]);
                    }
                }
                int nit, fl, bu;
                const int f = c2p_point(p, &m, Un, Pc, Pn, &nit, &fl, &bu);
                /* failed, floored or backed-up cells take the conserved state of
                 * their primitives (the energy is what could not be inverted) */
                if (f || fl || bu) p2c_point(p, &m, Pn, Un);
                cnt->fail += f;
                cnt->backup += bu;
                cnt->floors += (!f && fl);
                if (nit > cnt->max_iter) cnt->max_iter = nit;
                for (int v = 0; v < nv; v++) { Uo[v * ncp + c] = Un[v]; Po[v * ncp + c] = Pn[v]; }
            }
}

/* Flux correction of a block tree: every face of a block whose far side lies in
 * finer leaves takes the mean of the 2^(ndim-1) fine faces covering it (summed
 * with the second transverse axis outer), so what leaves a coarse cell through
 * that face is what the fine cells receive and the scheme conserves across levels. */
static void flux_fix(const orc_grid *G, double **F)
{
    const orc_params *p = &G->p;
    const int nd = p->ndim;
    for (int64_t bk = 0; bk < G->nb; bk++) {
        const orc_block *B = &G->blk[bk];
        for (int d = 0; d < nd; d++) {
            int fs[3];
            for (int e = 0; e < 3; e++) fs[e] = B->size[e] + (e == d);
            const int64_t nf = (int64_t)fs[0] * fs[1] * fs[2];
            const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;   /* transverse axes */
            for (int side = 0; side < 2; side++) {
                const int fidx = side ? B->size[d] : 0;          /* face index along d */
                for (int ib = 0; ib < B->size[tb]; ib++)
                    for (int ia = 0; ia < B->size[ta]; ia++) {
                        int l[3];
                        l[d] = side ? B->size[d] : -1;
                        l[ta] = ia;
                        l[tb] = ib;
                        int64_t Gi[3];
                        ghost_global(G, (int)bk, l, Gi);
                        if (leaf_at(G, B->level, Gi) >= 0) break;   /* same level: whole face */
                        const int64_t f[3] = { 2 * Gi[0], nd > 1 ? 2 * Gi[1] : 0, nd > 2 ? 2 * Gi[2] : 0 };
                        const int fb = leaf_at(G, B->level + 1, f);
                        if (fb < 0) break;                             /* not a finer neighbour */
                        const orc_block *Fb = &G->blk[fb];
                        int ffs[3];
                        for (int e = 0; e < 3; e++) ffs[e] = Fb->size[e] + (e == d);
                        const int64_t fnf = (int64_t)ffs[0] * ffs[1] * ffs[2];
                        double sum[NV];
                        for (int v = 0; v < NV; v++) sum[v] = 0.0;
                        const int nb_ = nd > 2 ? 2 : 1;
                        for (int sb = 0; sb < nb_; sb++)
                            for (int sa = 0; sa < 2; sa++) {
                                int fl[3];
                                /* fine face: adjacent to the coarse face on the fine side */
                                fl[d] = side ? (int)(f[d] - Fb->origin[d]) : (int)(f[d] + 1 - Fb->origin[d]) + 1;
                                fl[ta] = (int)(f[ta] + sa - Fb->origin[ta]);
                                fl[tb] = nd > 2 || tb < nd ? (int)(f[tb] + sb - Fb->origin[tb]) : 0;
                                const int64_t fi = ((int64_t)fl[2] * ffs[1] + fl[1]) * ffs[0] + fl[0];
                                for (int v = 0; v < NV; v++) sum[v] += F[fb * 3 + d][v * fnf + fi];
                            }
                        const double w = nd > 2 ? 0.25 : 0.5;
                        int cl[3];
                        cl[d] = fidx;
                        cl[ta] = ia;
                        cl[tb] = ib;
                        const int64_t ci = ((int64_t)cl[2] * fs[1] + cl[1]) * fs[0] + cl[0];
                        for (int v = 0; v < NV; v++) F[bk * 3 + d][v * nf + ci] = sum[v] * w;
                    }
            }
        }
    }
}

/* One RK substep on the selected blocks (NULL = all): U_out = a U_base + b (U_stage +
 * dt L), then P_out = con2prim(U_out) with P_stage as the guess; records the largest
 * wave speeds. P_stage ghost slots must be filled. For block trees the fluxes of all
 * blocks are formed first and corrected at level boundaries (flux_fix). */
int orc_substep(const orc_grid *G, const double *Ub, const double *Us, const double *Ps, double *Uo,
                double *Po, double a, double b, orc_state *st, const int64_t *blocks, int64_t nsel)
{
    if (!st->have_dt) return -1;
    const orc_params *p = &G->p;
    if (a == 0.0) {
        st->dt = st->dt_fixed > 0.0 ? st->dt_fixed : st->dt_next;
        double sinv = 0.0, dmin = 1e300;
        for (int d = 0; d < p->ndim; d++) {
            const double dx = level_dx(G, G->maxlevel, d);
            sinv += 1.0 / dx;
            if (dx < dmin) dmin = dx;
        }
        st->ch = p->cfl / (st->dt * sinv);
        st->kappa = p->glm_alpha * st->ch / dmin;
    }
    double lam[3] = { 0.0, 0.0, 0.0 };
    const int64_t n = blocks ? nsel : G->nb;
    if (!p->amr) {
        /* blocks are independent: each reads P_stage and U and writes only its own
         * cells of U_out and P_out (which alias no input read by another block) */
#pragma omp parallel for schedule(dynamic) num_threads(g_threads) reduction(max : lam[:3])
        for (int64_t q = 0; q < n; q++) {
            const int bk = (int)(blocks ? blocks[q] : q);
            const orc_block *B = &G->blk[bk];
            double *F[3] = { NULL, NULL, NULL };
            for (int d = 0; d < p->ndim; d++) {
                const int64_t nf = (int64_t)(B->size[0] + (d == 0)) * (B->size[1] + (d == 1)) * (B->size[2] + (d == 2));
                F[d] = malloc(nvar(p) * nf * sizeof(double));
            }
            ocount cnt = { 0, 0, 0, 0 };
            block_fluxes(G, bk, Ps, st->ch, F, lam, NULL);
            block_update(G, bk, F, Ub, Us, Ps, Uo, Po, a, b, st, &cnt, NULL);
#pragma omp critical(oracle_counts)
            ocount_merge(st, &cnt);
            for (int d = 0; d < p->ndim; d++) free(F[d]);
        }
    } else {
        /* block tree: every block's fluxes (a coarse face needs its fine neighbours'),
         * the level-boundary correction, then the update of the selected blocks */
        double **F = calloc(3 * G->nb, sizeof(double *));
#pragma omp parallel for schedule(dynamic) num_threads(g_threads) reduction(max : lam[:3])
        for (int64_t bk = 0; bk < G->nb; bk++) {
            const orc_block *B = &G->blk[bk];
            double *Fb[3] = { NULL, NULL, NULL };
            for (int d = 0; d < p->ndim; d++) {
                const int64_t nf = (int64_t)(B->size[0] + (d == 0)) * (B->size[1] + (d == 1)) * (B->size[2] + (d == 2));
                F[bk * 3 + d] = malloc(NV * nf * sizeof(double));
                Fb[d] = F[bk * 3 + d];
            }
            block_fluxes(G, (int)bk, Ps, st->ch, Fb, lam, NULL);
        }
        flux_fix(G, F);
#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
        for (int64_t q = 0; q < n; q++) {
            const int bk = (int)(blocks ? blocks[q] : q);
            ocount cnt = { 0, 0, 0, 0 };
            block_update(G, bk, &F[bk * 3], Ub, Us, Ps, Uo, Po, a, b, st, &cnt, NULL);
#pragma omp critical(oracle_counts)
            ocount_merge(st, &cnt);
        }
        for (int64_t t = 0; t < 3 * G->nb; t++) free(F[t]);
        free(F);
    }
    for (int d = 0; d < 3; d++) st->lam[d] = lam[d];
    st->dt_next = st->dt_fixed > 0.0 ? st->dt_fixed : dt_from_lam(G, lam);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Staggered-mesh constrained transport (Section 2: the paper's code evolves the
 * magnetic field by constrained transport on a staggered mesh). Reading:
 *  - the field is held as phi^d = sqrt(gamma) B^d at the centre of every d-face (a
 *    block holds all faces of its cells, so a face shared by two blocks has a copy in
 *    each, kept identical);
 *  - the face fluxes come from the usual reconstruction and Riemann solve, with the
 *    face's phi as the normal field of both states and no GLM solve;
 *  - the induction fluxes give the edge electric fields (i, j, k cyclic)
 *      E_k = F^j(B~^i) = -F^i(B~^j),
 *    each edge value the mean of the four face fluxes around the edge (two faces of
 *    each of the two directions normal to the edge);
 *  - phi is advanced by Stokes' theorem, d_t phi^i = -(d_j E_k - d_k E_j), in the
 *    same RK combination as U; the cell's densitised field in U is the mean of its two
 *    updated face fields along each resolved direction (with ndim = 2 the x3 field
 *    stays a cell-centred finite-volume variable);
 *  - a face flux across a block boundary is read from the same-level block beside
 *    it; where there is none (outflow), from the block's own nearest face.
 * The discrete divergence sum_d (phi^d(hi) - phi^d(lo)) / dx_d of every cell is then
 * kept at its initial value to round-off.
 * ------------------------------------------------------------------------------- */
/* flux row v of direction d at block bk's face f (f[d] a face index 0..s_d, the
 * other two cell indices, at most one of them outside the block) */
static double flux_at(const orc_grid *G, double **F, int bk, int d, int v, const int f[3])
{
    const orc_block *B = &G->blk[bk];
    int b = bk, g[3] = { f[0], f[1], f[2] };
    for (int e = 0; e < 3; e++) {
        if (e == d || (f[e] >= 0 && f[e] < B->size[e])) continue;
        int l[3] = { f[0], f[1], f[2] };
        if (l[d] > B->size[d] - 1) l[d] = B->size[d] - 1;
        int sb, src[3];
        ghost_source(G, bk, l, &sb, src);
        b = sb;
        g[e] = src[e];
    }
    const orc_block *N = &G->blk[b];
    int fs[3];
    for (int e = 0; e < 3; e++) fs[e] = N->size[e] + (e == d);
    const int64_t nf = (int64_t)fs[0] * fs[1] * fs[2];
    return F[b * 3 + d][v * nf + ((int64_t)g[2] * fs[1] + g[1]) * fs[0] + g[0]];
}

/* edge electric field E_k of block bk at the edge whose lower corner is (i, j, k) in
 * face-index units along the two axes normal to the edge (cell index along k) */
static double edge_emf(const orc_grid *G, double **F, int bk, int axis, int i, int j, int k)
{
    /* (a, b): the two axes normal to the edge, cyclic after the edge's axis */
    const int a = (axis + 1) % 3, b = (axis + 2) % 3;
    int fa0[3] = { i, j, k }, fa1[3] = { i, j, k }, fb0[3] = { i, j, k }, fb1[3] = { i, j, k };
    /* F^b(B~^a) on the two b-faces beside the edge (cells a-1 and a along a) */
    fb0[a] -= 1;
    /* F^a(B~^b) on the two a-faces beside the edge (cells b-1 and b along b) */
    fa0[b] -= 1;
    const double fb = flux_at(G, F, bk, b, IB1 + a, fb0) + flux_at(G, F, bk, b, IB1 + a, fb1);
    const double fa = flux_at(G, F, bk, a, IB1 + b, fa0) + flux_at(G, F, bk, a, IB1 + b, fa1);
    return 0.25 * (fb - fa);
}

/* new face fields of block bk: phi_out = a phi_base + b (phi_stage + dt L) with
 * L = -(d_j E_k - d_k E_j) on each face of direction i */
static void block_ct_update(const orc_grid *G, int bk, double **F, const double *Phib, const double *Phis,
                            double *Phio, double a, double b, double dt)
{
    const orc_params *p = &G->p;
    const orc_block *B = &G->blk[bk];
    double dx[3];
    for (int e = 0; e < 3; e++) dx[e] = level_dx(G, B->level, e);
    for (int d = 0; d < p->ndim; d++) {
        int fs[3];
        for (int e = 0; e < 3; e++) fs[e] = B->size[e] + (e == d);
        const int dj = (d + 1) % 3, dk = (d + 2) % 3;
        for (int k = 0; k < fs[2]; k++)
            for (int j = 0; j < fs[1]; j++)
                for (int i = 0; i < fs[0]; i++) {
                    double L = 0.0;
                    /* -d_j E_k: edges along dk at the low and high side along dj (with
                     * ndim = 2 only the edges along x3 exist: the other term vanishes) */
                    if (dj < p->ndim) {
                        int lo[3] = { i, j, k }, hi[3] = { i, j, k };
                        hi[dj] += 1;
                        L -= (edge_emf(G, F, bk, dk, hi[0], hi[1], hi[2]) - edge_emf(G, F, bk, dk, lo[0], lo[1], lo[2]))
                             / dx[dj];
                    }
                    /* +d_k E_j: edges along dj at the low and high side along dk */
                    if (dk < p->ndim) {
                        int lo[3] = { i, j, k }, hi[3] = { i, j, k };
                        hi[dk] += 1;
                        L += (edge_emf(G, F, bk, dj, hi[0], hi[1], hi[2]) - edge_emf(G, F, bk, dj, lo[0], lo[1], lo[2]))
                             / dx[dk];
                    }
                    const int64_t q = phi_index(G, d, bk, i, j, k);
                    Phio[q] = a * Phib[q] + b * (Phis[q] + dt * L);
                }
    }
}

/* One RK substep under constrained transport: as orc_substep, plus the face fields
 * (phi: every block's faces of each resolved direction, the directions one after
 * another). Every block's fluxes are formed first (the edge fields of a block read
 * its neighbours' faces), then the face fields and the cells of the selected
 * blocks. */
int orc_substep_ct(const orc_grid *G, const double *Ub, const double *Us, const double *Ps, const double *Phib,
                   const double *Phis, double *Uo, double *Po, double *Phio, double a, double b, orc_state *st,
                   const int64_t *blocks, int64_t nsel)
{
    if (!st->have_dt || !G->p.ct) return -1;
    const orc_params *p = &G->p;
    if (a == 0.0) {
        st->dt = st->dt_fixed > 0.0 ? st->dt_fixed : st->dt_next;
        double sinv = 0.0, dmin = 1e300;
        for (int d = 0; d < p->ndim; d++) {
            const double dx = level_dx(G, G->maxlevel, d);
            sinv += 1.0 / dx;
            if (dx < dmin) dmin = dx;
        }
        st->ch = p->cfl / (st->dt * sinv);
        st->kappa = p->glm_alpha * st->ch / dmin;
    }
    double lam[3] = { 0.0, 0.0, 0.0 };
    const int64_t n = blocks ? nsel : G->nb;
    double **F = calloc(3 * G->nb, sizeof(double *));
#pragma omp parallel for schedule(dynamic) num_threads(g_threads) reduction(max : lam[:3])
    for (int64_t bk = 0; bk < G->nb; bk++) {
        const orc_block *B = &G->blk[bk];
        double *Fb[3] = { NULL, NULL, NULL };
        for (int d = 0; d < p->ndim; d++) {
            const int64_t nf = (int64_t)(B->size[0] + (d == 0)) * (B->size[1] + (d == 1)) * (B->size[2] + (d == 2));
            F[bk * 3 + d] = malloc(NV * nf * sizeof(double));
            Fb[d] = F[bk * 3 + d];
        }
        block_fluxes(G, (int)bk, Ps, st->ch, Fb, lam, Phis);
    }
#pragma omp parallel for schedule(dynamic) num_threads(g_threads)
    for (int64_t q = 0; q < n; q++) {
        const int bk = (int)(blocks ? blocks[q] : q);
        block_ct_update(G, bk, F, Phib, Phis, Phio, a, b, st->dt);
        ocount cnt = { 0, 0, 0, 0 };
        block_update(G, bk, &F[bk * 3], Ub, Us, Ps, Uo, Po, a, b, st, &cnt, Phio);
#pragma omp critical(oracle_counts)
        ocount_merge(st, &cnt);
    }
    for (int64_t t = 0; t < 3 * G->nb; t++) free(F[t]);
    free(F);
    for (int d = 0; d < 3; d++) st->lam[d] = lam[d];
    st->dt_next = st->dt_fixed > 0.0 ? st->dt_fixed : dt_from_lam(G, lam);
    return 0;
}

/* Faces per direction (totals over the blocks) of the staggered field. */
void orc_face_count(const orc_grid *G, int64_t *nface)
{
    for (int d = 0; d < 3; d++) nface[d] = G->foff[d][G->nb];
}

/* Cell-centred field from the face field: P rows B^d (d < ndim) = the mean of the
 * cell's two face values of phi^d divided by sqrt(gamma) at the cell centre. */
void orc_ct_center(const orc_grid *G, const double *Phi, double *P)
{
    const int64_t ncp = G->off[G->nb];
    for (int64_t b = 0; b < G->nb; b++) {
        const orc_block *B = &G->blk[b];
        for (int k = 0; k < B->size[2]; k++)
            for (int j = 0; j < B->size[1]; j++)
                for (int i = 0; i < B->size[0]; i++) {
                    double x1, x2;
                    ometric m;
                    cell_center(G, (int)b, i, j, &x1, &x2);
                    metric_at(&G->p, x1, x2, &m);
                    const int64_t c = pad_index(G, (int)b, i, j, k);
                    for (int d = 0; d < G->p.ndim; d++) {
                        int hi[3] = { i, j, k };
                        hi[d] += 1;
                        const double mean = 0.5 * (Phi[phi_index(G, d, (int)b, i, j, k)]
                                                   + Phi[phi_index(G, d, (int)b, hi[0], hi[1], hi[2])]);
                        P[(IB1 + d) * ncp + c] = mean / m.sqrtg;
                    }
                }
    }
}

/* Discrete divergence of the face field per interior cell (interior-packed order):
 * sum_d (phi^d(hi) - phi^d(lo)) / dx_d. */
void orc_ct_divergence(const orc_grid *G, const double *Phi, double *div)
{
    for (int64_t b = 0; b < G->nb; b++) {
        const orc_block *B = &G->blk[b];
        int64_t c = G->ioff[b];
        for (int k = 0; k < B->size[2]; k++)
            for (int j = 0; j < B->size[1]; j++)
                for (int i = 0; i < B->size[0]; i++, c++) {
                    double s = 0.0;
                    for (int d = 0; d < G->p.ndim; d++) {
                        int hi[3] = { i, j, k };
                        hi[d] += 1;
                        s += (Phi[phi_index(G, d, (int)b, hi[0], hi[1], hi[2])] - Phi[phi_index(G, d, (int)b, i, j, k)])
                             / level_dx(G, B->level, d);
                    }
                    div[c] = s;
                }
    }
}

/* ---------------------------------------------------------------------------------
 * Pointwise entry points for the unit pins.
 * ------------------------------------------------------------------------------- */
void orc_metric(const orc_params *p, double x1, double x2, double *out)
{
    /* out: alpha, beta[3], g[9], gi[9], sqrtg, da[3], db[9] ([j][i]), dg[27] ([j][i][k]) = 62 */
    ometric m;
    metric_at(p, x1, x2, &m);
    int o = 0;
    out[o++] = m.alpha;
    for (int i = 0; i < 3; i++) out[o++] = m.beta[i];
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) out[o++] = m.g[i][j];
    for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) out[o++] = m.gi[i][j];
    out[o++] = m.sqrtg;
    for (int j = 0; j < 3; j++) out[o++] = m.da[j];
    for (int j = 0; j < 3; j++) for (int i = 0; i < 3; i++) out[o++] = m.db[j][i];
    for (int j = 0; j < 3; j++) for (int i = 0; i < 3; i++) for (int k = 0; k < 3; k++) out[o++] = m.dg[j][i][k];
}

void orc_p2c_point(const orc_params *p, double x1, double x2, const double *P, double *U)
{
    ometric m;
    metric_at(p, x1, x2, &m);
    p2c_point(p, &m, P, U);
}

/* info[0] = fail, info[1] = Newton steps, info[2] = floored, info[3] = entropy backup used */
void orc_c2p_point(const orc_params *p, double x1, double x2, const double *U, const double *Pg,
                   double *Pout, int *info)
{
    ometric m;
    metric_at(p, x1, x2, &m);
    int nit, fl, bk;
    info[0] = c2p_point(p, &m, U, Pg, Pout, &nit, &fl, &bk);
    info[1] = nit;
    info[2] = fl;
    info[3] = bk;
}

/* The two-unknown Newton iteration alone, from the guess primitives Pg (no 1-D
 * iteration first, no floors): P from U. Returns 0 on convergence to a physical state
 * (rho > 0, p >= 0); *nit = steps taken. */
static void c2p_system(const orc_params *p, const ometric *m, const double *U, c2p_sys *c, double Sl[3],
                       double B[3], double Bl[3])
{
    const double sg = m->sqrtg;
    c->gam = p->gamma_ad;
    c->D = U[ID] / sg;
    for (int i = 0; i < 3; i++) { Sl[i] = U[IS1 + i] / sg; B[i] = U[IB1 + i] / sg; }
    c->Ut = U[ITAU] / sg + c->D;
    c->S2 = 0.0;
    c->B2 = 0.0;
    c->SB = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) c->S2 += m->gi[i][j] * Sl[i] * Sl[j];
    for (int i = 0; i < 3; i++) {
        Bl[i] = 0.0;
        for (int j = 0; j < 3; j++) Bl[i] += m->g[i][j] * B[j];
    }
    for (int i = 0; i < 3; i++) { c->B2 += B[i] * Bl[i]; c->SB += Sl[i] * B[i]; }
}

int orc_c2p_2d_point(const orc_params *p, double x1, double x2, const double *U, const double *Pg, double *Pout,
                     int *nit)
{
    ometric m;
    metric_at(p, x1, x2, &m);
    c2p_sys c;
    double Sl[3], B[3], Bl[3];
    c2p_system(p, &m, U, &c, Sl, B, Bl);
    ostate g;
    state_from_prim(p, &m, Pg, &g);
    double xi, q;
    if (c2p_newton2(&c, g.xi, g.W * g.W - 1.0, p->c2p_tol, p->c2p_maxit, &xi, &q, nit)) return 1;
    const double W = sqrt(1.0 + q), rho = c.D / W;
    const double prs = (c.gam - 1.0) / c.gam * (xi / (W * W) - rho);
    if (!(rho > 0.0) || !(prs >= 0.0)) return 1;
    Pout[IRHO] = rho;
    for (int i = 0; i < 3; i++) {
        double vu = 0.0;
        for (int j = 0; j < 3; j++) vu += m.gi[i][j] * (Sl[j] + c.SB * Bl[j] / xi) / (xi + c.B2);
        Pout[IU1 + i] = W * vu;
    }
    Pout[IP] = prs;
    for (int i = 0; i < 3; i++) Pout[IB1 + i] = B[i];
    Pout[IPSI] = U[IPSI];
    return 0;
}

/* Residuals (F1, F2) and Jacobian (row-major) of the two-unknown system at (xi, q). */
void orc_c2p_2d_residual(const orc_params *p, double x1, double x2, const double *U, double xi, double q, double *F,
                         double *J)
{
    ometric m;
    metric_at(p, x1, x2, &m);
    c2p_sys c;
    double Sl[3], B[3], Bl[3];
    c2p_system(p, &m, U, &c, Sl, B, Bl);
    double Jm[2][2];
    c2p2_fj(&c, xi, q, F, Jm);
    J[0] = Jm[0][0];
    J[1] = Jm[0][1];
    J[2] = Jm[1][0];
    J[3] = Jm[1][1];
}

/* The entropy root alone (no energy inversion first): P from U (U[9] = U[0] K).
 * Returns 0 on success. */
int orc_c2p_entropy_point(const orc_params *p, double x1, double x2, const double *U, double Wg, double *Pout)
{
    ometric m;
    metric_at(p, x1, x2, &m);
    const double sg = m.sqrtg;
    c2p_sys c;
    c.gam = p->gamma_ad;
    c.D = U[ID] / sg;
    double Sl[3], B[3], Bl[3];
    for (int i = 0; i < 3; i++) { Sl[i] = U[IS1 + i] / sg; B[i] = U[IB1 + i] / sg; }
    c.Ut = 0.0;
    c.S2 = 0.0;
    c.B2 = 0.0;
    c.SB = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) c.S2 += m.gi[i][j] * Sl[i] * Sl[j];
    for (int i = 0; i < 3; i++) {
        Bl[i] = 0.0;
        for (int j = 0; j < 3; j++) Bl[i] += m.g[i][j] * B[j];
    }
    for (int i = 0; i < 3; i++) { c.B2 += B[i] * Bl[i]; c.SB += Sl[i] * B[i]; }
    const double K = U[IENT] / U[ID];
    double W, xi;
    if (c2p_entropy(&c, K, Wg, p->c2p_tol, &W, &xi)) return 1;
    const double rho = c.D / W;
    Pout[IRHO] = rho;
    for (int i = 0; i < 3; i++) {
        double vu = 0.0;
        for (int j = 0; j < 3; j++) vu += m.gi[i][j] * (Sl[j] + c.SB * Bl[j] / xi) / (xi + c.B2);
        Pout[IU1 + i] = W * vu;
    }
    Pout[IP] = K * pow(rho, c.gam);
    for (int i = 0; i < 3; i++) Pout[IB1 + i] = B[i];
    Pout[IPSI] = U[IPSI];
    Pout[IENT] = K;
    return 0;
}

void orc_phys_flux(const orc_params *p, double x1, double x2, const double *P, int d, double *U,
                   double *F, double *lam)
{
    ometric m;
    metric_at(p, x1, x2, &m);
    phys_flux(p, &m, P, d, U, F, &lam[0], &lam[1]);
}

double orc_riemann(const orc_params *p, double x1, double x2, int d, const double *PL,
                   const double *PR, double ch, double *F)
{
    ometric m;
    metric_at(p, x1, x2, &m);
    return riemann(p, &m, d, PL, PR, ch, F);
}

void orc_recon_face(int method, const double *q, double *qLR)
{
    recon_face(method, q, &qLR[0], &qLR[1]);
}

void orc_sources(const orc_params *p, double x1, double x2, const double *P, const double *U,
                 double kappa, double *S)
{
    ometric m;
    metric_at(p, x1, x2, &m);
    sources_point(p, &m, P, U, kappa, S);
}
