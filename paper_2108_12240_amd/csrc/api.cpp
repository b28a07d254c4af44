// C ABI of the GRMHD substep library: argument checks, device memory of a grid,
// and dispatch to the kernel launchers. No exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "device.h"

struct bhac_grid {
    bhac::DeviceGrid dg;
    hipStream_t last_stream = nullptr;
    hipStream_t cap_stream = nullptr;      // owned: capture of the RK2-step graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

// face-flux scratch of bhac_substep_noalloc (64 MiB per GPU; see below)
static __device__ __align__(256) unsigned char scratch[size_t(64) << 20];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return BHAC_EDEVICE;
}

template <typename T>
hipError_t upload(T **dst, const T *src, size_t n)
{
    *dst = nullptr;
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc((void **)dst, n * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

void release_timer(bhac::DeviceGrid &G)
{
    for (hipEvent_t e : G.timer.pool) (void)hipEventDestroy(e);
    G.timer.pool.clear();
    G.timer.recs.clear();
    G.timer.used = 0;
    G.timer.on = false;
}

void release(bhac::DeviceGrid &G)
{
    release_timer(G);
    void *ptrs[] = {G.d_blocks, G.d_levels, G.d_ctab, G.d_f0tab, G.d_f1tab, G.d_ctab32, G.d_f0tab32, G.d_f1tab32,
                    G.d_state, G.d_wcell,
                    G.d_wface[0], G.d_wface[1], G.d_wface[2], G.d_wupd1, G.d_wedge[0], G.d_wedge[1],
                    G.d_wedge[2], G.d_eofs, G.d_edge[0], G.d_edge[1], G.d_edge[2], G.d_wmarch[0], G.d_wmarch[1], G.d_wmarch[2],
                    G.d_gdst, G.d_gsrc, G.d_xoff, G.d_xdat, G.d_ffix, G.d_nbr, G.d_halo,
                    G.d_flux[0], G.d_flux[1], G.d_flux[2], G.d_div};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int q = 0; q < 2; q++) {
        if (G.side[q]) (void)hipStreamDestroy(G.side[q]);
        if (G.ev_join[q]) (void)hipEventDestroy(G.ev_join[q]);
        G.side[q] = nullptr;
        G.ev_join[q] = nullptr;
    }
    if (G.ev_fork) (void)hipEventDestroy(G.ev_fork);
    G.ev_fork = nullptr;
}

int check_grid(bhac_grid *g)
{
    if (!g) return fail(BHAC_EINVAL, "null grid");
    return BHAC_OK;
}

// ---------------------------------------------------------------------------------
// Static face-flux scratch of bhac_substep_noalloc: one array per GPU, resident until
// the process ends. Host code never uses the array's name as an address (on the host
// it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, taken once per device (in bhac_alloc_blocks, with that device
// current) and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------------
constexpr size_t kScratchBytes = sizeof(scratch);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's array (looked up on its first request)
int scratch_of_device(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(BHAC_EDEVICE, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(BHAC_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return BHAC_OK;
}

// argument checks shared by bhac_substep and bhac_substep_noalloc
int check_substep(bhac_grid *g, const double *U_base, const double *U_stage, const void *P_stage,
                  const double *U_out, const void *P_out, double a, double b)
{
    if (int rc = check_grid(g)) return rc;
    if (!U_base || !U_stage || !P_stage || !U_out || !P_out) return fail(BHAC_EINVAL, "null array");
    if (P_out == P_stage) return fail(BHAC_EALIAS, "P_out aliases P_stage");
    if ((const void *)U_out == P_stage || (const void *)U_out == P_out || (const void *)U_base == P_out ||
        (const void *)U_stage == P_out)
        return fail(BHAC_EALIAS, "a conserved array aliases a primitive array");
    if (!(a >= 0.0) || !(b > 0.0)) return fail(BHAC_EINVAL, "need a >= 0 and b > 0");
    if (!g->dg.have_dt) return fail(BHAC_EINVAL, "time step not initialised: call bhac_compute_dt or bhac_set_dt");
    return BHAC_OK;
}

}  // namespace

extern "C" {

const char *bhac_last_error(void) { return g_err.c_str(); }

int bhac_plan_ghosts(const bhac_params *params, const bhac_block_desc *blocks, int64_t nblocks, int64_t *block_offset,
                     int64_t *nslots, int32_t *dst, int32_t *src)
{
    try {
        bhac::Plan P;
        std::string err;
        const int rc = bhac::make_plan(params, blocks, nblocks, false, P, err);
        if (rc != BHAC_OK) return fail(rc, err);
        if (block_offset) std::memcpy(block_offset, P.off.data(), P.off.size() * sizeof(int64_t));
        if (nslots) *nslots = (int64_t)P.gdst.size();
        if (dst) std::memcpy(dst, P.gdst.data(), P.gdst.size() * sizeof(int32_t));
        if (src) std::memcpy(src, P.gsrc.data(), P.gsrc.size() * sizeof(int32_t));
        return BHAC_OK;
    } catch (const std::bad_alloc &) {
        return fail(BHAC_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(BHAC_EINVAL, "planning failed");
    }
}

int bhac_alloc_blocks(const bhac_params *params, const bhac_block_desc *blocks, int64_t nblocks, bhac_grid **out,
                      bhac_layout *layout)
{
    if (!out) return fail(BHAC_EINVAL, "null output handle");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(BHAC_EDEVICE, "no HIP device available");
    bhac_grid *g = nullptr;
    try {
        g = new bhac_grid();
    } catch (...) {
        return fail(BHAC_ENOMEM, "host allocation failed");
    }
    bhac::DeviceGrid &G = g->dg;
    try {
        std::string err;
        const int rc = bhac::make_plan(params, blocks, nblocks, true, G.plan, err);
        if (rc != BHAC_OK) {
            delete g;
            return fail(rc, err);
        }
    } catch (const std::bad_alloc &) {
        delete g;
        return fail(BHAC_ENOMEM, "host allocation failed");
    }
    if (params->fused) {
        const bhac::Plan &Q = G.plan;
        const char *why = nullptr;
        if (params->ndim != 3) why = "the block-tiled substep needs ndim = 3";
        else if (params->precision != BHAC_PREC_MIXED) why = "the block-tiled substep runs in mixed precision only";
        else if (params->recon != BHAC_RECON_PPM) why = "the block-tiled substep implements PPM reconstruction only";
        else if (params->nghost != 3) why = "the block-tiled substep needs nghost = 3";
        else if (Q.smax[0] > 16 || Q.smax[1] > 16) why = "the block-tiled substep needs block sizes <= 16 along x1 and x2";
        if (why) {
            delete g;
            return fail(BHAC_EUNSUPPORTED, why);
        }
    }
    const bhac::Plan &P = G.plan;
    const bhac_params &p = P.p;
    (void)hipGetDevice(&G.device);
    {
        // set-up of the static scratch of bhac_substep_noalloc on this device
        void *unused = nullptr;
        if (int rc = scratch_of_device(G.device, &unused)) {
            delete g;
            return rc;
        }
    }
    G.ks = p.metric == BHAC_METRIC_KS_SPH_LOGR;
    G.mixed = p.precision == BHAC_PREC_MIXED;
    bhac::KParams &kp = G.kp;
    kp.gam = p.gamma_ad;
    kp.gfac = p.gamma_ad / (p.gamma_ad - 1.0);
    kp.gfac_inv = (p.gamma_ad - 1.0) / p.gamma_ad;
    kp.rho_floor = p.rho_floor;
    kp.p_floor = p.p_floor;
    kp.w_max = p.w_max;
    kp.c2p_tol = p.c2p_tol;
    kp.c2p_maxit = p.c2p_maxit;
    kp.cfl = p.cfl;
    kp.glm_alpha = p.glm_alpha;
    kp.ndim = p.ndim;
    kp.recon = p.recon;
    kp.flux = p.flux;
    kp.nvar = bhac::NV + (p.entropy ? 1 : 0);
    for (int d = 0; d < 3; d++) kp.g[d] = P.gd[d];
    kp.ncp = P.off.back();
    kp.nci = P.ncell_interior;
    const bhac::DevLevel &fine = P.levels[P.maxlevel];
    kp.sinv_fine = 0.0;
    kp.dmin_fine = 1e300;
    for (int d = 0; d < 3; d++) kp.inv_dx_fine[d] = 0.0;
    for (int d = 0; d < p.ndim; d++) {
        kp.sinv_fine += 1.0 / fine.dx[d];
        kp.dmin_fine = fine.dx[d] < kp.dmin_fine ? fine.dx[d] : kp.dmin_fine;
        kp.inv_dx_fine[d] = 1.0 / fine.dx[d];
    }

#define UP(dst, vec)                                                    \
    do {                                                                \
        e = upload(&(dst), (vec).data(), (vec).size());                 \
        if (e != hipSuccess) goto hip_error;                            \
    } while (0)
    UP(G.d_blocks, P.dblocks);
    UP(G.d_levels, P.levels);
    UP(G.d_ctab, P.ctab);
    UP(G.d_f0tab, P.f0tab);
    UP(G.d_f1tab, P.f1tab);
    UP(G.d_ctab32, P.ctab32);
    UP(G.d_f0tab32, P.f0tab32);
    UP(G.d_f1tab32, P.f1tab32);
    UP(G.d_wcell, P.wcell);
    for (int d = 0; d < 3; d++) UP(G.d_wface[d], P.wface[d]);
    UP(G.d_wupd1, P.wupd1);
    for (int K = 0; K < 3; K++) UP(G.d_wedge[K], P.wedge[K]);
    UP(G.d_eofs, P.eofs);
    for (int d = 0; d < 3; d++) UP(G.d_wmarch[d], P.wmarch[d]);
    UP(G.d_gdst, P.gdst);
    UP(G.d_gsrc, P.gsrc);
    UP(G.d_xoff, P.xoff);
    UP(G.d_xdat, P.xdat);
    UP(G.d_ffix, P.ffix);
    UP(G.d_nbr, P.nbr);
    UP(G.d_halo, P.halo);
#undef UP
    G.nghost_slots = (long long)P.gdst.size();
    G.nface_slots = P.nface_slots;
    G.nxl = P.xoff.empty() ? 0 : (long long)P.xoff.size() - 1;
    G.nxl_face = P.nxl_face;
    G.nffix = (long long)P.ffix.size() / 6;
    {
        const size_t rsz = G.mixed ? sizeof(float) : sizeof(double);
        for (int d = 0; d < p.ndim && !p.fused; d++) {
            e = hipMalloc(&G.d_flux[d], (size_t)G.kp.nvar * P.nface[d] * rsz);
            if (e != hipSuccess) goto hip_error;
        }
        for (int K = 0; K < 3; K++)
            if (P.nedge[K] > 0) {
                e = hipMalloc((void **)&G.d_edge[K], (size_t)P.nedge[K] * sizeof(double));
                if (e != hipSuccess) goto hip_error;
            }
        if (p.fused) {
            e = hipMalloc(&G.d_div, (size_t)bhac::NV * P.ncell_interior * sizeof(float));
            if (e != hipSuccess) goto hip_error;
        }
        e = hipMalloc((void **)&G.d_state, sizeof(bhac::DevState));
        if (e != hipSuccess) goto hip_error;
        e = hipMemset(G.d_state, 0, sizeof(bhac::DevState));
        if (e != hipSuccess) goto hip_error;
        e = hipDeviceSynchronize();
        if (e != hipSuccess) goto hip_error;
    }
    G.gd.blocks = G.d_blocks;
    G.gd.levels = G.d_levels;
    G.gd.ctab = G.d_ctab;
    G.gd.f0tab = G.d_f0tab;
    G.gd.f1tab = G.d_f1tab;
    G.gd.ctab32 = G.d_ctab32;
    G.gd.f0tab32 = G.d_f0tab32;
    G.gd.f1tab32 = G.d_f1tab32;
    G.gd.nrec_c = P.nrec_c;
    G.gd.nrec_f0 = P.nrec_f0;
    G.gd.nrec_f1 = P.nrec_f1;
    G.gd.st = G.d_state;
    G.gd.nbr = G.d_nbr;
    G.gd.halo = G.d_halo;
    G.gd.hmax = P.hmax;
    for (int q = 0; q < 2; q++) {
        e = hipStreamCreateWithFlags(&G.side[q], hipStreamNonBlocking);
        if (e != hipSuccess) goto hip_error;
        e = hipEventCreateWithFlags(&G.ev_join[q], hipEventDisableTiming);
        if (e != hipSuccess) goto hip_error;
    }
    e = hipEventCreateWithFlags(&G.ev_fork, hipEventDisableTiming);
    if (e != hipSuccess) goto hip_error;
    if (layout) {
        layout->ncell_padded = P.off.back();
        layout->ncell_interior = P.ncell_interior;
        layout->nvar = G.kp.nvar;
        layout->nghost = p.nghost;
        layout->block_offset = P.off.data();
        layout->block_interior_offset = P.ioff.data();
    }
    *out = g;
    return BHAC_OK;
hip_error:
    {
        const int rc = e == hipErrorOutOfMemory ? fail(BHAC_ENOMEM, "device allocation failed")
                                                : hip_fail(e, "bhac_alloc_blocks");
        release(G);
        delete g;
        return rc;
    }
}

static void release_graph(bhac_grid *g)
{
    if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->graph_exec = nullptr;
    g->graph = nullptr;
}

int bhac_free_blocks(bhac_grid *g)
{
    if (!g) return BHAC_OK;
    (void)hipDeviceSynchronize();
    release_graph(g);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    release(g->dg);
    delete g;
    return BHAC_OK;
}

int bhac_fill_ghosts(bhac_grid *g, void *prim, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!prim) return fail(BHAC_EINVAL, "null prim");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_fill(g->dg, prim, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_fill_ghosts");
}

int bhac_fill_ghost_faces(bhac_grid *g, void *prim, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!prim) return fail(BHAC_EINVAL, "null prim");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_fill(g->dg, prim, (hipStream_t)stream, true);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_fill_ghost_faces");
}

int bhac_prim2con(bhac_grid *g, const void *prim, double *cons, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!prim || !cons) return fail(BHAC_EINVAL, "null array");
    if ((const void *)cons == prim) return fail(BHAC_EALIAS, "cons aliases prim");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_prim2con(g->dg, prim, cons, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_prim2con");
}

int bhac_con2prim(bhac_grid *g, const double *cons, void *prim_inout, int8_t *failflags, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!prim_inout || !cons) return fail(BHAC_EINVAL, "null array");
    if ((const void *)cons == prim_inout) return fail(BHAC_EALIAS, "cons aliases prim");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_con2prim(g->dg, cons, prim_inout, failflags, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_con2prim");
}

int bhac_substep(bhac_grid *g, const double *U_base, const double *U_stage, const void *P_stage, double *U_out,
                 void *P_out, double a, double b, void *stream)
{
    if (int rc = check_substep(g, U_base, U_stage, P_stage, U_out, P_out, a, b)) return rc;
    if (g->dg.plan.p.ct) return fail(BHAC_EINVAL, "the grid uses constrained transport: call bhac_substep_ct");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_substep(g->dg, U_base, U_stage, P_stage, U_out, P_out, a, b, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_substep");
}

int bhac_substep_ct(bhac_grid *g, const double *U_base, const double *U_stage, const void *P_stage,
                    const double *phi_base, const double *phi_stage, double *U_out, void *P_out, double *phi_out,
                    double a, double b, void *stream)
{
    if (int rc = check_substep(g, U_base, U_stage, P_stage, U_out, P_out, a, b)) return rc;
    if (!g->dg.plan.p.ct) return fail(BHAC_EINVAL, "bhac_substep_ct needs a grid with ct = 1");
    if (!phi_base || !phi_stage || !phi_out) return fail(BHAC_EINVAL, "null face field");
    const void *u[] = {U_base, U_stage, U_out}, *pr[] = {P_stage, P_out};
    for (const void *f : {(const void *)phi_base, (const void *)phi_stage, (const void *)phi_out}) {
        for (const void *x : u)
            if (x == f) return fail(BHAC_EALIAS, "a face field aliases a conserved array");
        for (const void *x : pr)
            if (x == f) return fail(BHAC_EALIAS, "a face field aliases a primitive array");
    }
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_substep_ct(g->dg, U_base, U_stage, P_stage, phi_base, phi_stage, U_out, P_out, phi_out, a,
                                           b, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_substep_ct");
}

int bhac_face_count(bhac_grid *g, int64_t nface[3])
{
    if (int rc = check_grid(g)) return rc;
    if (!nface) return fail(BHAC_EINVAL, "null output");
    for (int d = 0; d < 3; d++) nface[d] = d < g->dg.kp.ndim ? (int64_t)g->dg.plan.nface[d] : 0;
    return BHAC_OK;
}

int bhac_ct_center(bhac_grid *g, const double *phi, void *prim, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!phi || !prim) return fail(BHAC_EINVAL, "null array");
    if ((const void *)phi == prim) return fail(BHAC_EALIAS, "phi aliases prim");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_ct_center(g->dg, phi, prim, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_ct_center");
}

int bhac_ct_divergence(bhac_grid *g, const double *phi, double *div, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!phi || !div) return fail(BHAC_EINVAL, "null array");
    if (phi == div) return fail(BHAC_EALIAS, "div aliases phi");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_ct_div(g->dg, phi, div, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_ct_divergence");
}

int bhac_substep_noalloc(bhac_grid *g, const double *U_base, const double *U_stage, const void *P_stage,
                         double *U_out, void *P_out, double a, double b, void *stream)
{
    if (int rc = check_substep(g, U_base, U_stage, P_stage, U_out, P_out, a, b)) return rc;
    const bhac::DeviceGrid &G = g->dg;
    if (G.plan.p.fused) return fail(BHAC_EUNSUPPORTED, "bhac_substep_noalloc runs the unfused substep (fused = 0) only");
    if (G.plan.p.ct) return fail(BHAC_EUNSUPPORTED, "bhac_substep_noalloc does not run constrained transport");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != G.device)
        return fail(BHAC_EINVAL, "bhac_substep_noalloc: the grid's device is not the current device");
    // the three face-flux arrays, each starting on a 256-byte boundary
    const size_t rsz = G.mixed ? sizeof(float) : sizeof(double);
    size_t offs[3] = {0, 0, 0}, need = 0;
    for (int d = 0; d < G.kp.ndim; d++) {
        offs[d] = need;
        need += ((size_t)G.kp.nvar * (size_t)G.plan.nface[d] * rsz + 255) / 256 * 256;
    }
    if (need > kScratchBytes)
        return fail(BHAC_EINVAL, "bhac_substep_noalloc: the grid's face fluxes need " + std::to_string(need) +
                                     " bytes, beyond the static scratch of " + std::to_string(kScratchBytes) +
                                     " bytes; use bhac_substep");
    void *base = nullptr;
    if (int rc = scratch_of_device(dev, &base)) return rc;
    void *flux[3] = {nullptr, nullptr, nullptr};
    for (int d = 0; d < G.kp.ndim; d++) flux[d] = (unsigned char *)base + offs[d];
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_substep(G, U_base, U_stage, P_stage, U_out, P_out, a, b, (hipStream_t)stream, flux);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_substep_noalloc");
}

int bhac_compute_dt(bhac_grid *g, const void *prim, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!prim) return fail(BHAC_EINVAL, "null prim");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_compute_dt(g->dg, prim, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "bhac_compute_dt");
    g->dg.have_dt = true;
    return BHAC_OK;
}

int bhac_set_dt(bhac_grid *g, double dt, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!(dt >= 0.0)) return fail(BHAC_EINVAL, "dt must be >= 0");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_set_dt(g->dg, dt, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "bhac_set_dt");
    if (dt > 0.0) g->dg.have_dt = true;
    return BHAC_OK;
}

static int read_state(bhac_grid *g, bhac::DevState &st)
{
    hipError_t e = bhac::launch_finish_step(g->dg, g->last_stream);
    if (e != hipSuccess) return hip_fail(e, "finish step");
    e = hipStreamSynchronize(g->last_stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronise");
    e = hipMemcpy(&st, g->dg.d_state, sizeof st, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "state copy");
    return BHAC_OK;
}

int bhac_get_dt(bhac_grid *g, double *dt_host)
{
    if (int rc = check_grid(g)) return rc;
    if (!dt_host) return fail(BHAC_EINVAL, "null output");
    bhac::DevState st;
    if (int rc = read_state(g, st)) return rc;
    *dt_host = st.dt_next;
    return BHAC_OK;
}

int bhac_get_timestep(bhac_grid *g, bhac_timestep *out)
{
    if (int rc = check_grid(g)) return rc;
    if (!out) return fail(BHAC_EINVAL, "null output");
    bhac::DevState st;
    if (int rc = read_state(g, st)) return rc;
    out->dt = st.dt;
    out->dt_next = st.dt_next;
    out->ch = st.ch;
    out->kappa = st.kappa;
    for (int d = 0; d < 3; d++) out->lam[d] = st.lam_last[d];
    return BHAC_OK;
}

int bhac_get_stats(bhac_grid *g, int64_t *c2p_fail, int64_t *floor_hits, int *max_iter, int64_t *c2p_backup)
{
    if (int rc = check_grid(g)) return rc;
    bhac::DevState st;
    if (int rc = read_state(g, st)) return rc;
    if (c2p_fail) *c2p_fail = (int64_t)st.c2p_fail;
    if (floor_hits) *floor_hits = (int64_t)st.floor_hits;
    if (max_iter) *max_iter = st.max_iter;
    if (c2p_backup) *c2p_backup = (int64_t)st.c2p_backup;
    return BHAC_OK;
}

int bhac_get_schedule(bhac_grid *g, bhac_schedule *out)
{
    if (int rc = check_grid(g)) return rc;
    if (!out) return fail(BHAC_EINVAL, "null output");
    const bhac::Plan &P = g->dg.plan;
    out->set = 1;
    out->march_mask = P.march_mask;
    out->march_faces = P.march_faces;
    out->x1_staged = P.x1_in_update ? 2 : (P.x1_staged ? 1 : 0);
    return BHAC_OK;
}

// Records the two substeps that `record` launches on a stream the grid owns into the
// grid's step graph (replacing any previous one) and instantiates it.
extern "C++" {
template <typename Rec>
static int capture_step(bhac_grid *g, Rec record, const char *what)
{
    if (!g->dg.have_dt) return fail(BHAC_EINVAL, "time step not initialised: call bhac_compute_dt or bhac_set_dt");
    hipError_t e;
    if (!g->cap_stream) {
        e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "capture stream");
    }
    // work queued earlier on other streams must not race the capture's own launches
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, what);
    release_graph(g);
    const bool timing = g->dg.timer.on;
    g->dg.timer.on = false;                 // no event records inside the graph
    hipStream_t s = g->cap_stream;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        g->dg.timer.on = timing;
        return hip_fail(e, "hipStreamBeginCapture");
    }
    // every substep reads its halo cells from the neighbouring blocks' interiors,
    // so the step needs no ghost fill
    hipError_t le = record(s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    g->dg.timer.on = timing;
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "capture of the RK2 step");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    g->graph = graph;
    e = hipGraphInstantiate(&g->graph_exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        release_graph(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    return BHAC_OK;
}
}  // extern "C++"

int bhac_capture_rk2_step(bhac_grid *g, double *U, void *P, double *U1, void *P1)
{
    if (int rc = check_grid(g)) return rc;
    if (!U || !P || !U1 || !P1) return fail(BHAC_EINVAL, "null array");
    if (P == P1 || (void *)U == (void *)U1) return fail(BHAC_EALIAS, "stage buffers must differ");
    if (g->dg.plan.p.ct) return fail(BHAC_EUNSUPPORTED, "constrained transport: use bhac_capture_rk2_step_ct");
    return capture_step(
        g,
        [&](hipStream_t s) {
            hipError_t le = bhac::launch_substep(g->dg, U, U, P, U1, P1, 0.0, 1.0, s);
            if (le == hipSuccess) le = bhac::launch_substep(g->dg, U, U1, P1, U, P, 0.5, 0.5, s);
            return le;
        },
        "bhac_capture_rk2_step");
}

int bhac_capture_rk2_step_ct(bhac_grid *g, double *U, void *P, double *U1, void *P1, double *phi, double *phi1)
{
    if (int rc = check_grid(g)) return rc;
    if (!g->dg.plan.p.ct) return fail(BHAC_EINVAL, "bhac_capture_rk2_step_ct needs a grid with ct = 1");
    if (!U || !P || !U1 || !P1 || !phi || !phi1) return fail(BHAC_EINVAL, "null array");
    if (P == P1 || (void *)U == (void *)U1 || phi == phi1) return fail(BHAC_EALIAS, "stage buffers must differ");
    const void *st[] = {U, P, U1, P1};
    for (const void *f : {(const void *)phi, (const void *)phi1})
        for (const void *x : st)
            if (x == f) return fail(BHAC_EALIAS, "a face field aliases a state array");
    return capture_step(
        g,
        [&](hipStream_t s) {
            hipError_t le = bhac::launch_substep_ct(g->dg, U, U, P, phi, phi, U1, P1, phi1, 0.0, 1.0, s);
            if (le == hipSuccess) le = bhac::launch_substep_ct(g->dg, U, U1, P1, phi, phi1, U, P, phi, 0.5, 0.5, s);
            return le;
        },
        "bhac_capture_rk2_step_ct");
}

int bhac_launch_rk2_step(bhac_grid *g, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    if (!g->graph_exec) return fail(BHAC_EINVAL, "no captured RK2 step");
    g->last_stream = (hipStream_t)stream;
    hipError_t e = hipGraphLaunch(g->graph_exec, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "hipGraphLaunch");
}

int bhac_set_timing(bhac_grid *g, int enable)
{
    if (int rc = check_grid(g)) return rc;
    bhac::KTimer &t = g->dg.timer;
    if (enable && t.pool.empty()) {
        const size_t n = 16384;
        t.pool.reserve(n);
        t.recs.reserve(n / 2);
        for (size_t i = 0; i < n; i++) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) {
                release_timer(g->dg);
                return hip_fail(err, "bhac_set_timing");
            }
            t.pool.push_back(e);
        }
    }
    t.on = enable != 0;
    return BHAC_OK;
}

int bhac_get_timing(bhac_grid *g, bhac_kernel_time *out, int max_entries, int *n_entries)
{
    if (int rc = check_grid(g)) return rc;
    bhac::KTimer &t = g->dg.timer;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "bhac_get_timing");
    for (const auto &r : t.recs) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        t.total_ms[r.id] += ms;
        t.launches[r.id] += 1;
    }
    t.recs.clear();
    t.used = 0;
    int n = 0;
    for (int k = 0; k < bhac::K_COUNT; k++) {
        if (t.launches[k] == 0) continue;
        if (out && n < max_entries) out[n] = bhac_kernel_time{bhac::kKernelNames[k], t.launches[k], t.total_ms[k]};
        n++;
    }
    if (t.dropped) {
        if (out && n < max_entries) out[n] = bhac_kernel_time{"untimed", t.dropped, 0.0};
        n++;
    }
    for (int k = 0; k < bhac::K_COUNT; k++) { t.total_ms[k] = 0.0; t.launches[k] = 0; }
    t.dropped = 0;
    if (n_entries) *n_entries = n;
    return BHAC_OK;
}

int bhac_reset_stats(bhac_grid *g, void *stream)
{
    if (int rc = check_grid(g)) return rc;
    g->last_stream = (hipStream_t)stream;
    hipError_t e = bhac::launch_reset_stats(g->dg, (hipStream_t)stream);
    return e == hipSuccess ? BHAC_OK : hip_fail(e, "bhac_reset_stats");
}

}  // extern "C"
