// Device-side data of one grid and the kernel launchers (HIP).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace bhac {

// Scalars every kernel needs, passed by value.
struct KParams {
    double gam, gfac, gfac_inv;      // Gamma, Gamma/(Gamma-1), (Gamma-1)/Gamma
    double rho_floor, p_floor, w_max, c2p_tol;
    double cfl, glm_alpha;
    double sinv_fine, dmin_fine;     // sum_d 1/dx_d and min_d dx_d on the finest level
    double inv_dx_fine[3];
    long long ncp;                   // padded cells per primitive row
    long long nci;                   // interior cells per conserved row
    int c2p_maxit, ndim;
    int g[3];
    int recon, flux;
    int nvar;                        // rows of P and U: NV, or NV + 1 with the entropy field
};

// Time-step state and counters, resident on the device.
struct DevState {
    double dt, ch, kappa, dt_next, dt_fixed;
    double lam_last[3];
    unsigned long long lam_acc[3];   // bit patterns of non-negative doubles (atomicMax)
    unsigned long long c2p_fail, floor_hits;
    int max_iter;
    int lam_pending;                 // lam_acc holds a finished substep's maxima not yet turned into dt_next
    unsigned long long c2p_backup;   // cells inverted by the entropy backup
};

struct GridDev {
    const DevBlock *blocks;
    const DevLevel *levels;
    const double *ctab, *f0tab, *f1tab;
    const float *ctab32, *f0tab32, *f1tab32;
    long long nrec_c, nrec_f0, nrec_f1;
    DevState *st;
    const int32_t *nbr;              // fused: 27 neighbour ids per block
    const HaloAxis *halo;            // fused: per block and axis
    int hmax;
    int pad;
};

// Kernel families timed by the optional HIP-event timer.
enum KernelId { K_FILL, K_FLUX0, K_FLUX1, K_FLUX2, K_UPDATE, K_PRIM2CON, K_CON2PRIM, K_SPEEDS, K_BEGIN, K_END,
                K_BLOCK_FLUX, K_UPDATE_DIV, K_FILL_XL, K_FLUX_FIX, K_UPDATE_X1, K_CT_FACE, K_CT_EDGE, K_COUNT };
extern const char *const kKernelNames[K_COUNT];

// Optional per-launch timing: a pre-created pool of HIP events recorded on the
// launch stream around every kernel; harvested (with a synchronise) on request.
struct KTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int id; hipEvent_t a, b; hipStream_t s; };
    std::vector<Rec> recs;
    long long dropped = 0;
    double total_ms[K_COUNT] = {};
    long long launches[K_COUNT] = {};
};

// RAII helper: records the pair of events around one kernel launch when timing is on.
struct TimedLaunch {
    KTimer *t;
    int id;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(KTimer &timer, int kid, hipStream_t st) : t(timer.on ? &timer : nullptr), id(kid), s(st)
    {
        if (!t) return;
        if (t->used + 2 > t->pool.size()) { t->dropped++; t = nullptr; return; }
        a = t->pool[t->used++];
        b = t->pool[t->used++];
        (void)hipEventRecord(a, s);
    }
    ~TimedLaunch()
    {
        if (!t) return;
        (void)hipEventRecord(b, s);
        t->recs.push_back({id, a, b, s});
    }
};

struct DeviceGrid {
    Plan plan;
    mutable KTimer timer;
    KParams kp{};
    GridDev gd{};
    int device = 0;
    bool ks = false, mixed = false;
    // owned device buffers
    DevBlock *d_blocks = nullptr;
    DevLevel *d_levels = nullptr;
    double *d_ctab = nullptr, *d_f0tab = nullptr, *d_f1tab = nullptr;
    float *d_ctab32 = nullptr, *d_f0tab32 = nullptr, *d_f1tab32 = nullptr;
    DevState *d_state = nullptr;
    WorkItem *d_wcell = nullptr, *d_wface[3] = {nullptr, nullptr, nullptr}, *d_wupd1 = nullptr;
    MarchItem *d_wmarch[3] = {nullptr, nullptr, nullptr};
    WorkItem *d_wedge[3] = {nullptr, nullptr, nullptr};
    long long *d_eofs = nullptr;                     // constrained transport: edge offsets per block
    double *d_edge[3] = {nullptr, nullptr, nullptr}; // constrained transport: edge fields per direction
    int32_t *d_gdst = nullptr, *d_gsrc = nullptr;
    int32_t *d_xoff = nullptr, *d_xdat = nullptr;    // cross-level recipes (block trees)
    long long nxl = 0, nxl_face = 0;
    int32_t *d_ffix = nullptr;                       // flux correction records (block trees)
    long long nffix = 0;
    int32_t *d_nbr = nullptr;
    HaloAxis *d_halo = nullptr;
    void *d_flux[3] = {nullptr, nullptr, nullptr};   // face-flux scratch of the unfused path
    // owned side streams (default priority) and events: the three face kernels of a
    // substep are independent and run concurrently, forked from and joined back to
    // the caller's stream (a captured graph records the fork and join as edges)
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
    void *d_div = nullptr;                           // flux divergence of the block-tiled path [9][interior]
    long long nghost_slots = 0;
    long long nface_slots = 0;                       // leading slots of the map with one axis outside
    bool have_dt = false;
};

hipError_t launch_fill(const DeviceGrid &G, void *P, hipStream_t s, bool faces_only = false);
hipError_t launch_fill_cross(const DeviceGrid &G, void *P, hipStream_t s, bool faces_only);
hipError_t launch_fill_copies(const DeviceGrid &G, void *P, hipStream_t s, bool faces_only);
hipError_t launch_prim2con(const DeviceGrid &G, const void *P, double *U, hipStream_t s);
hipError_t launch_con2prim(const DeviceGrid &G, const double *U, void *P, int8_t *fail, hipStream_t s);
// turns pending wave-speed maxima into dt_next (before a host read of the state)
hipError_t launch_finish_step(const DeviceGrid &G, hipStream_t s);
hipError_t launch_compute_dt(const DeviceGrid &G, const void *P, hipStream_t s);
hipError_t launch_set_dt(const DeviceGrid &G, double dt, hipStream_t s);
hipError_t launch_reset_stats(const DeviceGrid &G, hipStream_t s);
hipError_t launch_fused_body(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                             void *Po, double a, double b, hipStream_t s);
// phi: the face field of direction D under constrained transport (else nullptr)
hipError_t launch_flux_march(const DeviceGrid &G, int D, const void *Ps, hipStream_t s, void *const *flux,
                             const double *phi = nullptr);
// the x2 and x3 line marches as one launch (both directions marched; independent
// patches without the entropy field, GLM)
hipError_t launch_flux_march_x23(const DeviceGrid &G, const void *Ps, hipStream_t s, void *const *flux);
// flux: the three face-flux arrays of the unfused path (nvar rows x nface[d] faces in
// the state's precision); nullptr = the grid's own (d_flux)
hipError_t launch_substep(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                          void *Po, double a, double b, hipStream_t s, void *const *flux = nullptr);
// constrained transport (plan.p.ct): face fields in the face layout (directions one after another)
hipError_t launch_substep_ct(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, const double *Phb,
                             const double *Phs, double *Uo, void *Po, double *Pho, double a, double b, hipStream_t s);
hipError_t launch_ct_center(const DeviceGrid &G, const double *Ph, void *P, hipStream_t s);
hipError_t launch_ct_div(const DeviceGrid &G, const double *Ph, double *div, hipStream_t s);

}  // namespace bhac
