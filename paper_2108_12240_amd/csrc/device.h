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
    long long ncp;                   // padded cells per state row
    int c2p_maxit, ndim;
    int g[3];
    int recon, flux;
};

// Time-step state and counters, resident on the device.
struct DevState {
    double dt, ch, kappa, dt_next, dt_fixed;
    double lam_last[3];
    unsigned long long lam_acc[3];   // bit patterns of non-negative doubles (atomicMax)
    unsigned long long c2p_fail, floor_hits;
    int max_iter;
    int pad;
};

struct GridDev {
    const DevBlock *blocks;
    const DevLevel *levels;
    const double *ctab, *f0tab, *f1tab;
    long long nrec_c, nrec_f0, nrec_f1;
    DevState *st;
    const int32_t *nbr;              // fused: 27 neighbour ids per block
    const HaloAxis *halo;            // fused: per block and axis
    int hmax;
    int pad;
};

struct DeviceGrid {
    Plan plan;
    KParams kp{};
    GridDev gd{};
    int device = 0;
    bool ks = false, mixed = false;
    // owned device buffers
    DevBlock *d_blocks = nullptr;
    DevLevel *d_levels = nullptr;
    double *d_ctab = nullptr, *d_f0tab = nullptr, *d_f1tab = nullptr;
    DevState *d_state = nullptr;
    WorkItem *d_wcell = nullptr, *d_wface[3] = {nullptr, nullptr, nullptr};
    int32_t *d_gdst = nullptr, *d_gsrc = nullptr;
    int32_t *d_nbr = nullptr;
    HaloAxis *d_halo = nullptr;
    void *d_flux[3] = {nullptr, nullptr, nullptr};   // face-flux scratch of the unfused path
    long long nghost_slots = 0;
    bool have_dt = false;
};

hipError_t launch_fill(const DeviceGrid &G, void *P, hipStream_t s);
hipError_t launch_prim2con(const DeviceGrid &G, const void *P, double *U, hipStream_t s);
hipError_t launch_con2prim(const DeviceGrid &G, const double *U, void *P, int8_t *fail, hipStream_t s);
hipError_t launch_compute_dt(const DeviceGrid &G, const void *P, hipStream_t s);
hipError_t launch_set_dt(const DeviceGrid &G, double dt, hipStream_t s);
hipError_t launch_reset_stats(const DeviceGrid &G, hipStream_t s);
hipError_t launch_substep(const DeviceGrid &G, const double *Ub, const double *Us, const void *Ps, double *Uo,
                          void *Po, double a, double b, hipStream_t s);

}  // namespace bhac
