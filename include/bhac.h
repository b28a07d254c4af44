/*
 * bhac.h -- C ABI of the MI355X (gfx950) GRMHD substep library.
 *
 * The library advances the ideal-GRMHD equations on a list of logically
 * Cartesian blocks with ghost layers by one Runge-Kutta substep at a time. The
 * paper's Section 2 ("Code overview") lists the method: a high-resolution
 * shock-capturing finite-volume scheme in covariant coordinates on block-based
 * grids, second-order time stepping, second- or third-order (PPM) reconstruction
 * and a Newton-Raphson conserved-to-primitive inversion with backups. Section 4.2
 * counts the work as substeps times cells ("cellupdates"); Section 4.3 names the
 * same-level ghost-cell fill; Section 5.1 the ghost-cell exchange. The formulas
 * the paper does not print follow the standard 3+1 form of GRMHD (described with
 * each call).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Return value: BHAC_OK (0) or a negative BHAC_E* code; bhac_last_error()
 *    gives a message (thread-local). No call throws. Numerical trouble inside a
 *    cell (an inversion that does not converge) is not an error: it is flagged
 *    and counted (bhac_get_stats).
 *  - Device calls are asynchronous on the caller's HIP stream (`stream` is a
 *    hipStream_t; NULL means the default stream). Only bhac_get_dt,
 *    bhac_get_timestep and bhac_get_stats synchronise that stream.
 *  - Ownership: the caller owns every state array (device pointers, e.g. from
 *    PyTorch). The library owns the grid metadata (ghost maps, metric tables,
 *    work lists, time-step state, counters); bhac_alloc_blocks allocates it and
 *    bhac_free_blocks releases it. No per-substep call allocates memory.
 *  - State layout (structure of arrays, 9 rows). Primitives P: rows rho, u~1,
 *    u~2, u~3 (Lorentz factor times Eulerian 3-velocity, contravariant), p, B1,
 *    B2, B3 (Eulerian magnetic field), psi (GLM scalar); each row has
 *    ncell_padded entries and block b occupies [block_offset[b],
 *    block_offset[b+1]): first its interior cells, x fastest, then y, then z
 *    (as in U), then the ghost slots of its (size + 2g) box (g ghost layers on
 *    each side of every axis in use; for ndim = 2 the z extent is 1 with no
 *    ghosts) in box order, x fastest, the interior skipped; the region is
 *    rounded up to a multiple of 32 slots. With a 128-byte aligned state
 *    pointer every block starts on a 128-byte line and consecutive interior
 *    rows fill whole lines. The slots after a block's ghost slots are padding
 *    that no call reads or writes. Conserved U: rows
 *    sqrt(gamma) * (D, S_1, S_2, S_3, tau, B1, B2, B3), psi; conserved variables
 *    need no ghost cells, so each row has ncell_interior entries and block b
 *    occupies [block_interior_offset[b], block_interior_offset[b+1]), x fastest.
 *    With the entropy field (entropy = 1) both carry a tenth row: P row 9 is the
 *    entropy function K (p / rho^gamma where it was last consistent), U row 9 is
 *    U row 0 times K. bhac_layout.nvar gives the row count (9 or 10); every
 *    "[9]" below then reads "[10]".
 *  - Precision: P is double when precision == BHAC_PREC_FP64 and float when
 *    precision == BHAC_PREC_MIXED. U is always double.
 */
#ifndef BHAC_H
#define BHAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BHAC_OK = 0,
    BHAC_EINVAL = -1,       /* invalid argument or block list */
    BHAC_ENOMEM = -2,       /* device or host allocation failed */
    BHAC_EDEVICE = -3,      /* no usable GPU, or a HIP runtime error */
    BHAC_EALIAS = -4,       /* an output aliases an input it must not alias */
    BHAC_EUNSUPPORTED = -5  /* a valid combination the library does not implement */
};
enum { BHAC_METRIC_MINKOWSKI_CART = 0, BHAC_METRIC_KS_SPH_LOGR = 1 };
enum { BHAC_BC_PERIODIC = 0, BHAC_BC_OUTFLOW = 1 };
enum { BHAC_RECON_MC = 0, BHAC_RECON_PPM = 1 };
enum { BHAC_FLUX_HLL = 0, BHAC_FLUX_TVDLF = 1 };
enum { BHAC_PREC_FP64 = 0, BHAC_PREC_MIXED = 1 };

/* Problem definition. Units G = c = M = 1.
 *  metric  BHAC_METRIC_MINKOWSKI_CART: flat space, Cartesian (x, y, z).
 *          BHAC_METRIC_KS_SPH_LOGR: stationary Kerr-Schild spacetime of spin
 *          `spin` in coordinates (ln r, theta, phi) (Section 2: any covariant
 *          coordinate system).
 *  x_lo, x_hi, ncell0   level-0 domain and cells per axis; level l has
 *          ncell0 * 2^l cells per axis.
 *  bc[d][side]          BHAC_BC_PERIODIC (both sides) or BHAC_BC_OUTFLOW.
 *  recon, flux          MC or PPM reconstruction (Section 2); HLL or TVDLF flux.
 *  precision            BHAC_PREC_FP64: everything in double.
 *                       BHAC_PREC_MIXED: P stored in float; reconstruction, face
 *                       fluxes and their divergence in float; metric, sources,
 *                       the RK accumulation (compensated) and the inversion in
 *                       double.
 *  fused                0: one kernel per direction computes the face fluxes,
 *                       one kernel per cell the update.
 *                       1: a block-tiled kernel per substep stages each block
 *                       with its halo in LDS, then the per-cell update.
 *                       Either way bhac_substep reads the halo of a block from
 *                       its neighbours' interior cells, by the rule of
 *                       bhac_fill_ghosts, and no ghost slot of P_stage.
 *  cfl                  Courant number C of dt = C / sum_d (lambda_d / dx_d).
 *  rho_floor, p_floor, w_max   floors applied after a converged inversion.
 *  glm_alpha            GLM damping: kappa = glm_alpha * c_h / min_d dx_d.
 *  c2p_tol, c2p_maxit   Newton stopping tolerance on |dxi|/xi and iteration cap.
 *  amr                  0: the blocks are independent patches; a block's halo comes
 *                       from blocks of its own (level, size) only.
 *                       1: the blocks are the leaves of a 2:1-balanced block tree
 *                       (Section 2's block-based adaptive mesh): one block size,
 *                       even and >= 2 * nghost along every axis in use (so every
 *                       ghost layer lies in a leaf adjacent to the block), no
 *                       leaf inside another;
 *                       where a block borders coarser or finer leaves its ghost
 *                       cells come from prolongation or restriction (see
 *                       bhac_fill_ghosts). Needs fused = 0 (else
 *                       BHAC_EUNSUPPORTED).
 *  entropy              0: nine variables. 1: also carry the entropy field K and
 *                       use it as the backup of the inversion (Section 2 names
 *                       backup strategies; see bhac_con2prim). K is transported
 *                       as rho W K, its face flux the mass flux times K
 *                       reconstructed on the upwind side, with no source. Needs
 *                       gamma_ad <= 2 (else BHAC_EINVAL), fused = 0 and amr = 0
 *                       (else BHAC_EUNSUPPORTED).
 *  sched                kernel schedule of the unfused substep (see bhac_schedule).
 *  ct                   0: divergence cleaning (GLM: the normal field of a face from
 *                       the exact (B~, psi) solve, psi damped). 1: staggered-mesh
 *                       constrained transport (Section 2: the paper's code evolves the
 *                       field by constrained transport on a staggered mesh): the field
 *                       is carried as face fluxes phi^d = sqrt(gamma) B^d and advanced
 *                       by bhac_substep_ct. Needs fused = 0, amr = 0 and entropy = 0
 *                       (else BHAC_EUNSUPPORTED). The face fluxes follow the schedule
 *                       as in the GLM substep (the x1 faces are never computed inside
 *                       the update under constrained transport).
 */

/* Schedule of the unfused substep (fused = 0; the block-tiled path ignores it).
 * Every schedule computes the same face fluxes by the same per-face arithmetic
 * (Section 2's reconstruction and Riemann solver); only the mapping of work onto
 * waves differs, so a schedule is a tuning choice, not a change of method.
 *  set          0: the library's defaults, the other fields are ignored.
 *  march_mask   bit d set: the fluxes along direction d come from the line-march
 *               kernel (one thread walks a line of cells and reconstructs each cell
 *               once); clear: from the face kernel (one thread per face).
 *  march_faces  longest line segment of the march kernel, in faces, 4..256; longer
 *               lines are cut into near-equal segments, each with its own warm-up.
 *  x1_staged    how the x1 faces are computed where x1 is not marched. 0: the face
 *               kernel reads cells straight from memory; 1: it stages block rows
 *               with their halo in LDS where every block's rows fit; 2: the update
 *               kernel stages the rows and computes the x1 faces itself, so no x1
 *               flux array is written or read (independent patches without the
 *               entropy field, rows fitting the LDS tile, no constrained transport;
 *               otherwise as 1).
 * Defaults (set = 0): x2 and x3 marched (march_mask 6), segments of 33 faces in mixed
 * precision and 17 in FP64, x1 faces staged in LDS (1) in mixed precision and inside
 * the update (2) in FP64.
 * Out-of-range values give BHAC_EINVAL. */
typedef struct bhac_schedule {
    int set;
    int march_mask;
    int march_faces;
    int x1_staged;
} bhac_schedule;

typedef struct bhac_params {
    int ndim;           /* 2 or 3 */
    int nghost;         /* >= 2 for MC, >= 3 for PPM */
    int metric;
    double spin;
    double gamma_ad;    /* ideal-gas adiabatic index */
    double x_lo[3], x_hi[3];
    int ncell0[3];
    int bc[3][2];
    int recon, flux, precision, fused;
    double cfl, rho_floor, p_floor, w_max, glm_alpha, c2p_tol;
    int c2p_maxit;
    int amr;            /* 0 independent patches, 1 block tree */
    int entropy;        /* 0 nine variables, 1 plus the entropy field (inversion backup) */
    bhac_schedule sched;
    int ct;             /* 0 GLM divergence cleaning, 1 staggered constrained transport */
} bhac_params;

/* One block: refinement level, interior cells per axis, and origin in level-l
 * cells. Blocks of one (level, size) must sit on that size's lattice
 * (origin % size == 0) and must not overlap. */
typedef struct bhac_block_desc {
    int level;
    int size[3];
    int origin[3];
} bhac_block_desc;

/* Layout of the state arrays, filled by bhac_alloc_blocks. block_offset (padded
 * primitive rows) and block_interior_offset (conserved rows) point to nblocks + 1
 * host entries owned by the grid (valid until bhac_free_blocks). */
typedef struct bhac_layout {
    int64_t ncell_padded;
    int64_t ncell_interior;
    int nvar;
    int nghost;
    const int64_t *block_offset;
    const int64_t *block_interior_offset;
} bhac_layout;

/* Time-step state as the device holds it. dt, ch and kappa belong to the step in
 * progress; dt_next is what the next step will use; lam[d] is the largest
 * |characteristic speed| along d seen by the last finished substep. */
typedef struct bhac_timestep {
    double dt, dt_next, ch, kappa;
    double lam[3];
} bhac_timestep;

typedef struct bhac_grid bhac_grid;

/* Build a grid on the current HIP device (Sections 2 and 4.3: blocks of cells
 * with ghost layers). Validates the parameters and the block list, builds the
 * same-level ghost gather map, the block neighbour tables, the FP64 metric
 * tables and the work lists, copies them to the device and returns the handle
 * and the state layout. Host-side cost is O(number of ghost cells).
 * Errors: BHAC_EINVAL (bad params or blocks; *out untouched), BHAC_ENOMEM,
 * BHAC_EDEVICE. */
int bhac_alloc_blocks(const bhac_params *params, const bhac_block_desc *blocks, int64_t nblocks,
                      bhac_grid **out, bhac_layout *layout);

/* Release the grid and its device memory (synchronises the device). NULL is a no-op. */
int bhac_free_blocks(bhac_grid *grid);

/* Ghost-cell fill (Section 4.3's same-refinement-level fill; with amr = 1 also
 * the exchange between refinement levels of Section 2's block-based mesh).
 * Rule per ghost slot at global level-l index G: wrap periodic axes, clamp
 * outflow axes to the domain; if a block of the same level and size holds that
 * cell, copy it bit for bit (all 9 primitives). Otherwise, with amr = 1:
 *   a level-(l+1) leaf holds it: restriction, the mean of the 2^ndim fine cells
 *     under it (summed z-outer, x-inner, times 1/2^ndim);
 *   a level-(l-1) leaf holds it: prolongation, the coarse cell's value q plus,
 *     for each axis d in order, +1/4 (upper half of the coarse cell) or -1/4
 *     (lower half) times minmod(q - q_lo, q_hi - q), where q_lo, q_hi are the
 *     coarse block's neighbour cells along d, read from its interior or, outside
 *     it, by this rule without prolongation (a neighbour that would need it
 *     makes that axis's slope zero).
 * Otherwise copy the own block's interior cell nearest to the slot
 * (zero-gradient). Restriction and prolongation are evaluated in double and
 * stored in the state's precision. prim: device, [9][ncell_padded], double or
 * float per precision; written in ghost slots only. */
int bhac_fill_ghosts(bhac_grid *grid, void *prim, void *stream);

/* The same fill restricted to the face-adjacent ghost slabs (slots with exactly
 * one coordinate outside the block): the halo cells that dimension-by-dimension
 * stencils (such as the substep's) read. Edge and corner slots are left as they
 * are. Same arguments and errors as bhac_fill_ghosts. */
int bhac_fill_ghost_faces(bhac_grid *grid, void *prim, void *stream);

/* Primitive -> conserved at interior cells (Section 2's integrated conserved
 * variables): W = sqrt(1 + gamma_ij u~^i u~^j), v^i = u~^i / W,
 * xi = rho h W^2 with h = 1 + Gamma/(Gamma-1) p/rho, D = rho W,
 * S_i = (xi + B^2) v_i - (B.v) B_i, tau = xi + B^2 - p - ((B.v)^2 + B^2/W^2)/2 - D,
 * all densitised by sqrt(gamma); psi copied; with the entropy field U row 9 =
 * U row 0 times P row 9. cons: device double [9][ncell_interior]. */
int bhac_prim2con(bhac_grid *grid, const void *prim, double *cons, void *stream);

/* Conserved -> primitive at interior cells (Section 2: Newton-Raphson with a
 * backup). One-dimensional Newton iteration on xi = rho h W^2 started from the
 * primitives already in prim_inout, safeguarded by halving the step towards the
 * previous iterate while xi <= 0 or v^2 >= 1; stops when |dxi| <= c2p_tol * xi,
 * then takes one more step. Then floors on rho, p and W. On failure (no
 * convergence in c2p_maxit steps, non-finite values, rho <= 0 or p < 0) and
 * with the entropy field carried, the entropy backup: with K = U9 / U0, p = K
 * rho^gamma and rho = D / W, the momentum relation
 *   (xi + B^2)^2 (1 - 1/W^2) - (S.B)^2 (2 xi + B^2) / xi^2 = S^2,
 *   xi = D W + Gamma/(Gamma-1) K D^Gamma W^(2-Gamma),
 * has one root W >= 1 (its left side grows with W); it is found by Newton steps
 * kept inside a bisection bracket, stopping at |dW| <= c2p_tol W, then floors as
 * above; the cell counts as backed up (bhac_get_stats). P row 9 = U9 / U0 on
 * success. If that fails too (or no entropy field is carried) the
 * cell keeps its input primitives and fail[cell] = 1, else 0. cons: device double
 * [9][ncell_interior]; fail: device int8 [ncell_interior], may be NULL. cons is not
 * modified. */
int bhac_con2prim(bhac_grid *grid, const double *cons, void *prim_inout, int8_t *fail, void *stream);

/* One Runge-Kutta substep (Section 2's second-order time stepping; Section 4.2's
 * unit of work): for every interior cell,
 *   U_out = a U_base + b (U_stage + dt L),
 *   L = -sum_d (F_d(i+1/2) - F_d(i-1/2)) / dx_d + S,
 * with F the face fluxes from reconstructed P_stage (MC or PPM), an exact solve
 * of the GLM (B~_normal, psi) subsystem and HLL or TVDLF for the rest, and S the
 * geometric sources of the stationary metric plus GLM damping -kappa psi; then
 * P_out = inversion of U_out started from P_stage (floors, entropy backup and
 * failure as in bhac_con2prim; cells that hit a floor, take the entropy backup or
 * fail get U_out rewritten from P_out). With the entropy field, U row 9 follows
 * the same RK combination with its own face flux and no source. SSP-RK2 is (a, b) = (0, 1) then (1/2, 1/2) with U_stage = U_base in
 * the first stage.
 * Time step: a substep with a == 0 starts a step and latches dt (and c_h, kappa)
 * from the previous substep's wave speeds; every substep records its own maximum
 * |lambda| per direction for the next latch. Call bhac_compute_dt or bhac_set_dt
 * once before the first substep (else BHAC_EINVAL).
 * Aliasing: U_out may alias U_base and/or U_stage; P_out must not alias P_stage
 * (BHAC_EALIAS). The halo cells of each block are read from the neighbouring
 * blocks' interiors (or the own edge cell, where bhac_fill_ghosts would copy
 * that), so the ghost slots of P_stage need not be filled; the ghost slots of
 * P_out are left unchanged. Exception, block trees (amr = 1): where a block
 * borders a coarser or finer leaf, the substep first writes those face-adjacent
 * ghost slots of P_stage by the cross-level rule of bhac_fill_ghosts (from
 * P_stage's interiors) and reads them; P_stage's interior is not modified. A face
 * whose far side lies in finer leaves uses the mean of the 2^(ndim-1) fine face
 * fluxes covering it (flux correction), so D, S, tau and B are conserved across
 * refinement levels. */
int bhac_substep(bhac_grid *grid, const double *U_base, const double *U_stage, const void *P_stage,
                 double *U_out, void *P_out, double a, double b, void *stream);

/* bhac_substep for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same substep
 * with the same kernels and bit-identical results, its face-flux scratch taken from
 * a static device array of 64 MiB that each GPU the library runs on holds until the
 * process ends, instead of the grid's own buffers; the call allocates nothing.
 * Limit: the grid's face fluxes (nvar rows x faces per direction x 4 bytes in mixed
 * precision, 8 in FP64, each direction rounded up to 256 bytes) must fit the 64 MiB
 * (about 80^3 cells in mixed precision, 64^3 in FP64), else BHAC_EINVAL with the
 * sizes in the message; fused = 1 or ct = 1 gives BHAC_EUNSUPPORTED; the grid's device must be
 * the current device (BHAC_EINVAL). Arguments, aliasing rules, time-step handling
 * and other errors as bhac_substep. Every call on one GPU shares that GPU's array and
 * leaves its contents behind; nothing in it has to start at zero (a substep writes
 * every face flux before it reads it). Calls that overlap on one GPU (concurrent
 * streams or host threads) race on the array: serialise them. */
int bhac_substep_noalloc(bhac_grid *grid, const double *U_base, const double *U_stage, const void *P_stage,
                         double *U_out, void *P_out, double a, double b, void *stream);

/* Staggered face field (constrained transport, params.ct = 1). Layout of a face
 * field phi (device double): the arrays of directions 0 .. ndim-1 one after another;
 * direction d holds nface[d] faces, block b's faces from the sum of the earlier
 * blocks' counts, (size_0 + [d == 0]) x (size_1 + [d == 1]) x (size_2 + [d == 2]) of
 * them, x fastest. Every block holds all faces of its cells, so a face between two
 * blocks has one copy in each; the calls keep the copies identical. phi^d is
 * sqrt(gamma) B^d at the centre of the d-face. bhac_face_count returns nface (host). */
int bhac_face_count(bhac_grid *grid, int64_t nface[3]);

/* Cell-centred field from a face field: P rows B^d (d < ndim) = the mean of the
 * cell's two faces of phi^d divided by sqrt(gamma) at the cell centre; the other rows
 * of prim are untouched (with ndim = 2 the x3 field stays the caller's). phi: device
 * double; prim: [nvar][ncell_padded] (interior cells written). */
int bhac_ct_center(bhac_grid *grid, const double *phi, void *prim, void *stream);

/* Discrete divergence of a face field at every interior cell, interior-packed:
 * div = sum_d (phi^d(high face) - phi^d(low face)) / dx_d. div: device double
 * [ncell_interior]. */
int bhac_ct_divergence(bhac_grid *grid, const double *phi, double *div, void *stream);

/* One RK substep under constrained transport (params.ct = 1): as bhac_substep, with
 * the face field advanced in the same combination,
 *   phi_out = a phi_base + b (phi_stage - dt curl E),  d_t phi^i = -(d_j E_k - d_k E_j)
 * ((i, j, k) cyclic), where E_k = F^j(B~^i) = -F^i(B~^j) at each cell edge is the mean
 * of the four induction fluxes of the faces around the edge (a face beyond the block
 * taken from the neighbouring block, or from the block's own nearest face where the
 * halo is zero-gradient). The face fluxes use the face's phi as the normal field of
 * both states (no GLM solve: normal-field and psi fluxes vanish); the cell's
 * densitised field in U_out is the mean of its two updated faces along each resolved
 * direction (with ndim = 2 the x3 field is a cell-centred finite-volume variable). The
 * discrete divergence (bhac_ct_divergence) is kept at its initial value to round-off.
 * phi_base, phi_stage, phi_out: device double in the face layout; phi_out may alias
 * phi_base or phi_stage. Other arguments and errors as bhac_substep; bhac_substep on
 * a grid with ct = 1 gives BHAC_EINVAL. */
int bhac_substep_ct(bhac_grid *grid, const double *U_base, const double *U_stage, const void *P_stage,
                    const double *phi_base, const double *phi_stage, double *U_out, void *P_out, double *phi_out,
                    double a, double b, void *stream);

/* Standalone wave-speed reduction over cell-centred states of prim (interior
 * cells): sets dt_next = C / sum_d (lambda_d / dx_d), dx on the finest level. */
int bhac_compute_dt(bhac_grid *grid, const void *prim, void *stream);

/* dt > 0: every following step uses this fixed dt (and the c_h, kappa that
 * follow from it). dt == 0: back to the CFL time step (which needs a wave-speed
 * reduction first). dt < 0: BHAC_EINVAL. */
int bhac_set_dt(bhac_grid *grid, double dt, void *stream);

/* Host copy of dt_next (synchronises the stream given to the last call). */
int bhac_get_dt(bhac_grid *grid, double *dt_host);

/* Host copy of the whole time-step state (synchronises). */
int bhac_get_timestep(bhac_grid *grid, bhac_timestep *out);

/* Inversion statistics accumulated since alloc or the last reset: failed cells,
 * floored cells, the largest Newton step count and the cells inverted by the
 * entropy backup (synchronises). Any pointer may be NULL. */
int bhac_get_stats(bhac_grid *grid, int64_t *c2p_fail, int64_t *floor_hits, int *max_iter, int64_t *c2p_backup);
int bhac_reset_stats(bhac_grid *grid, void *stream);

/* The schedule the grid's unfused substep runs, defaults resolved (set = 1;
 * x1_staged reads the mode actually used: 2 or 1 only where the grid allows it).
 * Host only. */
int bhac_get_schedule(bhac_grid *grid, bhac_schedule *out);

/* One whole SSP-RK2 step as a HIP graph (the launch-bound inner loop of a run).
 * bhac_capture_rk2_step records, on a stream the grid owns, the kernels of
 *   substep(U, U, P -> U1, P1, 0, 1) -> substep(U, U1, P1 -> U, P, 1/2, 1/2)
 * for these exact buffers, and instantiates it; a new capture replaces the
 * previous graph. bhac_launch_rk2_step replays it on the caller's stream: one
 * call per step, same results as the two calls made one by one. The time-step
 * state lives on the device, so replays need no host work. Needs an initialised
 * time step (BHAC_EINVAL otherwise); P/P1 aliasing rules as for bhac_substep.
 * Launching before a capture returns BHAC_EINVAL; a grid with ct = 1 gives
 * BHAC_EUNSUPPORTED (use bhac_capture_rk2_step_ct). */
int bhac_capture_rk2_step(bhac_grid *grid, double *U, void *P, double *U1, void *P1);
int bhac_launch_rk2_step(bhac_grid *grid, void *stream);

/* The same under constrained transport (params.ct = 1; otherwise BHAC_EINVAL): the
 * graph of
 *   substep_ct(U, U, P, phi, phi -> U1, P1, phi1, 0, 1)
 *   -> substep_ct(U, U1, P1, phi, phi1 -> U, P, phi, 1/2, 1/2)
 * for these exact buffers (phi, phi1: device double in the face layout, distinct
 * from each other and from the state arrays, BHAC_EALIAS otherwise), replayed by
 * bhac_launch_rk2_step. */
int bhac_capture_rk2_step_ct(bhac_grid *grid, double *U, void *P, double *U1, void *P1, double *phi, double *phi1);

/* Optional kernel timing (the measurement behind the roofline figures). While
 * enabled, every kernel the grid launches is bracketed by a pair of HIP events
 * recorded on its launch stream (from a pool created by bhac_set_timing, so no
 * call allocates). bhac_get_timing synchronises, adds the elapsed times per
 * kernel family into out[0..max_entries) (name, launches, total milliseconds;
 * names are static strings), writes the number of families with launches to
 * *n_entries, and restarts the accumulation. Launches beyond the pool are not
 * timed (their count is returned as a family named "untimed"). While timing is
 * enabled the face kernels of a 3-D substep run one after another on the
 * caller's stream (the x2 and x3 line marches as two launches) instead of
 * concurrently on the grid's side streams or as one x2+x3 launch, so each
 * measured duration is the kernel's own (results are the same either way). */
typedef struct bhac_kernel_time {
    const char *name;
    int64_t launches;
    double total_ms;
} bhac_kernel_time;

int bhac_set_timing(bhac_grid *grid, int enable);
int bhac_get_timing(bhac_grid *grid, bhac_kernel_time *out, int max_entries, int *n_entries);

/* Host-only planning, no GPU needed: validates params and blocks and returns
 * the layout offsets (nblocks + 1 entries, may be NULL) and the ghost gather
 * map the library would use: *nslots ghost slots with destination and source
 * padded-cell indices (dst/src may be NULL to query *nslots first). */
int bhac_plan_ghosts(const bhac_params *params, const bhac_block_desc *blocks, int64_t nblocks,
                     int64_t *block_offset, int64_t *nslots, int32_t *dst, int32_t *src);

/* Message of the last failed call on this thread ("" if none). */
const char *bhac_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BHAC_H */
