// Internal declarations of the GRMHD substep library (host planning <-> kernels <-> C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "bhac.h"

namespace bhac {

constexpr int NV = 9;
constexpr int WG = 256;          // work-group size of the unfused kernels (4 wave64)
constexpr int NXCD = 8;          // XCDs of an MI355X; work-groups are dealt to them round-robin

// Per-block description as the kernels see it.
struct DevBlock {
    long long off;               // first padded cell of the block in every state row
    long long fofs[3];           // first face of the block in each direction's face array
    int s[3];                    // interior cells per axis
    int o[3];                    // origin in level cells
    int n0, n1;                  // padded extents along x and y
    int level;
    int hclamp;                  // bit 2e+side: halo of axis e on that side (0 low, 1 high) is the
                                 // block's own edge cell (zero-gradient); else a neighbour's cells
    int hxl;                     // bit 2e+side: that halo lies in a coarser or finer leaf of a block
                                 // tree; the kernels read the block's own ghost slots there (shift 0)
    int pad2;
    long long ioff;              // first interior cell of the block in interior-packed arrays
    long long hshift[3][2];      // added to an own-frame padded index past the low / high end of
                                 // axis e, gives the same cell's padded index in that neighbour
};

// Per-level constants. Metric tables are 2-D in (x1, x2) because both supported
// metrics are independent of x3; records are stored field-major (SoA).
struct DevLevel {
    double dx[3], inv_dx[3];
    long long ctab;              // first record of the centre table of this level
    long long f0tab, f1tab;      // first record of the x1-face and x2-face tables
    int N0, N1;                  // cells along x1 and x2 on this level
    int pad[2];
};

// Centre-table fields. The first C_FACE_NF fields double as the face-table fields.
enum CField {
    C_ALPHA, C_BETA1, C_G11, C_G13, C_G22, C_G33, C_GI11, C_GI13, C_GI22, C_GI33, C_SG,
    C_DA1, C_DA2, C_DB1, C_DB2, C_DG11_1, C_DG11_2, C_DG13_1, C_DG13_2, C_DG22_1, C_DG22_2,
    C_DG33_1, C_DG33_2, C_NF
};
constexpr int C_FACE_NF = C_SG + 1;

struct WorkItem { int block; int start; };

// Line-marching face kernels: a work item is MWG lines of one block (lines along D,
// numbered with the fastest other axis first) and the faces [f0, f1) along D.
constexpr int MWG = 64;
struct MarchItem { int block; int line0; int f0; int f1; };
// Directions whose faces are computed by lines (bit D) and the longest segment a
// line is cut into (a longer line is split into equal segments, each with its own
// warm-up, for parallelism).
// x1 faces with LDS-staged rows: cells one work-group stages at most (rows it
// touches times the padded row length), per precision
template <typename R>
constexpr int x1s_max_cells() { return sizeof(R) == 4 ? 600 : 400; }
// rows of s0 cells one work-group of the update with in-place x1 faces takes: one
// thread per x1 face of the rows (s0 + 1 per row)
constexpr int x1u_rows(int s0) { return WG / (s0 + 1); }
constexpr int MARCH_MASK_F32 = 6;
constexpr int MARCH_MASK_F64 = 6;
// the x1 faces are computed inside the update kernel (sched.x1_staged = 2) by default
// in FP64, where the exhaustive search finds it fastest on the torus grids (-4 % per
// step at 128^3, -3 % at 384^3); in mixed precision it costs 8 % at 384^3, so there
// the staged face kernel is the default
constexpr int X1_IN_UPDATE_DEFAULT_F64 = 2;
constexpr int X1_IN_UPDATE_DEFAULT_F32 = 0;
// default longest march segment, per precision (exhaustive search: 33 is never
// slower in float and 5 % faster on the block tree; 17 is 1 % faster there in FP64)
constexpr int MARCH_FACES_F32 = 33;
constexpr int MARCH_FACES_F64 = 17;
constexpr int MARCH_MAX_FACES = MARCH_FACES_F64;

// Fused-kernel halo addressing: for each block and axis, the source of every
// padded local index l in [-g, s+g): which neighbour direction (-1, 0, +1) its
// lattice slot lies in, and the local index to read there.
struct HaloAxis { signed char dir; signed char pad; short src; };

struct Plan {
    bhac_params p{};
    std::vector<bhac_block_desc> blocks;
    std::vector<int64_t> off;            // padded offsets, nb + 1
    std::vector<int64_t> ioff;           // interior offsets, nb + 1
    int64_t ncell_interior = 0;
    std::vector<DevBlock> dblocks;
    std::vector<DevLevel> levels;        // indexed by level
    int maxlevel = 0;
    int gd[3] = {0, 0, 0};               // ghost layers per axis
    std::vector<int32_t> gdst, gsrc;     // same-level ghost gather map: face-adjacent slots first,
    long long nface_slots = 0;           // then edge and corner slots
    // block trees: cross-level ghost recipes (restriction / prolongation), slot q in
    // xdat[xoff[q] .. xoff[q+1]), the first nxl_face of them face-adjacent
    std::vector<int32_t> xoff, xdat;
    long long nxl_face = 0;
    // block trees: flux correction records [direction, coarse face, 4 fine faces]
    // (global indices into that direction's face array; 2 fine faces in 2-D)
    std::vector<int32_t> ffix;
    // metric tables (empty for flat space)
    long long nrec_c = 0, nrec_f0 = 0, nrec_f1 = 0;
    std::vector<double> ctab, f0tab, f1tab;
    std::vector<float> ctab32, f0tab32, f1tab32;   // face fields in float (face work of the mixed path)
    // work lists (one entry per work-group of WG items inside one block)
    std::vector<WorkItem> wcell, wface[3];
    std::vector<MarchItem> wmarch[3];
    // constrained transport: edge fields along each direction K, per block
    // (size_d + [d != K]) edges along d, x fastest; eofs[3 b + K] is block b's first edge
    std::vector<long long> eofs;
    std::vector<WorkItem> wedge[3];
    long long nedge[3] = {0, 0, 0};
    int march_mask = 0;                  // bit D: direction D uses the line kernel
    bool x1_staged = false;              // x1 faces by the LDS-staged face kernel
    bool x1_in_update = false;           // x1 faces computed inside the update kernel
    std::vector<WorkItem> wupd1;         // its work: x1u_rows(s0) whole rows per item (start = first row)
    int march_faces = MARCH_MAX_FACES;   // longest march segment, in faces
    long long nface[3] = {0, 0, 0};
    // fused-kernel neighbour data
    std::vector<int32_t> nbr;            // 27 per block: block id of neighbour slot (dir+1 base 3), -1 if none
    std::vector<HaloAxis> halo;          // per block: 3 axes x hmax entries
    int hmax = 0;                        // max padded extent over axes and blocks
    int smax[3] = {0, 0, 0};             // max interior size per axis
};

// Validate and build everything the device needs. tables == false skips the
// metric tables (host-only planning). Returns a BHAC_* code; err gets a message.
int make_plan(const bhac_params *p, const bhac_block_desc *blocks, int64_t nb, bool tables, Plan &out,
              std::string &err);

}  // namespace bhac
