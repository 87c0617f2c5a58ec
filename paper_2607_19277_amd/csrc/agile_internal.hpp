// agile_internal.hpp -- data layouts shared by the host bookkeeping and the
// gfx950 kernels of the block-AMR update.
//
// Device memory of a mesh (all float64, blocks in device order = level, then
// Morton order of the block coordinates, the space-filling-curve walk of the
// main update loop in Sec. 2.1.3):
//   U[2]   [block][var][16][16][16]   interiors only; stage input / output
//   XE[2]  [block][var][side][16][16][2]
//          copy of the two x-boundary columns of each row (side 0: i = 0,1;
//          side 1: i = 14,15) so that x-ghosts read whole 256-byte runs
//   halo   [slot][var][512]            ghost slabs of faces at a level jump
//   freg   [slot][var][256]            face fluxes kept for flux correction
// A ghost slab is 2 cells deep, stored in (k, j, i) order of the ghost box:
//   x-face [k][j][g], y-face [k][g][i], z-face [g][j][i],
// g increasing with the coordinate (for a -face g=0 is the far layer).
// A flux register is [b][a] with (a, b) the lower / upper tangential axis.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace agile {

constexpr int BN = 16;                    // cells per block edge
constexpr int NG = 2;                     // ghost layers
constexpr int CELLS = BN * BN * BN;       // 4096
constexpr int SLAB = NG * BN * BN;        // 512 cells in a ghost slab
constexpr int XE_CELLS = 2 * BN * BN * NG;// 1024 per block and variable
constexpr int REG = BN * BN;              // 256 faces per block face
constexpr int MAXLEV = 12;

// Per-block descriptor (64 bytes).
struct BlockDesc {
    int nb[6];       // face f: >= 0 same-level neighbour (device block index),
                     //         <  0 ghost slab -(slot+1) (neighbour at another level)
    int freg[6];     // flux register slot written by this face, or -1
    int level;       // 1 = base level
    int mesh;        // mesh slot (parameters, dt, reductions)
    int cf_coarse;   // bit f: face f is the coarse side of a coarse-fine face
    int pad;
};

// Per-mesh parameters and reduction slots on the device (88 bytes).
constexpr int PHYS_SRHD = 2;   // the value of AGILE_SRHD in MeshParams::physics

struct MeshParams {
    double gamma;
    double cfl;
    double inv_dx1;          // 1 / dx on level 1 (power-of-two scaling per level)
    double glm_alpha;
    double dt;               // dt of the step in progress / last step
    double t;                // simulated time reached (sum of the dt of all steps)
    double ch;               // MHD: GLM cleaning speed of the step in progress
    unsigned long long smax; // bits of max signal rate of the current state
    unsigned long long cmax; // MHD: bits of max_d (|v_d| + c_f,d) of the current state
    int first_block;         // block range of the mesh in the pool
    int nblocks;
    int flags;               // bit 0: non-physical state met
    int physics;             // AGILE_EULER, AGILE_MHD_GLM or AGILE_SRHD
};

// Index of ghost cell (layer g, tangential coordinates (ta, tb) in axis
// order) in the 512-cell slab of a face normal to axis d.
__host__ __device__ inline int slab_index(int d, int g, int ta, int tb) {
    if (d == 0) return (tb * 16 + ta) * 2 + g;
    if (d == 1) return (tb * 2 + g) * 16 + ta;
    return (g * 16 + tb) * 16 + ta;
}

// Restriction into the ghost slab of a coarse block face next to 4 finer blocks.
struct RestrictTask {
    int slot;        // destination ghost slab
    int face;        // face of the coarse block
    int block;       // coarse block
    int fine[4];     // fine blocks, quadrant q = qa + 2 qb over the (a, b) tangential axes
    int pad;
};

// Prolongation into the ghost slab of a fine block face next to a coarser block.
struct ProlongTask {
    int slot;        // destination ghost slab
    int face;        // face of the fine block
    int block;       // fine block
    int coarse;      // coarser neighbour block
    int ta, tb;      // offset (0 or 8 coarse cells) of the fine face inside the coarse face
    int pad[2];
};

// Flux correction of one coarse block: all its coarse-fine faces, in order.
struct RefluxTask {
    int block;
    int level;       // level of the coarse block
    int mesh;        // mesh slot of the coarse block
    int nface;
    int face[6];
    int cslot[6];    // coarse flux register of the face
    int fslot[6][4]; // fine flux registers of the 4 fine blocks (quadrant order)
};

// Data source of one new leaf of a regrid (pool indices of the old mesh):
// kind 0 copy of src[0], 1 child `octant` (x + 2y + 4z) of parent src[0],
// 2 mean of the 8 children src[0..7] in octant order.
struct RemapTask {
    int kind;
    int octant;
    int src[8];
};

struct StageArgs {
    const BlockDesc *desc;
    MeshParams *mp;
    const double *Uin;     // stage input (U^n or U^(1))
    double *Uout;          // stage output
    const double *Un;      // stage 2: U^n (pointwise); stage 1: unused
    const double *XEin;
    double *XEout;
    const double *halo;
    double *freg;
    unsigned long long *smax;  // per block: reset in stage 1, maximum in stage 2
    const int *list;       // blocks to update (pool indices), or null for [0, nblocks)
    int nblocks;           // number of blocks to update
    int kslab;             // planes per workgroup: 16, 8 or 4 (same arithmetic per cell)
    int xcd;               // 1: XCD-aware workgroup -> block mapping
    int stage;             // stage kind: 1 first, 2 last SSP-RK2, 3 middle / 4 last SSP-RK3
    int limiter;           // 0 minmod, 1 van Leer
};

// A stage's output and U^n are each touched once per launch: their accesses
// carry streaming (nontemporal) hints so that they do not displace, in L2, the
// input planes and ghost rows that neighbouring work items read again.
__device__ __forceinline__ void store_out(double *p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ double load_un(const double *p) { return __builtin_nontemporal_load(p); }

// The ideal-MHD stage (nvar 9) of the listed blocks.
struct SweepArgs {
    const BlockDesc *desc;
    MeshParams *mp;
    const double *Uin;     // stage input
    double *Uout;          // stage output
    const double *Un;      // stage 2: U^n
    const double *XEin;    // x-boundary copies of Uin and Uout
    double *XEout;
    const double *halo;
    double *freg;
    unsigned long long *smax;  // per block: reset in stage 1, maximum in stage 2
    unsigned long long *cmax;  // per block, as smax, for max_d (|v_d| + c_f,d)
    const int *list;
    int nblocks;
};

} // namespace agile
