// kernels.hip -- gfx950 kernels around the stage update: ghost fill at level
// jumps (restriction, prolongation; SRHD prolongs primitives), coarse-fine
// flux correction, x-boundary export, signal-speed reduction for dt, block
// permutation and ghost readout, and the regrid's Loehner estimate and data
// transfer.  Mostly one workgroup per task or block.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "agile_internal.hpp"
#include "device_math.hpp"

namespace agile {
// ---------------------------------------------------------------------------
// ghost-slab cell index (c in [0, 512)) -> (g, a, b) and back

// d = 0: [k][j][g], d = 1: [k][g][i], d = 2: [g][j][i]; written as selects
// (branches that each assign the three outputs are merged by the compiler
// into a small scratch array)
__device__ __forceinline__ void slab_coords(int d, int c, int &g, int &ta, int &tb) {
    g = d == 0 ? (c & 1) : (d == 1 ? ((c >> 4) & 1) : (c >> 8));
    ta = d == 0 ? ((c >> 1) & 15) : (c & 15);
    tb = d == 2 ? ((c >> 4) & 15) : (c >> 5);
}

// Value of variable v of block C at local cell (x, y, z), where at most one
// coordinate may lie one or two cells outside [0, 16): then it is a face ghost
// of C (same-level neighbour interior or C's ghost slab).
__device__ __forceinline__ double block_value(const BlockDesc *desc, const double *U, const double *halo, int NV,
                                              int C, int v, int x, int y, int z) {
    int o = -1;
    if (x < 0 || x >= BN) o = 0;
    else if (y < 0 || y >= BN) o = 1;
    else if (z < 0 || z >= BN) o = 2;
    if (o < 0) return U[(size_t(C) * NV + v) * CELLS + (z * 16 + y) * 16 + x];
    int c[3] = {x, y, z};
    const int side = c[o] >= BN;
    const int nb = desc[C].nb[2 * o + side];
    if (nb >= 0) {
        c[o] = side ? c[o] - BN : c[o] + BN;
        return U[(size_t(nb) * NV + v) * CELLS + (c[2] * 16 + c[1]) * 16 + c[0]];
    }
    const int g = side ? c[o] - BN : c[o] + NG;
    const int ta = o == 0 ? c[1] : c[0];
    const int tb = o == 2 ? c[1] : c[2];
    return halo[(size_t(-nb - 1) * NV + v) * SLAB + slab_index(o, g, ta, tb)];
}

// block_value reading the two x-boundary columns of a block (x = 0, 1, 14,
// 15) from the x-boundary copy XE, where rows of such cells are 256-byte runs
// instead of 16-byte pieces of 128-byte rows (XE holds the same values: the
// stage and flux-correction kernels write both); XE null: block_value.
__device__ __forceinline__ double block_value_xe(const BlockDesc *desc, const double *U, const double *XE,
                                                 const double *halo, int NV, int C, int v, int x, int y, int z) {
    if (XE && y >= 0 && y < BN && z >= 0 && z < BN) {
        int b = C, xx = x;
        if (x < 0 || x >= BN) {
            const int nb = desc[C].nb[x < 0 ? 0 : 1];
            if (nb < 0) return block_value(desc, U, halo, NV, C, v, x, y, z);
            b = nb;
            xx = x < 0 ? x + BN : x - BN;
        }
        if (xx < NG || xx >= BN - NG) {
            const int side = xx >= BN - NG;
            return XE[((size_t(b) * NV + v) * 2 + side) * SLAB + (z * 16 + y) * 2 + (xx - (side ? BN - NG : 0))];
        }
    }
    return block_value(desc, U, halo, NV, C, v, x, y, z);
}

// Restriction: coarse ghost = mean of its 8 fine children, summed pairwise
// ((c000+c100)+(c010+c110)) + ((c001+c101)+(c011+c111)) with x fastest.
// One lane per coarse ghost cell c of the slab; all 8 NV children of the cell
// are loaded before its NV sums are stored.
template <int NV>
__device__ __forceinline__ void restrict_cell(const RestrictTask *__restrict__ t, int c,
                                              const double *__restrict__ U, double *__restrict__ halo) {
    const int d = t->face >> 1, side = t->face & 1;
    int g, ta, tb;
    slab_coords(d, c, g, ta, tb);
    const int q = (ta >> 3) + 2 * (tb >> 3);
    const int F = t->fine[q];   // read through the pointer: a local copy indexed by q would live in scratch
    // first fine child along the normal (under coarse ghost layer g) and the
    // two tangential axes a (x, or y for d = 0) and b (z, or y for d = 2);
    // selects rather than an indexed array, which would live in scratch
    const int bn = side ? 2 * g : 12 + 2 * g, ba = 2 * (ta & 7), bb = 2 * (tb & 7);
    const int bx = d == 0 ? bn : ba;
    const int by = d == 1 ? bn : (d == 0 ? ba : bb);
    const int bz = d == 2 ? bn : bb;
    const double *u = U + size_t(F) * NV * CELLS + (bz * 16 + by) * 16 + bx;
    double ch[NV][8];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int k = 0; k < 8; ++k)
            ch[v][k] = u[v * CELLS + ((k >> 2) * 16 + ((k >> 1) & 1)) * 16 + (k & 1)];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double s = ((ch[v][0] + ch[v][1]) + (ch[v][2] + ch[v][3])) +
                         ((ch[v][4] + ch[v][5]) + (ch[v][6] + ch[v][7]));
        halo[(size_t(t->slot) * NV + v) * SLAB + c] = s * 0.125;
    }
}

// four workgroups of 128 lanes per restriction task
template <int NV>
__global__ __launch_bounds__(128) void k_restrict(const RestrictTask *__restrict__ tasks,
                                                  const double *__restrict__ U, double *__restrict__ halo) {
    restrict_cell<NV>(tasks + (blockIdx.x >> 2), threadIdx.x + 128 * (blockIdx.x & 3), U, halo);
}

// Prolongation: fine ghost = parent + sum over x, y, z (in that order) of
// +/- (1/4) minmod(parent - left, right - parent) of the parent's axis
// neighbours.  One workgroup per task: wave v takes variable v, lane p the
// coarse parent p of the face's 8 x 8 parents; the three limited slopes of a
// parent are formed once and give its 8 fine ghost cells (2 layers x 2 x 2).
template <int NV>
__global__ __launch_bounds__(64 * NV) void k_prolong(const ProlongTask *__restrict__ tasks,
                                                     const BlockDesc *__restrict__ desc,
                                                     const double *__restrict__ U, const double *__restrict__ XE,
                                                     double *__restrict__ halo) {
    const ProlongTask t = tasks[blockIdx.x];
    const int d = t.face >> 1, side = t.face & 1;
    const int da = d == 0 ? 1 : 0, dbx = d == 2 ? 1 : 2;
    const int v = threadIdx.x >> 6, p = threadIdx.x & 63;
    const int pa = p & 7, pb = p >> 3;
    int pc[3];
    pc[d] = side ? 0 : BN - 1;      // coarse layer next to the face
    pc[da] = t.ta + pa;
    pc[dbx] = t.tb + pb;
    const double vc = block_value_xe(desc, U, XE, halo, NV, t.coarse, v, pc[0], pc[1], pc[2]);
    double q[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        int m[3] = {pc[0], pc[1], pc[2]}, pp[3] = {pc[0], pc[1], pc[2]};
        m[e] -= 1;
        pp[e] += 1;
        const double vm = block_value_xe(desc, U, XE, halo, NV, t.coarse, v, m[0], m[1], m[2]);
        const double vp = block_value_xe(desc, U, XE, halo, NV, t.coarse, v, pp[0], pp[1], pp[2]);
        q[e] = 0.25 * minmod(vc - vm, vp - vc);
    }
    double *out = halo + (size_t(t.slot) * NV + v) * SLAB;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int g = k & 1, ca = (k >> 1) & 1, cb = k >> 2;
        int sg[3];
        sg[d] = g;                  // fine ghost layer g: the low child for g = 0
        sg[da] = ca;
        sg[dbx] = cb;
        double val = vc;
#pragma unroll
        for (int e = 0; e < 3; ++e) val = sg[e] ? val + q[e] : val - q[e];
        out[slab_index(d, g, 2 * pa + ca, 2 * pb + cb)] = val;
    }
}

// ---------------------------------------------------------------------------
// SRHD prolongation (Sec. 2.3.4): the same stencil on the primitives (rho,
// Gamma v, p) of the parent and its axis neighbours, each from the IEEE
// con2prim, and each child's primitives converted back with IEEE arithmetic
// without contraction -- the host's operations, so the ghosts and the regrid
// transfer keep the same bits.  Limited interpolation of the conserved
// variables could give |m| > tau + D next to a strong relativistic shock;
// minmod-limited primitives stay between neighbouring values.  A stencil cell
// without a physical state makes its children NaN (the next step reports
// it).

// (D, m, tau) from (rho, u, p): D = Gamma rho, m = Gamma rho h u,
// tau = Gamma^2 rho h - p - D, Gamma = sqrt(1 + u^2), rho h = rho + g/(g-1) p
__device__ __forceinline__ void srhd_prim2con_ieee(const double w[5], double g, double U[5]) {
#pragma clang fp contract(off)
    const double uu = (w[1] * w[1] + w[2] * w[2]) + w[3] * w[3];
    const double G = __builtin_sqrt(1.0 + uu);
    const double rhoh = w[0] + (g / (g - 1.0)) * w[4];
    U[0] = G * w[0];
    U[1] = (G * rhoh) * w[1];
    U[2] = (G * rhoh) * w[2];
    U[3] = (G * rhoh) * w[3];
    U[4] = ((G * G) * rhoh - w[4]) - U[0];
}

// primitives of cell (x, y, z) of block C (its ghosts included)
__device__ __forceinline__ bool srhd_cell_prims(const BlockDesc *desc, const double *U, const double *halo, int C,
                                                int x, int y, int z, double g, double w[5]) {
    double u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = block_value(desc, U, halo, 5, C, v, x, y, z);
    return srhd_con2prim(u, g, w);
}

// the parent cell's primitives wc and the quarter slopes q[axis][var]
__device__ __forceinline__ bool srhd_parent(const BlockDesc *desc, const double *U, const double *halo, int C,
                                            int x, int y, int z, double g, double wc[5], double q[3][5]) {
    bool ok = srhd_cell_prims(desc, U, halo, C, x, y, z, g, wc);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        double wm[5], wp[5];
        ok &= srhd_cell_prims(desc, U, halo, C, x - (e == 0), y - (e == 1), z - (e == 2), g, wm);
        ok &= srhd_cell_prims(desc, U, halo, C, x + (e == 0), y + (e == 1), z + (e == 2), g, wp);
#pragma unroll
        for (int v = 0; v < 5; ++v) q[e][v] = 0.25 * minmod(wc[v] - wm[v], wp[v] - wc[v]);
    }
    return ok;
}

// conserved state of the child on the (sx, sy, sz) side (1 = upper) of its
// parent: parent primitives +/- quarter slope per axis, in x, y, z order
__device__ __forceinline__ void srhd_child(const double wc[5], const double q[3][5], int sx, int sy, int sz, double g,
                                           bool ok, double out[5]) {
    double w[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        double val = wc[v];
        val = sx ? val + q[0][v] : val - q[0][v];
        val = sy ? val + q[1][v] : val - q[1][v];
        val = sz ? val + q[2][v] : val - q[2][v];
        w[v] = val;
    }
    srhd_prim2con_ieee(w, g, out);
    if (!ok) {
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v] = __builtin_nan("");
    }
}

// one 64-lane workgroup per prolongation task, lane p = coarse parent p
__global__ __launch_bounds__(64) void k_prolong_srhd(const ProlongTask *__restrict__ tasks,
                                                     const BlockDesc *__restrict__ desc,
                                                     const MeshParams *__restrict__ mp, const double *__restrict__ U,
                                                     double *__restrict__ halo) {
    const ProlongTask *t = tasks + blockIdx.x;
    const int d = t->face >> 1, side = t->face & 1;
    const int p = threadIdx.x, pa = p & 7, pb = p >> 3;
    const int da = d == 0 ? 1 : 0;
    const int lay = side ? 0 : BN - 1;      // coarse layer next to the face
    const int x = d == 0 ? lay : t->ta + pa;
    const int y = d == 1 ? lay : (da == 1 ? t->ta + pa : t->tb + pb);
    const int z = d == 2 ? lay : t->tb + pb;
    const double g = mp[desc[t->coarse].mesh].gamma;
    double wc[5], q[3][5];
    const bool ok = srhd_parent(desc, U, halo, t->coarse, x, y, z, g, wc, q);
    double *out = halo + size_t(t->slot) * 5 * SLAB;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int gl = k & 1, ca = (k >> 1) & 1, cb = k >> 2;
        // side of the child along each axis: the ghost layer along d, the
        // in-face offsets along the other two
        const int sx = d == 0 ? gl : ca;
        const int sy = d == 1 ? gl : (da == 1 ? ca : cb);
        const int sz = d == 2 ? gl : cb;
        double c[5];
        srhd_child(wc, q, sx, sy, sz, g, ok, c);
        const int o = slab_index(d, gl, 2 * pa + ca, 2 * pb + cb);
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v * SLAB + o] = c[v];
    }
}

// Coarse-fine flux correction of one coarse block: for each coarse-fine face
// the coarse flux F_c is replaced by the mean of the 4 fine fluxes covering it,
// F_f = ((f00+f10)+(f01+f11))/4, i.e. U += w dt/dx (+/-)(F_c - F_f).  Faces
// are taken in order (a cell on two such faces is corrected twice, in order);
// in the last stage of a step the signal rate of every corrected cell is
// taken from its final value (the lane of its last face) and joins the block
// maximum, which the stage left out for these cells.
template <int NV>
__device__ __forceinline__ void reflux_block(const RefluxTask *__restrict__ t, MeshParams *mp, double *__restrict__ U,
                                             double *__restrict__ XE, const double *__restrict__ freg,
                                             unsigned long long *smax, unsigned long long *cmax, double bw,
                                             int last) {
    // the task is read through its pointer (uniform scalar loads); a local
    // copy indexed by the face number would live in scratch
    const int block = t->block, nface = t->nface;
    MeshParams &P = mp[t->mesh];
    const double inv_dx = P.inv_dx1 * double(1 << (t->level - 1));
    const double w = (bw * P.dt) * inv_dx;   // the stage's weight of dt L
    // psi decay factor of the second half step (MHD; the expression of k_glm_decay)
    const double hdec = 0.5 * P.dt;
    const double fdec = NV == 9 ? exp(-hdec * P.ch * P.glm_alpha * inv_dx) : 1.0;
    unsigned long long m = 0, mc = 0;
    bool ok = true;
    // 256 lanes, one face cell each: (ta, tb) along the tangential axes,
    // quadrant q of the 4 fine blocks, first of its 2 x 2 fine faces (fa, fb)
    const int c = threadIdx.x;
    const int ta = c & 15, tb = c >> 4;
    const int q = (ta >> 3) + 2 * (tb >> 3);
    const int fa = 2 * (ta & 7), fb = 2 * (tb & 7);
    for (int n = 0; n < nface; ++n) {
        const int f = t->face[n], d = f >> 1, side = f & 1;
        const int xd = side ? BN - 1 : 0;
        const double *fr = freg + size_t(t->fslot[n][q]) * NV * REG;
        const double *cr = freg + size_t(t->cslot[n]) * NV * REG;
        // the face's cell: layer xd along the normal d, (ta, tb) along the
        // tangential axes (x or y, then z or y)
        const int cx = d == 0 ? xd : ta;
        const int cy = d == 1 ? xd : (d == 0 ? ta : tb);
        const int cz = d == 2 ? xd : tb;
        const size_t cell = (size_t(cz) * 16 + cy) * 16 + cx;
        // every load of the face before its stores
        double f4[NV][4], fc[NV], uo[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double *fp = fr + v * REG;
            f4[v][0] = fp[fb * 16 + fa];
            f4[v][1] = fp[fb * 16 + fa + 1];
            f4[v][2] = fp[(fb + 1) * 16 + fa];
            f4[v][3] = fp[(fb + 1) * 16 + fa + 1];
            fc[v] = cr[v * REG + c];
            uo[v] = U[(size_t(block) * NV + v) * CELLS + cell];
        }
        // final unless a later face of the list also holds the cell
        bool fin = true;
        for (int n2 = n + 1; n2 < nface; ++n2) {
            const int f2 = t->face[n2], d2 = f2 >> 1;
            const int cd = d2 == 0 ? cx : (d2 == 1 ? cy : cz);
            fin &= cd != ((f2 & 1) ? BN - 1 : 0);
        }
        double nu[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double fm = ((f4[v][0] + f4[v][1]) + (f4[v][2] + f4[v][3])) * 0.25;
            const double diff = fc[v] - fm;
            nu[v] = side ? uo[v] + w * diff : uo[v] - w * diff;
            // MHD, last stage: the second half of the GLM decay of psi, which
            // the stage kernel left out for the corrected cells, after the
            // cell's last correction
            if (NV == 9 && v == 8 && last && fin) nu[v] = nu[v] * fdec;
            U[(size_t(block) * NV + v) * CELLS + cell] = nu[v];
            if (XE && (cx < 2 || cx >= BN - 2)) {
                const int xs = cx >= BN - 2;
                XE[((size_t(block) * NV + v) * 2 + xs) * SLAB + (cz * 16 + cy) * 2 + (cx - (xs ? BN - 2 : 0))] = nu[v];
            }
        }
        if (last) {
            if (fin) {
                bool ok2;
                double sg, cm = 0.0;
                if (NV == 9) sg = mhd_signal(nu, P.gamma, inv_dx, cm, ok2);
                else if (P.physics == PHYS_SRHD) sg = srhd_signal(nu, P.gamma, inv_dx, ok2);
                else sg = signal_rate(nu, P.gamma, inv_dx, ok2);
                ok &= ok2;
                const unsigned long long sb = __double_as_longlong(sg), cb = __double_as_longlong(cm);
                m = sb > m ? sb : m;
                mc = cb > mc ? cb : mc;
            }
        }
        if (n + 1 < nface) __syncthreads();
    }
    if (last) {
        m = wave_max_u64(m);
        if ((threadIdx.x & 63) == 0) atomicMax(&smax[block], m);
        if (cmax) {
            mc = wave_max_u64(mc);
            if ((threadIdx.x & 63) == 0) atomicMax(&cmax[block], mc);
        }
        if (!ok) atomicOr(&P.flags, 1);
    }
}

template <int NV>
__global__ __launch_bounds__(256) void k_reflux(const RefluxTask *__restrict__ tasks, MeshParams *mp,
                                                double *__restrict__ U, double *__restrict__ XE,
                                                const double *__restrict__ freg, unsigned long long *smax,
                                                unsigned long long *cmax, double bw, int last) {
    reflux_block<NV>(tasks + blockIdx.x, mp, U, XE, freg, smax, cmax, bw, last);
}

// Flux correction of stage output U together with the restriction of the
// ghost fill that follows it, in one launch of 256-lane workgroups:
// [0, nref) correct, the others restrict (two per task).  Only used when no block that is
// corrected is also read by a restriction task, so the two sets are
// independent.
template <int NV>
__global__ __launch_bounds__(256) void k_reflux_restrict(const RefluxTask *__restrict__ rtasks, int nref,
                                                         const RestrictTask *__restrict__ stasks, MeshParams *mp,
                                                         double *__restrict__ U, double *__restrict__ XE,
                                                         const double *__restrict__ freg, double *__restrict__ halo,
                                                         unsigned long long *smax, unsigned long long *cmax,
                                                         double bw, int last) {
    const int bid = blockIdx.x;
    if (bid < nref) {
        reflux_block<NV>(rtasks + bid, mp, U, XE, freg, smax, cmax, bw, last);
    } else {
        const int r = bid - nref;
        restrict_cell<NV>(stasks + (r >> 1), threadIdx.x + 256 * (r & 1), U, halo);
    }
}

// x-boundary columns of every row into XE, for pool blocks [first, first + n)
__global__ __launch_bounds__(256) void k_xexport(const double *U, double *XE, int first, int NV) {
    const int b = first + blockIdx.x;
    for (int e = threadIdx.x; e < NV * XE_CELLS; e += blockDim.x) {
        const int v = e / XE_CELLS, r = e - v * XE_CELLS;
        const int side = r / SLAB, s = r - side * SLAB;
        const int g = s & 1, row = s >> 1;   // row = k*16 + j
        const int x = side ? BN - 2 + g : g;
        XE[(size_t(b) * NV + v) * XE_CELLS + r] = U[(size_t(b) * NV + v) * CELLS + row * 16 + x];
    }
}

// per-block maximum signal rate (and, with cmax, the MHD speed max_d |v_d| +
// c_f,d) of the current state, pool blocks [first, first + n)
__global__ __launch_bounds__(256) void k_smax(const BlockDesc *desc, MeshParams *mp, const double *U,
                                              unsigned long long *smax, unsigned long long *cmax, int first, int NV) {
    __shared__ unsigned long long sMax[2][4];
    const int b = first + blockIdx.x;
    const BlockDesc D = desc[b];
    MeshParams &P = mp[D.mesh];
    const double inv_dx = P.inv_dx1 * double(1 << (D.level - 1));
    unsigned long long m = 0, mc = 0;
    bool ok = true;
    for (int c = threadIdx.x; c < CELLS; c += blockDim.x) {
        double u[9];
        for (int v = 0; v < NV; ++v) u[v] = U[(size_t(b) * NV + v) * CELLS + c];
        bool ok2;
        double s, cm = 0.0;
        if (NV == 9) s = mhd_signal(u, P.gamma, inv_dx, cm, ok2);
        else if (P.physics == PHYS_SRHD) s = srhd_signal(u, P.gamma, inv_dx, ok2);
        else s = signal_rate(u, P.gamma, inv_dx, ok2);
        ok &= ok2;
        const unsigned long long sb = __double_as_longlong(s), cb = __double_as_longlong(cm);
        m = sb > m ? sb : m;
        mc = cb > mc ? cb : mc;
    }
    m = wave_max_u64(m);
    mc = wave_max_u64(mc);
    if ((threadIdx.x & 63) == 0) {
        sMax[0][threadIdx.x >> 6] = m;
        sMax[1][threadIdx.x >> 6] = mc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = sMax[0][0], rc = sMax[1][0];
        for (int w = 1; w < 4; ++w) {
            r = sMax[0][w] > r ? sMax[0][w] : r;
            rc = sMax[1][w] > rc ? sMax[1][w] : rc;
        }
        smax[b] = r;
        if (cmax) cmax[b] = rc;
    }
    if (!ok) atomicOr(&P.flags, 1);
}

// Per-mesh reductions, one workgroup per mesh of `meshes` (cmax: MHD only):
//   mode 0 (end of a step): smax (and cmax) = max over the mesh's blocks, t += dt;
//   mode 1 (start of a CFL step): dt = cfl / smax, c_h = cmax;
//   mode 2 (after an upload): smax (and cmax) = max over the mesh's blocks;
//   mode 3 (start of a step with a given dt): c_h = cmax.
__global__ __launch_bounds__(256) void k_mesh_reduce(MeshParams *mp, const int *meshes,
                                                     const unsigned long long *smax,
                                                     const unsigned long long *cmax, int mode) {
    __shared__ unsigned long long sMax[2][4];
    MeshParams &P = mp[meshes[blockIdx.x]];
    if (mode == 1 || mode == 3) {
        if (threadIdx.x == 0) {
            if (mode == 1) P.dt = P.cfl / __longlong_as_double(P.smax);
            P.ch = __longlong_as_double(P.cmax);
        }
        return;
    }
    const int first = P.first_block, n = P.nblocks;
    unsigned long long m = 0, mc = 0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const unsigned long long v = smax[first + q];
        m = v > m ? v : m;
        if (cmax) {
            const unsigned long long w = cmax[first + q];
            mc = w > mc ? w : mc;
        }
    }
    m = wave_max_u64(m);
    mc = wave_max_u64(mc);
    if ((threadIdx.x & 63) == 0) {
        sMax[0][threadIdx.x >> 6] = m;
        sMax[1][threadIdx.x >> 6] = mc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = sMax[0][0], rc = sMax[1][0];
        for (int w = 1; w < 4; ++w) {
            r = sMax[0][w] > r ? sMax[0][w] : r;
            rc = sMax[1][w] > rc ? sMax[1][w] : rc;
        }
        P.smax = r;
        P.cmax = rc;
        if (mode == 0) P.t = P.t + P.dt;
    }
}

__global__ void k_set_dt(MeshParams *mp, int mesh, double dt) {
    if (threadIdx.x == 0) mp[mesh].dt = dt;
}

// block copies between the caller's order (local index b) and the pool
// (block first + map[b]); gather = 1: pool -> caller, 0: caller -> pool
__global__ __launch_bounds__(256) void k_permute(const double *src, double *dst, const int *map, int first,
                                                 int per_block, int gather) {
    const int b = blockIdx.x;
    const size_t o = size_t(first) + map[b];
    const double *s = src + (gather ? o : size_t(b)) * per_block;
    double *d = dst + (gather ? size_t(b) : o) * per_block;
    for (int e = threadIdx.x; e < per_block; e += blockDim.x) d[e] = s[e];
}

// Streaming copy of n 16-byte words, the measure of the bandwidth the chip
// sustains on a plain read + write stream: one word per lane and pass,
// nontemporal loads and stores (the fastest of the shapes measured on gfx950:
// 4, 8 words in flight per lane and smaller grids were slower).
typedef double v2d __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_stream_copy(const v2d *__restrict__ src, v2d *__restrict__ dst, size_t n) {
    const size_t stride = size_t(gridDim.x) * 256;
    for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const size_t want = (n + 255) / 256;
    const unsigned grid = unsigned(want < (size_t(1) << 22) ? want : (size_t(1) << 22));
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, s, static_cast<const v2d *>(src),
                       static_cast<v2d *>(dst), n);
    return hipGetLastError();
}

// Copies between a caller's state in blocks of (16 te)^3 cells and the pool's
// 16^3 tiles: caller tile q is sub-tile (tx, ty, tz) = (q mod te, ...) of
// caller block q / te^3, and lives at pool tile first + map[q].  gather = 1:
// pool -> caller layout, 0: caller layout -> pool.  One workgroup per tile.
__global__ __launch_bounds__(256) void k_permute_tiles(const double *src, double *dst, const int *map, int first,
                                                       int NV, int te, int gather) {
    const int q = blockIdx.x, t3 = te * te * te;
    const int bq = q / t3, t = q - bq * t3;
    const int tx = t % te, ty = (t / te) % te, tz = t / (te * te);
    const int B = BN * te;
    const size_t pool = (size_t(first) + map[q]) * NV * CELLS;
    for (int e = threadIdx.x; e < NV * CELLS; e += blockDim.x) {
        const int v = e >> 12, c = e & (CELLS - 1);
        const int i = c & 15, j = (c >> 4) & 15, k = c >> 8;
        const size_t outer = ((size_t(bq) * NV + v) * B + (tz * BN + k)) * B * B + size_t(ty * BN + j) * B +
                             tx * BN + i;
        if (gather) dst[outer] = src[pool + e];
        else dst[pool + e] = src[outer];
    }
}

// face ghosts of pool blocks [first, first + n) as the update reads them:
// out[local block][face][var][512]
__global__ __launch_bounds__(256) void k_read_ghosts(const BlockDesc *desc, const double *U, const double *halo,
                                                     double *out, int first, int NV) {
    const int lb = blockIdx.x, b = first + lb;
    for (int e = threadIdx.x; e < 6 * SLAB; e += blockDim.x) {
        const int f = e / SLAB, c = e - f * SLAB;
        const int d = f >> 1, side = f & 1;
        int g, ta, tb;
        slab_coords(d, c, g, ta, tb);
        int x[3];
        x[d] = side ? BN + g : g - NG;
        x[d == 0 ? 1 : 0] = ta;
        x[d == 2 ? 1 : 2] = tb;
        for (int v = 0; v < NV; ++v)
            out[((size_t(lb) * 6 + f) * NV + v) * SLAB + c] = block_value(desc, U, halo, NV, b, v, x[0], x[1], x[2]);
    }
}

// ---------------------------------------------------------------------------
// launch wrappers (host)

hipError_t launch_restrict(const RestrictTask *t, int n, const double *U, double *halo, int NV, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (NV == 9) hipLaunchKernelGGL(k_restrict<9>, dim3(4 * n), dim3(128), 0, s, t, U, halo);
    else hipLaunchKernelGGL(k_restrict<5>, dim3(4 * n), dim3(128), 0, s, t, U, halo);
    return hipGetLastError();
}

hipError_t launch_prolong(const ProlongTask *t, int n, const BlockDesc *desc, const MeshParams *mp, const double *U,
                          const double *XE, double *halo, int NV, int srhd, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (srhd && NV != 5) return hipErrorInvalidValue;
    if (srhd) hipLaunchKernelGGL(k_prolong_srhd, dim3(n), dim3(64), 0, s, t, desc, mp, U, halo);
    else if (NV == 9) hipLaunchKernelGGL(k_prolong<9>, dim3(n), dim3(64 * 9), 0, s, t, desc, U, XE, halo);
    else hipLaunchKernelGGL(k_prolong<5>, dim3(n), dim3(64 * 5), 0, s, t, desc, U, XE, halo);
    return hipGetLastError();
}

hipError_t launch_reflux(const RefluxTask *t, int n, MeshParams *mp, double *U, double *XE, const double *freg,
                         unsigned long long *smax, unsigned long long *cmax, int NV, double bw, int last,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (NV == 9)
        hipLaunchKernelGGL(k_reflux<9>, dim3(n), dim3(256), 0, s, t, mp, U, XE, freg, smax, cmax, bw, last);
    else hipLaunchKernelGGL(k_reflux<5>, dim3(n), dim3(256), 0, s, t, mp, U, XE, freg, smax, cmax, bw, last);
    return hipGetLastError();
}

hipError_t launch_reflux_restrict(const RefluxTask *rt, int nref, const RestrictTask *st, int nres, MeshParams *mp,
                                  double *U, double *XE, const double *freg, double *halo, unsigned long long *smax,
                                  unsigned long long *cmax, int NV, double bw, int last, hipStream_t s) {
    if (nref <= 0 || nres <= 0) return hipErrorInvalidValue;
    const dim3 grid(nref + 2 * nres), block(256);
    if (NV == 9)
        hipLaunchKernelGGL(k_reflux_restrict<9>, grid, block, 0, s, rt, nref, st, mp, U, XE, freg, halo, smax, cmax, bw,
                           last);
    else
        hipLaunchKernelGGL(k_reflux_restrict<5>, grid, block, 0, s, rt, nref, st, mp, U, XE, freg, halo, smax, cmax, bw,
                           last);
    return hipGetLastError();
}

hipError_t launch_xexport(const double *U, double *XE, int first, int n, int NV, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_xexport, dim3(n), dim3(256), 0, s, U, XE, first, NV);
    return hipGetLastError();
}

hipError_t launch_smax(const BlockDesc *desc, MeshParams *mp, const double *U, unsigned long long *smax,
                       unsigned long long *cmax, int first, int n, int NV, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_smax, dim3(n), dim3(256), 0, s, desc, mp, U, smax, cmax, first, NV);
    return hipGetLastError();
}

hipError_t launch_mesh_reduce(MeshParams *mp, const int *meshes, int nmesh, const unsigned long long *smax,
                              const unsigned long long *cmax, int mode, hipStream_t s) {
    if (nmesh <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mesh_reduce, dim3(nmesh), dim3(256), 0, s, mp, meshes, smax, cmax, mode);
    return hipGetLastError();
}

hipError_t launch_set_dt(MeshParams *mp, int mesh, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(64), 0, s, mp, mesh, dt);
    return hipGetLastError();
}

hipError_t launch_permute(const double *src, double *dst, const int *map, int first, int nblocks, int per_block,
                          int gather, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute, dim3(nblocks), dim3(256), 0, s, src, dst, map, first, per_block, gather);
    return hipGetLastError();
}

hipError_t launch_permute_tiles(const double *src, double *dst, const int *map, int first, int ntiles, int NV,
                                int te, int gather, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_tiles, dim3(ntiles), dim3(256), 0, s, src, dst, map, first, NV, te, gather);
    return hipGetLastError();
}

hipError_t launch_read_ghosts(const BlockDesc *desc, const double *U, const double *halo, double *out, int first,
                              int n, int NV, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_read_ghosts, dim3(n), dim3(256), 0, s, desc, U, halo, out, first, NV);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// regrid: error estimate and data transfer

// Loehner's normalised second difference of variable v per cell, summed over
// the three axes without cross terms (face ghosts at block sides),
//   E = sqrt(sum_d a_d^2 / sum_d b_d^2),  a_d = (u+ - u) - (u - u-),
//   b_d = (|u+ - u| + |u - u-|) + eps((|u+| + 2|u|) + |u-|),
// sums in x, y, z order, no contraction and IEEE division and square root
// (E = 0 where v is zero on the whole stencil and both sums vanish),
// so the block maximum is the same number on any machine.  One workgroup per
// block, lane = column; out[block - first] = max over the block's cells.
template <int NV>
__global__ __launch_bounds__(256) void k_lohner(const BlockDesc *__restrict__ desc, const double *__restrict__ U,
                                                const double *__restrict__ halo, int first, int v, double eps,
                                                double *__restrict__ out) {
#pragma clang fp contract(off)
    __shared__ unsigned long long sMax[4];
    const int b = first + blockIdx.x;
    const int i = threadIdx.x & 15, j = threadIdx.x >> 4;
    unsigned long long m = 0;
    for (int k = 0; k < BN; ++k) {
        const double u0 = U[(size_t(b) * NV + v) * CELLS + (k * 16 + j) * 16 + i];
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double up = block_value(desc, U, halo, NV, b, v, i + (d == 0), j + (d == 1), k + (d == 2));
            const double um = block_value(desc, U, halo, NV, b, v, i - (d == 0), j - (d == 1), k - (d == 2));
            const double a = (up - u0) - (u0 - um);
            const double c = (__builtin_fabs(up - u0) + __builtin_fabs(u0 - um)) +
                             eps * ((__builtin_fabs(up) + 2.0 * __builtin_fabs(u0)) + __builtin_fabs(um));
            num = num + a * a;
            den = den + c * c;
        }
        const double e = den > 0.0 ? __builtin_sqrt(num / den) : 0.0;   // den = 0: v is 0 on the stencil
        const unsigned long long eb = __double_as_longlong(e);   // e >= 0: bit order = numeric order
        m = eb > m ? eb : m;
    }
    m = wave_max_u64(m);
    if ((threadIdx.x & 63) == 0) sMax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = sMax[0];
        for (int w = 1; w < 4; ++w) r = sMax[w] > r ? sMax[w] : r;
        out[blockIdx.x] = __longlong_as_double(r);
    }
}

// Data of the new leaves of a regrid, one workgroup per new leaf, lane =
// column: kind 0 copies block src[0]; kind 1 is child `octant` of parent
// src[0] -- parent cell plus, in x, y, z order, +/- 1/4 minmod of the
// parent's axis differences (the parent's face ghosts at its sides), as the
// ghost prolongation; kind 2 is the mean of the 8 children src[octant],
// summed pairwise as the restriction.  All indices are pool indices of the
// old mesh, whose ghosts must be filled.  SRHD (srhd != 0) prolongs the
// primitives, as its ghost prolongation: one lane per child cell.
template <int NV>
__global__ __launch_bounds__(256) void k_remap(const RemapTask *__restrict__ tasks, const BlockDesc *__restrict__ desc,
                                               const MeshParams *__restrict__ mp, const double *__restrict__ U,
                                               const double *__restrict__ halo, double *__restrict__ out, int srhd) {
    const RemapTask *t = tasks + blockIdx.x;   // read through the pointer (no scratch copy)
    const int kind = t->kind, oc = t->octant;
    double *o = out + size_t(blockIdx.x) * NV * CELLS;
    if (kind == 0) {
        const double *src = U + size_t(t->src[0]) * NV * CELLS;
#pragma unroll 4
        for (int e = threadIdx.x; e < NV * CELLS; e += 256) o[e] = src[e];
        return;
    }
    if (NV == 5 && srhd && kind == 1) {
        const int P = t->src[0];
        const double g = mp[desc[P].mesh].gamma;
#pragma unroll 1
        for (int cell = threadIdx.x; cell < CELLS; cell += 256) {
            const int i = cell & 15, j = (cell >> 4) & 15, k = cell >> 8;
            double wc[5], q[3][5], c[5];
            const bool ok = srhd_parent(desc, U, halo, P, (oc & 1) * 8 + (i >> 1), ((oc >> 1) & 1) * 8 + (j >> 1),
                                        (oc >> 2) * 8 + (k >> 1), g, wc, q);
            srhd_child(wc, q, i & 1, j & 1, k & 1, g, ok, c);
#pragma unroll
            for (int v = 0; v < 5; ++v) o[v * CELLS + cell] = c[v];
        }
        return;
    }
#pragma unroll 1
    for (int e = threadIdx.x; e < NV * CELLS; e += 256) {
        const int v = e >> 12, cell = e & (CELLS - 1);
        const int i = cell & 15, j = (cell >> 4) & 15, k = cell >> 8;
        double val;
        if (kind == 2) {
            const int F = t->src[(i >> 3) + 2 * (j >> 3) + 4 * (k >> 3)];
            const double *u = U + (size_t(F) * NV + v) * CELLS + ((2 * (k & 7)) * 16 + 2 * (j & 7)) * 16 + 2 * (i & 7);
            const double s = ((u[0] + u[1]) + (u[16] + u[17])) + ((u[256] + u[257]) + (u[272] + u[273]));
            val = s * 0.125;
        } else {
            const int P = t->src[0];
            const int cx = (oc & 1) * 8 + (i >> 1), cy = ((oc >> 1) & 1) * 8 + (j >> 1), cz = (oc >> 2) * 8 + (k >> 1);
            const double vc = U[(size_t(P) * NV + v) * CELLS + (cz * 16 + cy) * 16 + cx];
            val = vc;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double vm = block_value(desc, U, halo, NV, P, v, cx - (d == 0), cy - (d == 1), cz - (d == 2));
                const double vp = block_value(desc, U, halo, NV, P, v, cx + (d == 0), cy + (d == 1), cz + (d == 2));
                const double q = 0.25 * minmod(vc - vm, vp - vc);
                const int odd = d == 0 ? (i & 1) : (d == 1 ? (j & 1) : (k & 1));
                val = odd ? val + q : val - q;
            }
        }
        o[e] = val;
    }
}

hipError_t launch_lohner(const BlockDesc *desc, const double *U, const double *halo, int first, int n, int NV, int v,
                         double eps, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (v < 0 || v >= NV) return hipErrorInvalidValue;
    if (NV == 9) hipLaunchKernelGGL(k_lohner<9>, dim3(n), dim3(256), 0, s, desc, U, halo, first, v, eps, out);
    else hipLaunchKernelGGL(k_lohner<5>, dim3(n), dim3(256), 0, s, desc, U, halo, first, v, eps, out);
    return hipGetLastError();
}

hipError_t launch_remap(const RemapTask *t, int n, const BlockDesc *desc, const MeshParams *mp, const double *U,
                        const double *halo, int NV, int srhd, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (srhd && NV != 5) return hipErrorInvalidValue;
    if (NV == 9) hipLaunchKernelGGL(k_remap<9>, dim3(n), dim3(256), 0, s, t, desc, mp, U, halo, out, 0);
    else hipLaunchKernelGGL(k_remap<5>, dim3(n), dim3(256), 0, s, t, desc, mp, U, halo, out, srhd);
    return hipGetLastError();
}

} // namespace agile
