// mhd.hip -- gfx950 kernels of the ideal-MHD + GLM stage update (Sec. 2.3.3),
// nvar 9: (rho, m, e, B, psi).
//
// A stage is one launch of k_mhd_stage, one workgroup of 256 lanes per block
// marching in z: PLM minmod on primitives, the GLM interface step and the HLL
// flux (mhd_hll) for the z faces from a per-lane register window and for the
// x and y faces from the plane in LDS, L = -((dFx + dFy) + dFz)/dx, the
// SSP-RK2 stage combination, flux registers and, in stage 2, the exact
// signal rate and GLM speed of the new state (cells about to be
// flux-corrected excepted).  The GLM source is split off exactly: psi decays
// by exp(-dt/2 c_h alpha/dx) before the two stages (k_glm_decay) and after
// them (applied to the output by the last stage, and by the flux correction to
// the cells it corrects, after their last correction).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "agile_internal.hpp"
#include "device_math.hpp"

namespace agile {

namespace {

constexpr int NV = 9;
constexpr int NF = BN + 1;        // 17 faces per line
constexpr int NXY = BN * NF;      // 272 x (and y) faces per plane

} // namespace

// The whole stage of one block in one workgroup of 256 lanes, marching in z
// (lane (i, j) owns the z-column (i, j)); per plane k:
//   (1) the z face k+1/2 from a register window of the column's rotated
//       primitives (cells k, k+1 and the next cell, converted as it arrives;
//       the left state of the face carried from the previous plane), then
//       the x faces and the y faces of plane k from the plane's primitives
//       in LDS (global variable order, 20 x 20 with the x / y ghosts), each
//       flux into its own LDS buffer;
//   (2) after a barrier: dFx + dFy of the lane's cell from LDS, dFz from the
//       z fluxes in registers, L = -((dFx + dFy) + dFz)/dx, the stage
//       combination with the cell's input (kept from its load three planes
//       earlier, or read again, see AGILE_MHD_RING) and, in stage 2, U^n; flux registers of
//       faces that carry one; stage 2: the signal rate and GLM speed of the
//       new state; the next plane's primitives into LDS; a barrier.
// Each face flux is computed once; the state is read once per stage (in the
// FP32 first stage the cell's input a second time, partly from cache; x
// ghosts from the neighbour's x-boundary copy), and nothing but the output with the x-boundary
// copy of its boundary columns, the flux registers and the signal maxima is
// written.  The next cell of the window and, after the output, the next
// plane's ghosts are loaded in (2), so they are not live during the face work
// of (1).
// Occupancy: the FP64 stages hold 2 waves per SIMD (256 VGPRs).  With FP32
// fluxes the first stage fits 3 (168 VGPRs, 12 bytes of scratch; 12% faster
// than at 2), the last stage would spill 23 registers at 3 and is kept at 2.
// Which instantiations keep the column's conserved values of planes k, k+1
// and k+2 in registers instead of reading plane k again for its update (bit
// 0: FP64 first stage, 1: FP64 last, 2: FP32 first, 3: FP32 last).  Measured
// on the Orszag-Tang mesh: the FP64 stages and the FP32 last stage gain
// 2.5-2.7% of a step with it (the FP64 last stage then spills 36 bytes); the
// FP32 first stage would drop from 3 waves per SIMD to 2 and lose that.
#ifndef AGILE_MHD_RING
#define AGILE_MHD_RING 11
#endif
#ifndef AGILE_MHD_WAVES_F32_FIRST
#define AGILE_MHD_WAVES_F32_FIRST 3
#endif
#ifndef AGILE_MHD_WAVES_F32_LAST
#define AGILE_MHD_WAVES_F32_LAST 2
#endif

template <int STAGE, typename R>
__global__ __launch_bounds__(256, sizeof(R) == 8 ? 2 : (STAGE == 1 ? AGILE_MHD_WAVES_F32_FIRST : AGILE_MHD_WAVES_F32_LAST))
void k_mhd_stage(SweepArgs a) {
    constexpr bool RING = (AGILE_MHD_RING >> ((sizeof(R) == 4 ? 2 : 0) + (STAGE == 2 ? 1 : 0))) & 1;
    constexpr int PW = BN + 2 * NG;   // 20
    __shared__ R sW[NV][PW][PW];
    __shared__ R sF[NV][2 * NXY];   // x face fluxes, then y face fluxes, global variable order
    __shared__ unsigned long long sMax[2][4];
    const int bi = blockIdx.x;
    if (bi >= a.nblocks) return;
    const int b = a.list ? a.list[bi] : bi;
    const int tid = threadIdx.x;
    const int i = tid & 15, j = tid >> 4;
    const BlockDesc *Dsc = a.desc + b;
    MeshParams &mp = a.mp[Dsc->mesh];
    const double gamma = mp.gamma, gm1 = gamma - 1.0;
    const double inv_dx = mp.inv_dx1 * double(1 << (Dsc->level - 1));
    const double dt = mp.dt;
    const double ch = mp.ch;
    // the last stage also applies the second half of the GLM decay of psi
    // (the factor of k_glm_decay for h = dt/2, the same expression) to every
    // cell that no flux correction follows; k_reflux applies it to the
    // corrected cells after their last correction
    const double hdec = 0.5 * dt;
    const double fdec = STAGE == 2 ? exp(-hdec * ch * mp.glm_alpha * inv_dx) : 1.0;
    const R gammaR = R(gamma), igm1R = R(1.0 / gm1), chR = R(ch), inv2chR = R(0.5 / ch);
    const size_t blk = size_t(b) * NV * CELLS;
    const int colp = j * 16 + i;
    bool ok = true;
    if (STAGE == 1 && tid == 0) {
        a.smax[b] = 0;
        a.cmax[b] = 0;
    }

    // conserved values of this column's cell at z index kk in [-2, 18)
    auto zload = [&](int kk, double C[NV]) {
        const double *p;
        int st;
        if (kk >= 0 && kk < BN) {
            p = a.Uin + blk + kk * 256 + colp;
            st = CELLS;
        } else {
            const int nb = kk < 0 ? Dsc->nb[4] : Dsc->nb[5];
            if (nb >= 0) {
                p = a.Uin + size_t(nb) * NV * CELLS + (kk < 0 ? kk + BN : kk - BN) * 256 + colp;
                st = CELLS;
            } else {
                p = a.halo + size_t(-nb - 1) * NV * SLAB + (kk < 0 ? kk + NG : kk - BN) * 256 + colp;
                st = SLAB;
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) C[v] = p[v * st];
    };
    // rotated primitives for the z normal: (rho, vz, vx, vy, p, Bz, Bx, By, psi)
    auto prim_z = [&](const double C[NV], R w[NV]) {
        double q[NV];
        ok &= mhd_cons2prim(C, gm1, q);
        w[0] = R(q[0]); w[1] = R(q[3]); w[2] = R(q[1]); w[3] = R(q[2]); w[4] = R(q[4]);
        w[5] = R(q[7]); w[6] = R(q[5]); w[7] = R(q[6]); w[8] = R(q[8]);
    };
    // x / y ghost cell of plane k: lanes 0..127, one each (4 faces x 2 layers
    // x 16); lanes 128.. repeat lanes 0..127
    const int g = tid & 127, gf = g >> 5, gr = g & 31;
    const int gd = gf >> 1, gside = gf & 1;
    const int ggl = gd == 0 ? (gr & 1) : (gr >> 4), gt = gd == 0 ? (gr >> 1) : (gr & 15);
    const int gp = gside ? BN + ggl : ggl - NG;   // position along the face normal
    const int gx = gd == 0 ? gp : gt, gy = gd == 0 ? gt : gp;
    const int gnb = Dsc->nb[gf];
    // lanes of the two x-boundary columns also write the x-boundary copy
    const bool xcol = i < NG || i >= BN - NG;
    double *const xo = a.XEout + (size_t(b) * NV * 2 + (i >= BN - NG)) * SLAB + j * 2 + (i >= BN - NG ? i - (BN - NG) : i);
    auto gload = [&](int k, double G[NV]) {
        const double *src;
        int st;
        if (gnb >= 0 && gd == 0) {
            // x ghosts: the neighbour's boundary columns from its x-boundary
            // copy (whole 256-byte runs instead of 16 bytes of each row)
            src = a.XEin + (size_t(gnb) * NV * 2 + (gside ? 0 : 1)) * SLAB + (k * 16 + gy) * 2 + ggl;
            st = 2 * SLAB;
        } else if (gnb >= 0) {
            const int yn = gside ? gp - BN : gp + BN;
            src = a.Uin + size_t(gnb) * NV * CELLS + (k * 16 + yn) * 16 + gx;
            st = CELLS;
        } else {
            src = a.halo + size_t(-gnb - 1) * NV * SLAB + slab_index(gd, gside ? gp - BN : gp + NG, gt, k);
            st = SLAB;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) G[v] = src[v * st];
    };
    // plane primitives into LDS: the lane's own cell (from its z-rotated
    // primitives) and its ghost cell
    auto put_plane = [&](const R w[NV], const double G[NV]) {
        sW[0][j + NG][i + NG] = w[0];
        sW[1][j + NG][i + NG] = w[2];
        sW[2][j + NG][i + NG] = w[3];
        sW[3][j + NG][i + NG] = w[1];
        sW[4][j + NG][i + NG] = w[4];
        sW[5][j + NG][i + NG] = w[6];
        sW[6][j + NG][i + NG] = w[7];
        sW[7][j + NG][i + NG] = w[5];
        sW[8][j + NG][i + NG] = w[8];
        double q[NV];
        ok &= mhd_cons2prim(G, gm1, q);
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v][gy + NG][gx + NG] = R(q[v]);
    };

    // prologue: cells -2 .. 2 of the column, face -1/2, plane 0 in LDS
    R wk[NV], wk1[NV], wLz[NV], Flo[NV];
    double C2[NV];
    double Ck[RING ? NV : 1], Ck1[RING ? NV : 1];   // ring: conserved values of planes k, k+1
    {
        double Cm2[NV], Cm1[NV], C0[NV], C1[NV], G0[NV];
        zload(-2, Cm2);
        zload(-1, Cm1);
        zload(0, C0);
        zload(1, C1);
        zload(2, C2);
        gload(0, G0);
        R wm2[NV], wm1[NV], wL[NV], wR[NV];
        prim_z(Cm2, wm2);
        prim_z(Cm1, wm1);
        prim_z(C0, wk);
        prim_z(C1, wk1);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const R d0 = wm1[v] - wm2[v], d1 = wk[v] - wm1[v], d2 = wk1[v] - wk[v];
            wL[v] = wm1[v] + R(0.5) * minmod(d0, d1);
            wR[v] = wk[v] - R(0.5) * minmod(d1, d2);
            wLz[v] = wk[v] + R(0.5) * minmod(d1, d2);
        }
        mhd_hll<R>(wL, wR, gammaR, igm1R, chR, inv2chR, Flo);
        put_plane(wk, G0);
        if (RING) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Ck[v] = C0[v];
                Ck1[v] = C1[v];
            }
        }
    }
    if (Dsc->freg[4] >= 0) {   // z flux register of face -1/2, global variable order
        double *r = a.freg + size_t(Dsc->freg[4]) * NV * REG + colp;
        r[0] = double(Flo[0]); r[REG] = double(Flo[2]); r[2 * REG] = double(Flo[3]); r[3 * REG] = double(Flo[1]);
        r[4 * REG] = double(Flo[4]); r[5 * REG] = double(Flo[6]); r[6 * REG] = double(Flo[7]);
        r[7 * REG] = double(Flo[5]); r[8 * REG] = double(Flo[8]);
    }
    __syncthreads();

    // the x (D = 0) or y (D = 1) face f = l * NF + fi of plane k, from LDS
    // (line l, face fi before position fi), flux into sF[.][D * NXY + f]
    auto face_task = [&](auto Dc, int f, int k) {
        constexpr int D = decltype(Dc)::value;
        constexpr int n1 = (D + 1) % 3, n2 = (D + 2) % 3;
        const int l = f / NF, fi = f - NF * l;
        R wL[NV], wR[NV], F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            // rotated variable v <- global variable
            const int gv = v == 1 ? 1 + D : (v == 2 ? 1 + n1 : (v == 3 ? 1 + n2 : (v == 5 ? 5 + D : (v == 6 ? 5 + n1 : (v == 7 ? 5 + n2 : v)))));
            R c[4];
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                const int yy = D == 0 ? l + NG : fi + s2, xx = D == 0 ? fi + s2 : l + NG;
                c[s2] = sW[gv][yy][xx];
            }
            const R d0 = c[1] - c[0], d1 = c[2] - c[1], d2 = c[3] - c[2];
            wL[v] = c[1] + R(0.5) * minmod(d0, d1);
            wR[v] = c[2] - R(0.5) * minmod(d1, d2);
        }
        mhd_hll<R>(wL, wR, gammaR, igm1R, chR, inv2chR, F);
        R G[NV];
        G[0] = F[0]; G[1 + D] = F[1]; G[1 + n1] = F[2]; G[1 + n2] = F[3]; G[4] = F[4];
        G[5 + D] = F[5]; G[5 + n1] = F[6]; G[5 + n2] = F[7]; G[8] = F[8];
#pragma unroll
        for (int v = 0; v < NV; ++v) sF[v][D * NXY + f] = G[v];
        if (fi == 0 || fi == BN) {
            const int slot = Dsc->freg[2 * D + (fi == BN)];
            if (slot >= 0) {
                double *r = a.freg + size_t(slot) * NV * REG + k * 16 + l;
#pragma unroll
                for (int v = 0; v < NV; ++v) r[v * REG] = double(G[v]);
            }
        }
    };
    // 272 x and 272 y faces over 256 lanes: every lane one x face and one y
    // face; the 16 remaining x faces go to one wave and the 16 remaining y
    // faces to another (wave-uniform branches), two different waves from
    // block to block, so that no wave takes more than three faces
    const int wave = tid >> 6, lane16 = tid & 15;
    const bool xextra = wave == (bi & 3) && (tid & 63) < 16;
    const bool yextra = wave == ((bi + 2) & 3) && (tid & 63) < 16;

    unsigned long long sm = 0, cm = 0;
    const int cf = Dsc->cf_coarse;
    for (int k = 0; k < BN; ++k) {
        // (1) z face k+1/2, then the x and y faces of plane k
        R Fhi[NV];
        {
            R wk2[NV], wR[NV], wLn[NV];
            prim_z(C2, wk2);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const R d1 = wk1[v] - wk[v], d2 = wk2[v] - wk1[v];
                const R s1 = minmod(d1, d2);
                wR[v] = wk1[v] - R(0.5) * s1;
                wLn[v] = wk1[v] + R(0.5) * s1;
            }
            mhd_hll<R>(wLz, wR, gammaR, igm1R, chR, inv2chR, Fhi);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                wLz[v] = wLn[v];
                wk[v] = wk1[v];
                wk1[v] = wk2[v];
            }
        }
        face_task(std::integral_constant<int, 0>(), tid, k);
        face_task(std::integral_constant<int, 1>(), tid, k);
        if (xextra) face_task(std::integral_constant<int, 0>(), 256 + lane16, k);
        if (yextra) face_task(std::integral_constant<int, 1>(), 256 + lane16, k);
        __syncthreads();

        // (2) update of cell (i, j, k); the next cell of the window, the next
        // plane's ghosts and primitives
        {
            double C0[NV], Un[NV], G[NV], Cn[NV];
            if (RING) {
#pragma unroll
                for (int v = 0; v < NV; ++v) C0[v] = Ck[v];
            } else {
                zload(k, C0);
            }
            if (STAGE == 2) {
#pragma unroll
                for (int v = 0; v < NV; ++v) Un[v] = load_un(a.Un + blk + v * CELLS + k * 256 + colp);
            }
            zload(min(k + 3, BN + NG - 1), RING ? Cn : C2);
            // z fluxes back to the global variable order
            const double fz[NV] = {double(Fhi[0]) - double(Flo[0]), double(Fhi[2]) - double(Flo[2]),
                                   double(Fhi[3]) - double(Flo[3]), double(Fhi[1]) - double(Flo[1]),
                                   double(Fhi[4]) - double(Flo[4]), double(Fhi[6]) - double(Flo[6]),
                                   double(Fhi[7]) - double(Flo[7]), double(Fhi[5]) - double(Flo[5]),
                                   double(Fhi[8]) - double(Flo[8])};
            const size_t cell = blk + size_t(k) * 256 + colp;
            // cells on a face where a flux correction follows (coarse side of
            // a level jump): left out of the signal maxima and the decay here
            const bool skip = STAGE == 2 &&
                              (((cf & 1) && i == 0) || ((cf & 2) && i == BN - 1) || ((cf & 4) && j == 0) ||
                               ((cf & 8) && j == BN - 1) || ((cf & 16) && k == 0) || ((cf & 32) && k == BN - 1));
            double out[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double dfx = double(sF[v][j * NF + i + 1]) - double(sF[v][j * NF + i]);
                const double dfy = double(sF[v][NXY + i * NF + j + 1]) - double(sF[v][NXY + i * NF + j]);
                const double L = -((dfx + dfy) + fz[v]) * inv_dx;
                if (STAGE == 1) out[v] = C0[v] + dt * L;
                else out[v] = 0.5 * (Un[v] + (C0[v] + dt * L));
                if (STAGE == 2 && v == 8 && !skip) out[v] = out[v] * fdec;
                store_out(a.Uout + cell + size_t(v) * CELLS, out[v]);
                if (xcol) store_out(xo + size_t(k) * 32 + v * 2 * SLAB, out[v]);   // the x-boundary copy
            }
            gload(min(k + 1, BN - 1), G);
            if (STAGE == 2) {
                bool ok2;
                double c;
                const double sg = mhd_signal(out, gamma, inv_dx, c, ok2);
                ok &= ok2;
                if (!skip) {
                    const unsigned long long sb = __double_as_longlong(sg), cb = __double_as_longlong(c);
                    sm = sb > sm ? sb : sm;
                    cm = cb > cm ? cb : cm;
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) Flo[v] = Fhi[v];
            if (RING) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Ck[v] = Ck1[v];
                    Ck1[v] = C2[v];
                    C2[v] = Cn[v];
                }
            }
            // plane k's primitives were read before the barrier above: the
            // buffer takes plane k+1 (wk now holds the primitives of cell k+1)
            put_plane(wk, G);
        }
        __syncthreads();   // plane k+1 complete; plane k's fluxes read
    }
    if (Dsc->freg[5] >= 0) {   // z flux register of face 15+1/2
        double *r = a.freg + size_t(Dsc->freg[5]) * NV * REG + colp;
        r[0] = double(Flo[0]); r[REG] = double(Flo[2]); r[2 * REG] = double(Flo[3]); r[3 * REG] = double(Flo[1]);
        r[4 * REG] = double(Flo[4]); r[5 * REG] = double(Flo[6]); r[6 * REG] = double(Flo[7]);
        r[7 * REG] = double(Flo[5]); r[8 * REG] = double(Flo[8]);
    }
    if (!ok) atomicOr(&mp.flags, 1);
    if (STAGE == 2) {
        sm = wave_max_u64(sm);
        cm = wave_max_u64(cm);
        if ((tid & 63) == 0) {
            sMax[0][tid >> 6] = sm;
            sMax[1][tid >> 6] = cm;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long r = sMax[0][0], rc = sMax[1][0];
            for (int w = 1; w < 4; ++w) {
                r = sMax[0][w] > r ? sMax[0][w] : r;
                rc = sMax[1][w] > rc ? sMax[1][w] : rc;
            }
            atomicMax(&a.smax[b], r);
            atomicMax(&a.cmax[b], rc);
        }
    }
}

// psi <- psi exp(-h c_h alpha / dx) for the listed blocks (exact solution of
// the GLM damping term over a time h), and in the x-boundary copy XE.  One
// workgroup per block: the factor once, then the block's 4096 psi values as
// 16-byte pairs, 4 KB per round of the 256 lanes, with streaming hints (each
// value is read and written once); the pairs (0,1) and (14,15) of a row also
// go to XE.
typedef double v2d __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_glm_decay(const BlockDesc *desc, MeshParams *mp, double *U, double *XE,
                                                   const int *list, int nblocks, double hfrac) {
    const int bi = blockIdx.x;
    if (bi >= nblocks) return;
    const int b = list ? list[bi] : bi;
    const BlockDesc D = desc[b];
    const MeshParams &P = mp[D.mesh];
    const double inv_dx = P.inv_dx1 * double(1 << (D.level - 1));
    const double h = hfrac * P.dt;
    const double f = exp(-h * P.ch * P.glm_alpha * inv_dx);
    v2d *psi = reinterpret_cast<v2d *>(U + (size_t(b) * NV + 8) * CELLS);
    double *xe = XE ? XE + (size_t(b) * NV + 8) * 2 * SLAB : nullptr;
#pragma unroll
    for (int r = 0; r < CELLS / 512; ++r) {
        const int q = threadIdx.x + 256 * r;   // cells 2q, 2q + 1: pair q & 7 of row q >> 3 (row = k * 16 + j)
        v2d x = __builtin_nontemporal_load(psi + q);
        x.x *= f;
        x.y *= f;
        __builtin_nontemporal_store(x, psi + q);
        const int ip = q & 7;
        if (xe && (ip == 0 || ip == 7)) *reinterpret_cast<v2d *>(xe + (ip == 7) * SLAB + (q >> 3) * 2) = x;
    }
}

hipError_t launch_mhd_stage(const SweepArgs &a, int stage, int precision, hipStream_t s) {
    if (a.nblocks <= 0) return hipSuccess;
    const dim3 grid(a.nblocks), block(256);
    if (precision == 0) {
        if (stage == 1) hipLaunchKernelGGL((k_mhd_stage<1, double>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_mhd_stage<2, double>), grid, block, 0, s, a);
    } else {
        if (stage == 1) hipLaunchKernelGGL((k_mhd_stage<1, float>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_mhd_stage<2, float>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_glm_decay(const BlockDesc *desc, MeshParams *mp, double *U, double *XE, const int *list,
                            int nblocks, double hfrac, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_glm_decay, dim3(nblocks), dim3(256), 0, s, desc, mp, U, XE, list, nblocks, hfrac);
    return hipGetLastError();
}

} // namespace agile
