// mhd.hip -- gfx950 kernels of the ideal-MHD + GLM stage update (Sec. 2.3.3),
// nvar 9: (rho, m, e, B, psi).
//
// A stage is two launches over (block, z-plane) work items, 256 lanes (4
// wave64) each:
//   - k_mhd_xy: the x and y faces of the plane (PLM minmod on primitives, GLM
//     interface step and HLL flux, mhd_hll), flux registers at block faces
//     that carry one, and dFx + dFy of every cell into an accumulator;
//   - k_mhd_sweep<2>: the z lines of a y-plane with their ghosts, the z
//     faces, L = -((dFx + dFy) + dFz)/dx, the SSP-RK2 stage combination, the
//     stage output and, in stage 2, the exact signal rate and GLM speed of
//     the new state (cells about to be flux-corrected excepted).
// The sweep kernel is written for any direction D (line loads, rotation to
// the frame (n, t1, t2) = cyclic(D)); only D = 2 is launched.
// The GLM source is split off exactly: psi decays by exp(-dt/2 c_h alpha/dx)
// before and after the two stages (k_glm_decay).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "agile_internal.hpp"
#include "device_math.hpp"

namespace agile {

namespace {

constexpr int NV = 9;
constexpr int NP = BN + 2 * NG;   // 20 cells per line with ghosts
constexpr int NF = BN + 1;        // 17 faces per line

// block-local cell index of line l, position i along D, plane q
template <int D>
__device__ __forceinline__ int cell_of(int l, int i, int q) {
    if (D == 0) return (q * 16 + l) * 16 + i;    // (x = i, y = l, z = q)
    if (D == 1) return (q * 16 + i) * 16 + l;    // (x = l, y = i, z = q)
    return (i * 16 + q) * 16 + l;                // (x = l, y = q, z = i)
}

} // namespace

template <int D, int STAGE, typename R>
__global__ __launch_bounds__(256) void k_mhd_sweep(SweepArgs a) {
    __shared__ R sW[NV][BN][NP];
    __shared__ R sF[NV][BN][NF];
    __shared__ unsigned long long sMax[2][4];
    const int bi = blockIdx.x >> 4, q = blockIdx.x & 15;
    if (bi >= a.nblocks) return;
    const int b = a.list ? a.list[bi] : bi;
    const int tid = threadIdx.x;
    const BlockDesc Dsc = a.desc[b];
    MeshParams &mp = a.mp[Dsc.mesh];
    const double gamma = mp.gamma, gm1 = gamma - 1.0;
    const double inv_dx = mp.inv_dx1 * double(1 << (Dsc.level - 1));
    const double ch = mp.ch;
    const R gammaR = R(gamma), igm1R = R(1.0 / gm1), chR = R(ch), inv2chR = R(0.5 / ch);
    const size_t blk = size_t(b) * NV * CELLS;
    constexpr int n1 = (D + 1) % 3, n2 = (D + 2) % 3;
    bool ok = true;

    // (1) the plane's lines with ghosts -> rotated primitives in LDS
    for (int e = tid; e < BN * NP; e += 256) {
        int l, p;
        if (D == 0) { l = e / NP; p = e - NP * l - NG; }
        else { p = e / BN - NG; l = e - BN * (p + NG); }
        const double *src;
        int st;
        if (p >= 0 && p < BN) {
            src = a.Uin + blk + cell_of<D>(l, p, q);
            st = CELLS;
        } else {
            const int side = p >= BN;
            const int nb = Dsc.nb[2 * D + side];
            if (nb >= 0) {
                src = a.Uin + size_t(nb) * NV * CELLS + cell_of<D>(l, side ? p - BN : p + BN, q);
                st = CELLS;
            } else {
                src = a.halo + size_t(-nb - 1) * NV * SLAB + slab_index(D, side ? p - BN : p + NG, l, q);
                st = SLAB;
            }
        }
        double U[NV], w[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = src[v * st];
        ok &= mhd_cons2prim(U, gm1, w);
        const int pp = p + NG;
        sW[0][l][pp] = R(w[0]);
        sW[1][l][pp] = R(w[1 + D]);
        sW[2][l][pp] = R(w[1 + n1]);
        sW[3][l][pp] = R(w[1 + n2]);
        sW[4][l][pp] = R(w[4]);
        sW[5][l][pp] = R(w[5 + D]);
        sW[6][l][pp] = R(w[5 + n1]);
        sW[7][l][pp] = R(w[5 + n2]);
        sW[8][l][pp] = R(w[8]);
    }
    __syncthreads();

    // (2) faces: line l, face i (between positions i-1 and i)
    for (int f = tid; f < BN * NF; f += 256) {
        const int l = f / NF, i = f - NF * l;
        R wL[NV], wR[NV], F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const R c0 = sW[v][l][i], c1 = sW[v][l][i + 1], c2 = sW[v][l][i + 2], c3 = sW[v][l][i + 3];
            const R d0 = c1 - c0, d1 = c2 - c1, d2 = c3 - c2;
            wL[v] = c1 + R(0.5) * minmod(d0, d1);
            wR[v] = c2 - R(0.5) * minmod(d1, d2);
        }
        mhd_hll<R>(wL, wR, gammaR, igm1R, chR, inv2chR, F);
        // back to the global variable order
        R G[NV];
        G[0] = F[0]; G[1 + D] = F[1]; G[1 + n1] = F[2]; G[1 + n2] = F[3]; G[4] = F[4];
        G[5 + D] = F[5]; G[5 + n1] = F[6]; G[5 + n2] = F[7]; G[8] = F[8];
#pragma unroll
        for (int v = 0; v < NV; ++v) sF[v][l][i] = G[v];
        if (i == 0 || i == BN) {
            const int slot = Dsc.freg[2 * D + (i == BN)];
            if (slot >= 0) {
                double *r = a.freg + size_t(slot) * NV * REG + q * 16 + l;
#pragma unroll
                for (int v = 0; v < NV; ++v) r[v * REG] = double(G[v]);
            }
        }
    }
    __syncthreads();

    // (3) cells: flux difference along D; the z sweep completes the stage
    int l, i;
    if (D == 0) { i = tid & 15; l = tid >> 4; }
    else { l = tid & 15; i = tid >> 4; }
    const size_t cell = blk + cell_of<D>(l, i, q);
    unsigned long long sm = 0, cm = 0;
    if (D < 2) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double df = double(sF[v][l][i + 1]) - double(sF[v][l][i]);
            double *acc = a.acc + cell + size_t(v) * CELLS;
            *acc = D == 0 ? df : *acc + df;
        }
    } else {
        if (STAGE == 1 && q == 0 && tid == 0) {
            a.smax[b] = 0;
            a.cmax[b] = 0;
        }
        const double dt = mp.dt;
        double out[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double df = double(sF[v][l][i + 1]) - double(sF[v][l][i]);
            const double L = -(a.acc[cell + size_t(v) * CELLS] + df) * inv_dx;
            const double u = a.Uin[cell + size_t(v) * CELLS];
            if (STAGE == 1) out[v] = u + dt * L;
            else out[v] = 0.5 * (a.Un[cell + size_t(v) * CELLS] + (u + dt * L));
            a.Uout[cell + size_t(v) * CELLS] = out[v];
        }
        if (STAGE == 2) {
            // cell (x = l, y = q, z = i)
            const int cf = Dsc.cf_coarse;
            const bool skip = ((cf & 1) && l == 0) || ((cf & 2) && l == BN - 1) || ((cf & 4) && q == 0) ||
                              ((cf & 8) && q == BN - 1) || ((cf & 16) && i == 0) || ((cf & 32) && i == BN - 1);
            bool ok2;
            double c;
            const double s = mhd_signal(out, gamma, inv_dx, c, ok2);
            ok &= ok2;
            if (!skip) {
                sm = __double_as_longlong(s);
                cm = __double_as_longlong(c);
            }
        }
    }
    if (!ok) atomicOr(&mp.flags, 1);
    if (D == 2 && STAGE == 2) {
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

// The x and y sweeps of one (block, z-plane) in one workgroup (256 lanes):
//   - the plane's 16 x 16 cells and its 128 x / y ghost cells are loaded,
//     turned into primitives and kept in LDS in the global variable order
//     (a 20 x 20 plane; its corners are never read);
//   - x faces (16 rows x 17), one lane per face: PLM minmod and the GLM /
//     HLL flux in the frame (x, y, z), fluxes in LDS; each lane keeps the x
//     flux difference of its cell in registers;
//   - y faces (16 columns x 17) in the frame (y, z, x) through the same flux
//     buffer; the lane stores dFx + dFy of its cell into the accumulator.
// Same expressions as the separate x and y sweeps, so the accumulator holds
// the same numbers; the U plane is read once and the accumulator written
// once instead of read, written and re-read.  48 KB of LDS (FP64): three
// workgroups per CU.
template <typename R>
__global__ __launch_bounds__(256) void k_mhd_xy(SweepArgs a) {
    constexpr int PW = BN + 2 * NG;   // 20
    __shared__ R sW[NV][PW][PW];
    __shared__ R sF[NV][BN * NF];
    const int bi = blockIdx.x >> 4, q = blockIdx.x & 15;
    if (bi >= a.nblocks) return;
    const int b = a.list ? a.list[bi] : bi;
    const int tid = threadIdx.x;
    // the descriptor is read through its pointer: a local copy indexed by a
    // lane's face would live in scratch
    const BlockDesc *Dsc = a.desc + b;
    MeshParams &mp = a.mp[Dsc->mesh];
    const double gamma = mp.gamma, gm1 = gamma - 1.0;
    const double ch = mp.ch;
    const R gammaR = R(gamma), igm1R = R(1.0 / gm1), chR = R(ch), inv2chR = R(0.5 / ch);
    const size_t blk = size_t(b) * NV * CELLS;
    bool ok = true;

    // (1) 256 interior cells, then 128 ghost cells (4 faces x 2 layers x 16)
    for (int e = tid; e < BN * BN + 8 * BN; e += 256) {
        int x, y;
        const double *src;
        int st;
        if (e < BN * BN) {
            x = e & 15;
            y = e >> 4;
            src = a.Uin + blk + (q * 16 + y) * 16 + x;
            st = CELLS;
        } else {
            const int g = e - BN * BN, f = g >> 5, r = g & 31;
            const int d = f >> 1, side = f & 1;
            int gl, t;   // ghost layer (0 nearest the low side) and tangential index
            if (d == 0) { gl = r & 1; t = r >> 1; }
            else { gl = r >> 4; t = r & 15; }
            const int p = side ? BN + gl : gl - NG;   // position along d
            x = d == 0 ? p : t;
            y = d == 0 ? t : p;
            const int nb = Dsc->nb[f];
            if (nb >= 0) {
                const int xn = d == 0 ? (side ? p - BN : p + BN) : x;
                const int yn = d == 0 ? y : (side ? p - BN : p + BN);
                src = a.Uin + size_t(nb) * NV * CELLS + (q * 16 + yn) * 16 + xn;
                st = CELLS;
            } else {
                src = a.halo + size_t(-nb - 1) * NV * SLAB + slab_index(d, side ? p - BN : p + NG, t, q);
                st = SLAB;
            }
        }
        double U[NV], w[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = src[v * st];
        ok &= mhd_cons2prim(U, gm1, w);
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v][y + NG][x + NG] = R(w[v]);
    }
    __syncthreads();

    // faces of direction D (0: x, 1: y): face (l, i) lies on line l before
    // position i; the flux is stored at l * NF + i in the global order
    auto faces = [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        constexpr int n1 = (D + 1) % 3, n2 = (D + 2) % 3;
        for (int f = tid; f < BN * NF; f += 256) {
            const int l = f / NF, i = f - NF * l;
            R c[4][NV];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int yy = D == 0 ? l + NG : i + s, xx = D == 0 ? i + s : l + NG;
                c[s][0] = sW[0][yy][xx];
                c[s][1] = sW[1 + D][yy][xx];
                c[s][2] = sW[1 + n1][yy][xx];
                c[s][3] = sW[1 + n2][yy][xx];
                c[s][4] = sW[4][yy][xx];
                c[s][5] = sW[5 + D][yy][xx];
                c[s][6] = sW[5 + n1][yy][xx];
                c[s][7] = sW[5 + n2][yy][xx];
                c[s][8] = sW[8][yy][xx];
            }
            R wL[NV], wR[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const R d0 = c[1][v] - c[0][v], d1 = c[2][v] - c[1][v], d2 = c[3][v] - c[2][v];
                wL[v] = c[1][v] + R(0.5) * minmod(d0, d1);
                wR[v] = c[2][v] - R(0.5) * minmod(d1, d2);
            }
            mhd_hll<R>(wL, wR, gammaR, igm1R, chR, inv2chR, F);
            R G[NV];
            G[0] = F[0]; G[1 + D] = F[1]; G[1 + n1] = F[2]; G[1 + n2] = F[3]; G[4] = F[4];
            G[5 + D] = F[5]; G[5 + n1] = F[6]; G[5 + n2] = F[7]; G[8] = F[8];
#pragma unroll
            for (int v = 0; v < NV; ++v) sF[v][f] = G[v];
            if (i == 0 || i == BN) {
                const int slot = Dsc->freg[2 * D + (i == BN)];
                if (slot >= 0) {
                    double *r = a.freg + size_t(slot) * NV * REG + q * 16 + l;
#pragma unroll
                    for (int v = 0; v < NV; ++v) r[v * REG] = double(G[v]);
                }
            }
        }
    };
    const int cx = tid & 15, cy = tid >> 4;   // this lane's cell
    faces(std::integral_constant<int, 0>());
    __syncthreads();
    double dfx[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) dfx[v] = double(sF[v][cy * NF + cx + 1]) - double(sF[v][cy * NF + cx]);
    __syncthreads();
    faces(std::integral_constant<int, 1>());
    __syncthreads();
    const size_t cell = blk + (q * 16 + cy) * 16 + cx;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double dfy = double(sF[v][cx * NF + cy + 1]) - double(sF[v][cx * NF + cy]);
        a.acc[cell + size_t(v) * CELLS] = dfx[v] + dfy;
    }
    if (!ok) atomicOr(&mp.flags, 1);
}

// psi <- psi exp(-h c_h alpha / dx) for the listed blocks (exact solution of
// the GLM damping term over a time h)
__global__ __launch_bounds__(256) void k_glm_decay(const BlockDesc *desc, MeshParams *mp, double *U, const int *list,
                                                   int nblocks, double hfrac) {
    const int bi = blockIdx.x >> 4, part = blockIdx.x & 15;
    if (bi >= nblocks) return;
    const int b = list ? list[bi] : bi;
    const BlockDesc D = desc[b];
    const MeshParams &P = mp[D.mesh];
    const double inv_dx = P.inv_dx1 * double(1 << (D.level - 1));
    const double h = hfrac * P.dt;
    const double f = exp(-h * P.ch * P.glm_alpha * inv_dx);
    double *psi = U + (size_t(b) * NV + 8) * CELLS + part * 256;
    psi[threadIdx.x] *= f;
}

hipError_t launch_mhd_stage(const SweepArgs &a, int stage, int precision, hipStream_t s) {
    if (a.nblocks <= 0) return hipSuccess;
    const dim3 grid(a.nblocks * 16), block(256);
#define AGILE_MHD_SWEEPS(ST, R)                                            \
    do {                                                                   \
        hipLaunchKernelGGL((k_mhd_xy<R>), grid, block, 0, s, a);           \
        hipLaunchKernelGGL((k_mhd_sweep<2, ST, R>), grid, block, 0, s, a); \
    } while (0)
    if (precision == 0) {
        if (stage == 1) AGILE_MHD_SWEEPS(1, double);
        else AGILE_MHD_SWEEPS(2, double);
    } else {
        if (stage == 1) AGILE_MHD_SWEEPS(1, float);
        else AGILE_MHD_SWEEPS(2, float);
    }
#undef AGILE_MHD_SWEEPS
    return hipGetLastError();
}

hipError_t launch_glm_decay(const BlockDesc *desc, MeshParams *mp, double *U, const int *list, int nblocks,
                            double hfrac, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_glm_decay, dim3(nblocks * 16), dim3(256), 0, s, desc, mp, U, list, nblocks, hfrac);
    return hipGetLastError();
}

} // namespace agile
