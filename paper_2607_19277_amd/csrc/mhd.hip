// mhd.hip -- gfx950 kernels of the ideal-MHD + GLM stage update (Sec. 2.3.3),
// nvar 9: (rho, m, e, B, psi).
//
// A stage is three directional sweeps.  One workgroup (256 lanes = 4 wave64)
// takes one (block, plane) and one sweep axis D:
//   - the plane's 16 lines along D plus the 2 ghost cells at each end are
//     loaded row by row (x rows are contiguous in every sweep: the x and y
//     sweeps take z-planes, the z sweep y-planes), turned into primitives and
//     stored in LDS in a frame rotated to the normal (n, t1, t2) = cyclic(D);
//   - one lane per face (16 x 17 faces): minmod-limited PLM on the
//     primitives, GLM interface step and HLL flux (mhd_hll), flux kept in
//     LDS and, at block faces that carry a flux register, in the register;
//   - one lane per cell: the flux difference along D is added to the
//     accumulator (x: stored, y: added); the z sweep adds its own, forms
//     L = -((dFx + dFy) + dFz)/dx, the SSP-RK2 stage combination, writes the
//     stage output and, in stage 2, reduces the exact signal rate and the GLM
//     speed of the new state (cells about to be flux-corrected excepted).
// The GLM source is split off exactly: psi decays by exp(-dt/2 c_h alpha/dx)
// before and after the two stages (k_glm_decay).
#include <hip/hip_runtime.h>

#include <cstdint>

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
        hipLaunchKernelGGL((k_mhd_sweep<0, ST, R>), grid, block, 0, s, a); \
        hipLaunchKernelGGL((k_mhd_sweep<1, ST, R>), grid, block, 0, s, a); \
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
