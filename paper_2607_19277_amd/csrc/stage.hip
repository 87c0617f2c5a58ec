// stage.hip -- the fused SSP Runge-Kutta stage update of one 16^3 block per
// workgroup on gfx950 (the paper's macro-kernel, Sec. 2.1.3, re-designed for
// CDNA4), for the Euler equations (HLL, HLLC, LF) and the SRHD module (LF;
// its con2prim per cell and ghost), with minmod or van Leer slopes.
//
// 256 lanes = 4 wave64; lane (i, j) owns the z-column (i, j) of the block.
// The block is marched plane by plane in z (2.5-D):
//   - the conserved values of the column are streamed through a register
//     ring (cells k, k+1, k+2) with the next cell (k+3) and the next plane's
//     x/y ghosts prefetched one iteration ahead, so each interior value is
//     read from HBM once per stage;
//   - z faces: each lane keeps the primitives of cells k, k+1 and the left
//     PLM state of face k+1/2, and computes one z-face flux per plane;
//   - x/y faces of plane k: the plane's primitives (interior + 2 ghost
//     columns / rows) go to LDS (double-buffered: plane k+1 is written while
//     plane k's faces are computed, one barrier per plane) and 544 face tasks
//     (272 x, 272 y) are spread over the lanes; each face flux is computed exactly once (the paper
//     evaluates both faces of every cell) and in a frame rotated to the face
//     normal, so x and y faces run one instruction stream;
//   - update: L = -((dFx + dFy) + dFz)/dx, then
//     SSP-RK2 stage 1: U1 = U + dt L;  stage 2: U' = (U^n + (U1 + dt L))/2;
//     SSP-RK3: U1 = U + dt L, U2 = 3/4 U^n + 1/4 (U1 + dt L),
//     U' = 1/3 U^n + 2/3 (U2 + dt L); written with the x-boundary export and
//     the face fluxes kept for coarse-fine flux correction; the last stage
//     also reduces the CFL signal rate of the new state (cells to be
//     flux-corrected excepted).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "agile_internal.hpp"
#include "device_math.hpp"

namespace agile {

namespace {

constexpr int NV = 5;
constexpr int PW = BN + 2 * NG;      // 20: padded plane width
constexpr int PLANE = PW * PW;       // 400
constexpr int NXF = BN * (BN + 1);   // 272 x-face (and y-face) tasks per plane
constexpr int NTASK = 2 * NXF;       // 544

// Workgroups are dealt to the 8 XCDs of the chip round-robin.  With xcd = 1
// each XCD gets one contiguous range of work items (blocks in level + Morton
// order, slabs of a block adjacent) so that most same-level neighbours run on
// the same XCD and their boundary rows can be served from that XCD's L2.
__device__ __forceinline__ int xcd_item(int w, int n, int xcd) {
    if (!xcd) return w;
    const int chunk = (n + 7) >> 3;
    return (w & 7) * chunk + (w >> 3);
}
inline int xcd_grid(int n, int xcd) { return xcd ? 8 * ((n + 7) >> 3) : n; }

// primitives of a conserved state: Euler (rho, v, p), or for the SRHD
// module (RS = 3) (rho, Gamma v, p) from the root finding in xi
template <int RS>
__device__ __forceinline__ bool phys_prim(const double C[NV], double gamma, double gm1, double q[NV]) {
    if (RS == 3) return srhd_con2prim_fast(C, gamma, q);
    return cons2prim(C, gm1, q);
}

template <int RS, typename R>
__device__ __forceinline__ void to_prim_z(const double C[NV], double gamma, double gm1, R w[NV], bool &ok) {
    double q[NV];
    ok &= phys_prim<RS>(C, gamma, gm1, q);
    // rotated to the z normal: (rho, vz, vx, vy, p)
    w[0] = R(q[0]); w[1] = R(q[3]); w[2] = R(q[1]); w[3] = R(q[2]); w[4] = R(q[4]);
}

} // namespace

#ifndef AGILE_STAGE_WAVES_F64
#define AGILE_STAGE_WAVES_F64 2
#endif
#ifndef AGILE_STAGE_WAVES_F32
#define AGILE_STAGE_WAVES_F32 3
#endif

// RS: 0 HLL, 1 HLLC, 2 local Lax-Friedrichs, 3 the SRHD module (local
// Lax-Friedrichs on (rho, Gamma v, p)); LIM: 0 minmod, 1 van Leer;
// KIND: 1 first stage (U1 = U + dt L), 2 last SSP-RK2 stage
// ((U^n + (U1 + dt L))/2), 3 middle SSP-RK3 stage (3/4 U^n + 1/4 (U1 + dt L)),
// 4 last SSP-RK3 stage (1/3 U^n + 2/3 (U2 + dt L)).  The last stage of a step
// also reduces the signal rate of the new state.
template <int RS, int LIM, int KIND, typename R>
__global__ __launch_bounds__(256, sizeof(R) == 8 ? AGILE_STAGE_WAVES_F64 : AGILE_STAGE_WAVES_F32) void k_stage(StageArgs a) {
    constexpr bool FIRST = KIND == 1, LAST = KIND == 2 || KIND == 4;
    // plane primitives and x/y face fluxes, double-buffered by plane parity so
    // that one barrier per plane separates producers from consumers
    __shared__ R sP[2][NV][PLANE];
    __shared__ R sF[2][NV][NTASK];
    __shared__ unsigned long long sMax[4];

    // work item = (block, slab of kslab planes)
    const int nslab = BN / a.kslab;
    const int item = xcd_item(blockIdx.x, a.nblocks * nslab, a.xcd);
    if (item >= a.nblocks * nslab) return;
    const int bi = item / nslab, slab = item - bi * nslab;
    const int b = a.list ? a.list[bi] : bi;
    const int k0 = slab * a.kslab, k1 = k0 + a.kslab;
    const int tid = threadIdx.x;
    const int i = tid & 15, j = tid >> 4;
    const BlockDesc D = a.desc[b];
    MeshParams &mp = a.mp[D.mesh];
    const double gamma = mp.gamma;
    const double gm1 = gamma - 1.0;
    const R gammaR = R(gamma), igm1R = R(1.0 / gm1);
    const double inv_dx = mp.inv_dx1 * double(1 << (D.level - 1));
    const double dt = mp.dt;
    const size_t blk = size_t(b) * NV * CELLS;
    const double *Ub = a.Uin + blk;
    const int colp = j * 16 + i;
    const int pown = (j + 2) * PW + i + 2;   // LDS position of this lane's own cell
    bool ok = true;

    // conserved value source of this column's cell at z index kk in [-2, 18)
    auto zload = [&](int kk, double C[NV]) {
        const double *p;
        int st;
        if (kk >= 0 && kk < BN) {
            p = Ub + kk * 256 + colp;
            st = CELLS;
        } else {
            const int nb = kk < 0 ? D.nb[4] : D.nb[5];
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
    // x / y ghost cells of a plane: 32 per face, lanes 0..127; lanes 128..255
    // repeat the same cells (same loads, same LDS slots and values), which
    // keeps the plane loop free of branches
    const int gf = (tid >> 5) & 3, gr = tid & 31;
    int glp;   // LDS position of this lane's ghost cell
    if (gf < 2) glp = ((gr >> 1) + 2) * PW + (gf == 0 ? (gr & 1) : BN + NG + (gr & 1));
    else glp = (gf == 2 ? (gr >> 4) : BN + NG + (gr >> 4)) * PW + (gr & 15) + 2;
    const int gnb = gf == 0 ? D.nb[0] : (gf == 1 ? D.nb[1] : (gf == 2 ? D.nb[2] : D.nb[3]));
    auto gload = [&](int k, double G[NV]) {
        const double *p;
        int st;
        if (gnb < 0) {
            p = a.halo + size_t(-gnb - 1) * NV * SLAB + k * 32 + gr;
            st = SLAB;
        } else if (gf < 2) {
            p = a.XEin + (size_t(gnb) * NV * 2 + (gf == 0 ? 1 : 0)) * SLAB + k * 32 + gr;
            st = 2 * SLAB;
        } else {
            p = a.Uin + size_t(gnb) * NV * CELLS + k * 256 + (gf == 2 ? 224 : 0) + gr;
            st = CELLS;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) G[v] = p[v * st];
    };
    // SRHD ghosts: the con2prim is an iteration, and lanes 128.. would only
    // repeat the ghost cells of lanes 0..127.  There, on even planes k lanes
    // 0..127 convert the ghosts of plane k+1 and lanes 128.. those of plane
    // k+2, which they keep (in G) and store on the odd plane k+1, when that
    // LDS buffer is free; odd planes convert no ghost.  Each wave then does
    // 1.5 con2prims per plane instead of 2.
    const int gB = (RS == 3 && tid >= 128) ? 1 : 0;
    // write a plane into LDS buffer `buf`: own cell (z-rotated primitives)
    // and one ghost cell from its conserved values.  mode 0: every lane
    // converts and stores its ghost; SRHD mode 1 (even plane): convert, lanes
    // 128.. keep the result in G; mode 2 (odd plane): lanes 128.. store G.
    auto put_plane = [&](int buf, const R w[NV], double G[NV], int mode) {
        sP[buf][0][pown] = w[0]; sP[buf][1][pown] = w[2]; sP[buf][2][pown] = w[3];
        sP[buf][3][pown] = w[1]; sP[buf][4][pown] = w[4];
        if (mode != 2) {
            double q[NV];
            ok &= phys_prim<RS>(G, gamma, gm1, q);
            if (mode == 1 && gB) {
#pragma unroll
                for (int v = 0; v < NV; ++v) G[v] = q[v];
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) sP[buf][v][glp] = R(q[v]);
            }
        } else if (gB) {
#pragma unroll
            for (int v = 0; v < NV; ++v) sP[buf][v][glp] = R(G[v]);
        }
    };

    // ---- prologue: cells k0-2 .. k0+2 of the column, face k0-1/2, plane k0 in
    // LDS.  Its expressions are the loop body's; the library is built with
    // per-expression contraction only, so each expression rounds the same way
    // wherever it is compiled and results do not depend on the slab shape.
    double C0[NV], C1[NV], C2[NV], Cn[NV], Gn[NV], Gn2[NV];
    R wk[NV], wk1[NV], wLz[NV], Flo[NV], Fhi[NV];
    {
        double Cm2[NV], Cm1[NV], G0[NV];
        zload(k0 - 2, Cm2);
        zload(k0 - 1, Cm1);
        zload(k0, C0);
        zload(k0 + 1, C1);
        zload(k0 + 2, C2);
        gload(k0, G0);
        gload(min(k0 + 1 + gB, k1 - 1), Gn);
        R wm2[NV], wm1[NV], wL[NV], wR[NV];
        to_prim_z<RS>(Cm2, gamma, gm1, wm2, ok);
        to_prim_z<RS>(Cm1, gamma, gm1, wm1, ok);
        to_prim_z<RS>(C0, gamma, gm1, wk, ok);
        to_prim_z<RS>(C1, gamma, gm1, wk1, ok);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const R sm = slope<LIM>(wm1[v] - wm2[v], wk[v] - wm1[v]);
            wL[v] = wm1[v] + R(0.5) * sm;
            const R s0 = slope<LIM>(wk[v] - wm1[v], wk1[v] - wk[v]);
            wR[v] = wk[v] - R(0.5) * s0;
            wLz[v] = wk[v] + R(0.5) * s0;
        }
        riemann<RS, R>(wL, wR, gammaR, igm1R, Flo);
        put_plane(k0 & 1, wk, G0, 0);
    }
    if (k0 == 0 && D.freg[4] >= 0) {
        double *r = a.freg + size_t(D.freg[4]) * NV * REG + colp;
        r[0] = double(Flo[0]); r[REG] = double(Flo[2]); r[2 * REG] = double(Flo[3]);
        r[3 * REG] = double(Flo[1]); r[4 * REG] = double(Flo[4]);
    }
    __syncthreads();

    const int tt = (tid + 64 * (item & 3)) & 255;   // rotate the extra x/y face tasks over the waves
    unsigned long long smax = 0;
    const int cf = D.cf_coarse;
    if (FIRST && slab == 0 && tid == 0) a.smax[b] = 0;   // the last stage takes the maximum

    // One plane of the march.  The body has no branch before the barrier
    // except the third face task: loads past the slab re-read its last valid
    // cell or ghost row, and the last plane writes an unused LDS plane, so the
    // z face, the plane store and the first two x/y tasks form one scheduling
    // region.
    auto plane = [&](const int k) __attribute__((always_inline)) {
        const int cur = k & 1, nxt = cur ^ 1;
        // SRHD: ghosts load on odd planes only (see put_plane)
        const bool gl = RS != 3 || cur == 1;
        // prefetch: z cell k+3, ghosts of plane k+2 (SRHD lanes 128..: k+3),
        // U^n of plane k (stage 2)
        zload(min(k + 3, k1 + NG - 1), Cn);
        if (gl) gload(min(k + 2 + gB, k1 - 1), Gn2);
        double Un[NV];

        // (A) z face k+1/2, and plane k+1 into the other LDS buffer
        {
            R wk2[NV], wR[NV], wLn[NV];
            to_prim_z<RS>(C2, gamma, gm1, wk2, ok);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const R s1 = slope<LIM>(wk1[v] - wk[v], wk2[v] - wk1[v]);
                wR[v] = wk1[v] - R(0.5) * s1;
                wLn[v] = wk1[v] + R(0.5) * s1;
            }
            riemann<RS, R>(wLz, wR, gammaR, igm1R, Fhi);
            put_plane(nxt, wk1, Gn, RS != 3 ? 0 : 1 + cur);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                wLz[v] = wLn[v];
                wk[v] = wk1[v];
                wk1[v] = wk2[v];
            }
        }

        // (B) x and y faces of plane k: tasks [0, 272) x, [272, 544) y; every
        // lane takes tasks tt and tt + 256, lanes with tt < 32 also tt + 512
        auto face_task = [&](int t) {
            const int d = t >= NXF;
            const int u = t - NXF * d;
            int base, st;
            if (!d) {
                const int jj = u / 17, fi = u - 17 * jj;
                base = (jj + 2) * PW + fi;
                st = 1;
            } else {
                base = (u >> 4) * PW + (u & 15) + 2;
                st = PW;
            }
            R c[4][NV];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int p = base + s * st;
                c[s][0] = sP[cur][0][p];
                c[s][1] = sP[cur][1 + d][p];
                c[s][2] = sP[cur][2 - d][p];
                c[s][3] = sP[cur][3][p];
                c[s][4] = sP[cur][4][p];
            }
            R wL[NV], wR[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const R d0 = c[1][v] - c[0][v], d1 = c[2][v] - c[1][v], d2 = c[3][v] - c[2][v];
                wL[v] = c[1][v] + R(0.5) * slope<LIM>(d0, d1);
                wR[v] = c[2][v] - R(0.5) * slope<LIM>(d1, d2);
            }
            riemann<RS, R>(wL, wR, gammaR, igm1R, F);
            sF[cur][0][t] = F[0];
            sF[cur][1][t] = d ? F[2] : F[1];
            sF[cur][2][t] = d ? F[1] : F[2];
            sF[cur][3][t] = F[3];
            sF[cur][4][t] = F[4];
        };
        face_task(tt);
        face_task(tt + 256);
        if (tt < NTASK - 512) face_task(tt + 512);
        // U^n of plane k (its load crosses the barrier; issued here it is not
        // live during the face work)
        if (!FIRST) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Un[v] = load_un(a.Un + blk + v * CELLS + k * 256 + colp);
        }
        __syncthreads();

        // (C) divergence, stage combination, stores of plane k
        {
            const double fz[NV] = {double(Fhi[0]) - double(Flo[0]), double(Fhi[2]) - double(Flo[2]),
                                   double(Fhi[3]) - double(Flo[3]), double(Fhi[1]) - double(Flo[1]),
                                   double(Fhi[4]) - double(Flo[4])};
            const size_t cell = size_t(k) * 256 + colp;
            double out[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double dfx = double(sF[cur][v][j * 17 + i + 1]) - double(sF[cur][v][j * 17 + i]);
                const double dfy = double(sF[cur][v][NXF + (j + 1) * 16 + i]) - double(sF[cur][v][NXF + j * 16 + i]);
                const double L = -((dfx + dfy) + fz[v]) * inv_dx;
                if (KIND == 1) out[v] = C0[v] + dt * L;
                else if (KIND == 3) out[v] = 0.75 * Un[v] + 0.25 * (C0[v] + dt * L);
                else if (KIND == 4) out[v] = (1.0 / 3.0) * Un[v] + (2.0 / 3.0) * (C0[v] + dt * L);
                else out[v] = 0.5 * (Un[v] + (C0[v] + dt * L));
                store_out(a.Uout + blk + v * CELLS + cell, out[v]);
            }
            if (i < 2 || i >= BN - 2) {
                const int side = i >= BN - 2;
                double *x = a.XEout + (size_t(b) * NV * 2 + side) * SLAB + k * 32 + j * 2 + (i - (side ? BN - 2 : 0));
#pragma unroll
                for (int v = 0; v < NV; ++v) store_out(x + v * 2 * SLAB, out[v]);
            }
            if (LAST) {
                const bool skip = ((cf & 1) && i == 0) || ((cf & 2) && i == BN - 1) || ((cf & 4) && j == 0) ||
                                  ((cf & 8) && j == BN - 1) || ((cf & 16) && k == 0) || ((cf & 32) && k == BN - 1);
                bool ok2;
                const double s = RS == 3 ? srhd_signal(out, gamma, inv_dx, ok2) : signal_rate(out, gamma, inv_dx, ok2);
                ok &= ok2;
                const unsigned long long sb = __double_as_longlong(s);
                if (!skip && sb > smax) smax = sb;
            }
        }
        // flux registers of the x / y boundary faces of plane k
        if (tid < 32) {
            const int lane = tid & 15;
            const int fs = tid < 16 ? D.freg[0] : D.freg[2];   // -x / -y face register
            const int gs = tid < 16 ? D.freg[1] : D.freg[3];   // +x / +y face register
            const int lo = tid < 16 ? lane * 17 : NXF + lane;
            const int hi = tid < 16 ? lane * 17 + 16 : NXF + BN * 16 + lane;
            if (fs >= 0) {
                double *r = a.freg + size_t(fs) * NV * REG + k * 16 + lane;
#pragma unroll
                for (int v = 0; v < NV; ++v) r[v * REG] = double(sF[cur][v][lo]);
            }
            if (gs >= 0) {
                double *r = a.freg + size_t(gs) * NV * REG + k * 16 + lane;
#pragma unroll
                for (int v = 0; v < NV; ++v) r[v * REG] = double(sF[cur][v][hi]);
            }
        }
        // slide the conserved ring and the prefetched ghosts
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            C0[v] = C1[v];
            C1[v] = C2[v];
            C2[v] = Cn[v];
            if (gl) Gn[v] = Gn2[v];
            Flo[v] = Fhi[v];
        }
    };
    if (sizeof(R) == 8) {
        // two planes per trip (slabs have an even number of planes, starting
        // at an even plane): the register ring then needs about half the
        // moves, 6% fewer instructions per plane
        for (int k = k0; k < k1; k += 2) {
            __builtin_assume((k & 1) == 0);
            plane(k);
            __builtin_amdgcn_sched_barrier(0);
            plane(k + 1);
        }
    } else {
        // FP32 runs three waves per SIMD; the longer body would not fit
        for (int k = k0; k < k1; ++k) plane(k);
    }
    // flux register of the +z face (Flo holds the flux of face 15+1/2)
    if (k1 == BN && D.freg[5] >= 0) {
        double *r = a.freg + size_t(D.freg[5]) * NV * REG + colp;
        r[0] = double(Flo[0]); r[REG] = double(Flo[2]); r[2 * REG] = double(Flo[3]);
        r[3 * REG] = double(Flo[1]); r[4 * REG] = double(Flo[4]);
    }
    if (!ok) atomicOr(&mp.flags, 1);
    if (LAST) {
        smax = wave_max_u64(smax);
        if ((tid & 63) == 0) sMax[tid >> 6] = smax;
        __syncthreads();
        if (tid == 0) {
            unsigned long long m = sMax[0];
            for (int w = 1; w < 4; ++w) m = sMax[w] > m ? sMax[w] : m;
            atomicMax(&a.smax[b], m);
        }
    }
}

hipError_t launch_stage(const StageArgs &a, int riemann, int precision, hipStream_t s) {
    if (a.nblocks <= 0) return hipSuccess;
    if (a.kslab != 16 && a.kslab != 8 && a.kslab != 4) return hipErrorInvalidValue;
    if (a.stage < 1 || a.stage > 4 || riemann < 0 || riemann > 3 || a.limiter < 0 || a.limiter > 1)
        return hipErrorInvalidValue;
    const dim3 grid(xcd_grid(a.nblocks * (BN / a.kslab), a.xcd)), block(256);
#define AGILE_STAGE_KIND(RSV, LIMV, R)                                                        \
    do {                                                                                      \
        if (a.stage == 1) hipLaunchKernelGGL((k_stage<RSV, LIMV, 1, R>), grid, block, 0, s, a); \
        else if (a.stage == 2) hipLaunchKernelGGL((k_stage<RSV, LIMV, 2, R>), grid, block, 0, s, a); \
        else if (a.stage == 3) hipLaunchKernelGGL((k_stage<RSV, LIMV, 3, R>), grid, block, 0, s, a); \
        else hipLaunchKernelGGL((k_stage<RSV, LIMV, 4, R>), grid, block, 0, s, a);             \
    } while (0)
#define AGILE_STAGE_LIM(RSV, R)                                   \
    do {                                                          \
        if (a.limiter == 1) AGILE_STAGE_KIND(RSV, 1, R);          \
        else AGILE_STAGE_KIND(RSV, 0, R);                         \
    } while (0)
#define AGILE_STAGE_LAUNCH(R)                                     \
    do {                                                          \
        if (riemann == 0) AGILE_STAGE_LIM(0, R);                  \
        else if (riemann == 1) AGILE_STAGE_LIM(1, R);             \
        else if (riemann == 2) AGILE_STAGE_LIM(2, R);             \
        else AGILE_STAGE_LIM(3, R);                               \
    } while (0)
    if (precision == 0) AGILE_STAGE_LAUNCH(double);
    else AGILE_STAGE_LAUNCH(float);
#undef AGILE_STAGE_KIND
#undef AGILE_STAGE_LIM
#undef AGILE_STAGE_LAUNCH
    return hipGetLastError();
}

} // namespace agile
