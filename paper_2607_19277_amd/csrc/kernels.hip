// kernels.hip -- gfx950 kernels of the block-AMR finite-volume update.
//
// One workgroup (256 lanes = 4 wave64) per 16^3 block.  The stage kernel
// marches the block plane by plane in z (2.5-D): each lane owns one (i, j)
// column and keeps a 4-cell z window of primitives in registers for its
// z-faces; the x/y faces of the current plane are computed from an LDS copy
// of the plane (interior + x/y ghosts) as one flat list of 544 face tasks, so
// every face flux is computed exactly once (the paper's macro-kernel computes
// both faces of every cell, Sec. 2.1.3; here fluxes are shared through LDS).
// Fluxes are evaluated in a frame rotated to the face normal, so x and y
// faces run the same instruction stream without divergence.
//
// Numerics (paper: Sec. 2.3.1 closure and get_flux listing; Table 1 solvers):
//   primitives (rho, v, p) from conserved U, PLM minmod on primitives,
//   HLL or HLLC (Davis wave speeds), divergence
//   L = -((dFx + dFy) + dFz)/dx, SSP-RK2 stage combination.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "agile_internal.hpp"

namespace agile {

// ---------------------------------------------------------------------------
// small device helpers

__device__ __forceinline__ double rcp64(double x) {
    // hardware reciprocal estimate refined by two Newton steps (~1 ulp)
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpR(double x) { return rcp64(x); }
__device__ __forceinline__ float rcpR(float x) { return rcp32(x); }
__device__ __forceinline__ double sqrtR(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float sqrtR(float x) { return __builtin_sqrtf(x); }

template <typename R>
__device__ __forceinline__ R minmod(R a, R b) {
    // zero unless a, b have the same strict sign; else the smaller magnitude (a on ties)
    R lo = (a <= b) ? a : b;
    R hi = (a >= b) ? a : b;
    R r = (a > R(0) && b > R(0)) ? lo : R(0);
    return (a < R(0) && b < R(0)) ? hi : r;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// Euler conserved -> primitives (rho, vx, vy, vz, p); returns physical?
__device__ __forceinline__ bool cons2prim(const double U[5], double gm1, double w[5]) {
    double rho = U[0];
    double r = 1.0 / rho;
    double vx = U[1] * r, vy = U[2] * r, vz = U[3] * r;
    double vv = (vx * vx + vy * vy) + vz * vz;
    double p = gm1 * (U[4] - 0.5 * rho * vv);
    w[0] = rho; w[1] = vx; w[2] = vy; w[3] = vz; w[4] = p;
    return rho > 0.0 && p > 0.0;
}

// Cell signal rate s = ((|vx|+c)/dx + (|vy|+c)/dx) + (|vz|+c)/dx with
// c = sqrt(gamma p / rho), evaluated operation by operation (no contraction)
// so that the CFL maximum is the same number on every device.
__device__ __forceinline__ double signal_rate(const double U[5], double gamma, double inv_dx, bool &ok) {
#pragma clang fp contract(off)
    double rho = U[0];
    double r = 1.0 / rho;
    double vx = U[1] * r, vy = U[2] * r, vz = U[3] * r;
    double vv = (vx * vx + vy * vy) + vz * vz;
    double p = (gamma - 1.0) * (U[4] - 0.5 * rho * vv);
    ok = rho > 0.0 && p > 0.0;
    double c = __builtin_sqrt(gamma * p / rho);
    double s = (__builtin_fabs(vx) + c) * inv_dx;
    s = s + (__builtin_fabs(vy) + c) * inv_dx;
    s = s + (__builtin_fabs(vz) + c) * inv_dx;
    return s;
}

// Conserved state and physical flux of a rotated primitive state
// (rho, u_n, u_t1, u_t2, p): mass rho u_n, momentum rho u u_n + p e_n,
// energy u_n (p/(gamma-1) + rho u^2/2 + p) -- the get_flux listing.
template <typename R>
__device__ __forceinline__ void euler_UF(const R w[5], R igm1, R U[5], R F[5]) {
    R rho = w[0], un = w[1], v1 = w[2], v2 = w[3], p = w[4];
    R vv = (un * un + v1 * v1) + v2 * v2;
    R e = p * igm1 + R(0.5) * rho * vv;
    R mn = rho * un;
    U[0] = rho; U[1] = mn; U[2] = rho * v1; U[3] = rho * v2; U[4] = e;
    F[0] = mn; F[1] = mn * un + p; F[2] = U[2] * un; F[3] = U[3] * un; F[4] = un * (e + p);
}

// HLL / HLLC flux across a face from rotated left / right states, branch-free.
// Davis speeds S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).
// HLLC star flux F*_K = (S*(S_K U_K - F_K) + S_K P_K D*)/(S_K - S*),
// D* = (0, 1, 0, 0, S*), P_K = p_K + rho_K (S_K - u_K)(S* - u_K).
template <int RS, typename R>
__device__ __forceinline__ void riemann(const R wL[5], const R wR[5], R gamma, R igm1, R F[5]) {
    R UL[5], FL[5], UR[5], FRt[5];
    euler_UF(wL, igm1, UL, FL);
    euler_UF(wR, igm1, UR, FRt);
    R cL = sqrtR(gamma * wL[4] * rcpR(wL[0]));
    R cR = sqrtR(gamma * wR[4] * rcpR(wR[0]));
    R uL = wL[1], uR = wR[1];
    R SL = (uL - cL) < (uR - cR) ? (uL - cL) : (uR - cR);
    R SR = (uL + cL) > (uR + cR) ? (uL + cL) : (uR + cR);
    R Fm[5];
    if (RS == 0) {
        R inv = rcpR(SR - SL);
        R sLR = SL * SR;
#pragma unroll
        for (int v = 0; v < 5; ++v) Fm[v] = ((SR * FL[v] - SL * FRt[v]) + sLR * (UR[v] - UL[v])) * inv;
    } else {
        R dL = wL[0] * (SL - uL), dR = wR[0] * (SR - uR);
        R Ss = ((wR[4] - wL[4]) + (uL * dL - uR * dR)) * rcpR(dL - dR);
        bool left = Ss >= R(0);
        R SK = left ? SL : SR;
        R dK = left ? dL : dR;
        R uK = left ? uL : uR;
        R pK = left ? wL[4] : wR[4];
        R PK = pK + dK * (Ss - uK);
        R inv = rcpR(SK - Ss);
        R SP = SK * PK;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            R Uk = left ? UL[v] : UR[v];
            R Fk = left ? FL[v] : FRt[v];
            R Dv = (v == 1) ? R(1) : (v == 4 ? Ss : R(0));
            Fm[v] = (Ss * (SK * Uk - Fk) + SP * Dv) * inv;
        }
    }
    bool supL = SL >= R(0), supR = SR <= R(0);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = supL ? FL[v] : (supR ? FRt[v] : Fm[v]);
}

// PLM minmod face states from the 4-cell stencil (c-2, c-1, c, c+1) and flux.
template <int RS, typename R>
__device__ __forceinline__ void face_flux(const R a[5], const R b[5], const R c[5], const R d[5], R gamma, R igm1,
                                          R F[5]) {
    R wL[5], wR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        R sb = minmod(b[v] - a[v], c[v] - b[v]);
        R sc = minmod(c[v] - b[v], d[v] - c[v]);
        wL[v] = b[v] + R(0.5) * sb;
        wR[v] = c[v] - R(0.5) * sc;
    }
    riemann<RS, R>(wL, wR, gamma, igm1, F);
}

// ---------------------------------------------------------------------------
// stage kernel

constexpr int PW = BN + 2 * NG;      // 20: padded plane width
constexpr int PLANE = PW * PW;       // 400
constexpr int NXF = BN * (BN + 1);   // 272 x-face (and y-face) tasks per plane
constexpr int NTASK = 2 * NXF;       // 544

template <int RS, typename R>
__global__ __launch_bounds__(256) void k_stage(StageArgs a) {
    constexpr int NV = 5;
    __shared__ R sP[NV][PLANE];
    __shared__ R sF[NV][NTASK];
    __shared__ unsigned long long sMax[4];

    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const int i = tid & 15, j = tid >> 4;
    const BlockDesc D = a.desc[b];
    MeshParams &mp = a.mp[D.mesh];
    const double gamma = mp.gamma;
    const double gm1 = gamma - 1.0;
    const R gammaR = R(gamma), igm1R = R(1.0 / gm1);
    const double inv_dx = mp.inv_dx1 * double(1 << (D.level - 1));
    const double dt = mp.dt;
    const size_t vstr = CELLS;
    const double *Ub = a.Uin + size_t(b) * NV * CELLS;
    bool ok = true;

    // source of the conserved value at z-index kk in [-2, 18) of this column
    auto zsrc = [&](int kk, size_t &stride) -> const double * {
        if (kk >= 0 && kk < BN) {
            stride = vstr;
            return Ub + kk * 256 + j * 16 + i;
        }
        const int f = kk < 0 ? 4 : 5;
        const int nb = D.nb[f];
        if (nb >= 0) {
            stride = vstr;
            const int kn = kk < 0 ? kk + BN : kk - BN;
            return a.Uin + size_t(nb) * NV * CELLS + kn * 256 + j * 16 + i;
        }
        stride = SLAB;
        const int g = kk < 0 ? kk + NG : kk - BN;
        return a.halo + size_t(-nb - 1) * NV * SLAB + g * 256 + j * 16 + i;
    };
    auto load_prim = [&](int kk, R w[NV]) {
        size_t st;
        const double *p = zsrc(kk, st);
        double U[NV], q[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = p[v * st];
        ok &= cons2prim(U, gm1, q);
        // rotated to the z normal: (rho, vz, vx, vy, p)
        w[0] = R(q[0]); w[1] = R(q[3]); w[2] = R(q[1]); w[3] = R(q[2]); w[4] = R(q[4]);
    };

    // z window (rotated primitives) of cells k-1 .. k+2, z-face flux of face k-1/2
    R W0[NV], W1[NV], W2[NV], W3[NV], Flo[NV], Fhi[NV];
    {
        R Wm2[NV];
        load_prim(-2, Wm2);
        load_prim(-1, W0);
        load_prim(0, W1);
        load_prim(1, W2);
        face_flux<RS, R>(Wm2, W0, W1, W2, gammaR, igm1R, Flo);
    }
    // z flux register of the -z face
    if (D.freg[4] >= 0) {
        double *r = a.freg + size_t(D.freg[4]) * NV * REG + j * 16 + i;
        r[0] = double(Flo[0]); r[1 * REG] = double(Flo[2]); r[2 * REG] = double(Flo[3]);
        r[3 * REG] = double(Flo[1]); r[4 * REG] = double(Flo[4]);
    }

    const int tt = (tid + 64 * (b & 3)) & 255;   // rotate the extra face tasks over the waves
    unsigned long long smax = 0;
    const double *Xin = a.XEin;

    for (int k = 0; k < BN; ++k) {
        load_prim(k + 2, W3);
        face_flux<RS, R>(W0, W1, W2, W3, gammaR, igm1R, Fhi);

        // plane k into LDS: own cell (un-rotated) and the x / y ghosts
        {
            const int p = (j + 2) * PW + i + 2;
            sP[0][p] = W1[0]; sP[1][p] = W1[2]; sP[2][p] = W1[3]; sP[3][p] = W1[1]; sP[4][p] = W1[4];
        }
        if (tid < 128) {
            const int f = tid >> 5, r = tid & 31;
            const int nb = D.nb[f];
            const double *src;
            size_t st;
            int lp;
            if (f < 2) {
                const int jj = r >> 1, g = r & 1;
                lp = (jj + 2) * PW + (f == 0 ? g : BN + NG + g);
                if (nb >= 0) {
                    src = Xin + (size_t(nb) * NV * 2 + (f == 0 ? 1 : 0)) * SLAB + k * 32 + r;
                    st = 2 * SLAB;
                } else {
                    src = a.halo + size_t(-nb - 1) * NV * SLAB + k * 32 + r;
                    st = SLAB;
                }
            } else {
                const int g = r >> 4, ii = r & 15;
                lp = (f == 2 ? g : BN + NG + g) * PW + ii + 2;
                if (nb >= 0) {
                    src = a.Uin + size_t(nb) * NV * CELLS + k * 256 + (f == 2 ? 224 : 0) + r;
                    st = vstr;
                } else {
                    src = a.halo + size_t(-nb - 1) * NV * SLAB + k * 32 + r;
                    st = SLAB;
                }
            }
            double U[NV], q[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v] = src[v * st];
            ok &= cons2prim(U, gm1, q);
#pragma unroll
            for (int v = 0; v < NV; ++v) sP[v][lp] = R(q[v]);
        }
        __syncthreads();

        // x and y faces of plane k: tasks [0, 272) x, [272, 544) y
#pragma unroll
        for (int rr = 0; rr < 3; ++rr) {
            const int t = tt + 256 * rr;
            if (t < NTASK) {
                const int d = t >= NXF;
                const int u = t - NXF * d;
                int base, st;
                if (!d) {
                    const int jj = u / 17, fi = u - 17 * jj;
                    base = (jj + 2) * PW + fi;
                    st = 1;
                } else {
                    const int fj = u >> 4, ii = u & 15;
                    base = fj * PW + ii + 2;
                    st = PW;
                }
                R c[4][NV];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int p = base + s * st;
                    c[s][0] = sP[0][p];
                    c[s][1] = sP[1 + d][p];
                    c[s][2] = sP[2 - d][p];
                    c[s][3] = sP[3][p];
                    c[s][4] = sP[4][p];
                }
                R F[NV];
                face_flux<RS, R>(c[0], c[1], c[2], c[3], gammaR, igm1R, F);
                sF[0][t] = F[0];
                sF[1][t] = d ? F[2] : F[1];
                sF[2][t] = d ? F[1] : F[2];
                sF[3][t] = F[3];
                sF[4][t] = F[4];
            }
        }
        __syncthreads();

        // divergence, stage combination, stores
        {
            const double fz[NV] = {double(Fhi[0]) - double(Flo[0]), double(Fhi[2]) - double(Flo[2]),
                                   double(Fhi[3]) - double(Flo[3]), double(Fhi[1]) - double(Flo[1]),
                                   double(Fhi[4]) - double(Flo[4])};
            const size_t cell = size_t(k) * 256 + j * 16 + i;
            double out[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double dfx = double(sF[v][j * 17 + i + 1]) - double(sF[v][j * 17 + i]);
                const double dfy = double(sF[v][NXF + (j + 1) * 16 + i]) - double(sF[v][NXF + j * 16 + i]);
                const double L = -((dfx + dfy) + fz[v]) * inv_dx;
                const double uin = Ub[v * vstr + cell];
                if (a.stage == 1) {
                    out[v] = uin + dt * L;
                } else {
                    const double un = a.Un[size_t(b) * NV * CELLS + v * vstr + cell];
                    out[v] = 0.5 * (un + (uin + dt * L));
                }
                a.Uout[size_t(b) * NV * CELLS + v * vstr + cell] = out[v];
            }
            if (i < 2 || i >= BN - 2) {
                const int side = i >= BN - 2;
                const int g = i - (side ? BN - 2 : 0);
                double *x = a.XEout + (size_t(b) * NV * 2 + side) * SLAB + k * 32 + j * 2 + g;
#pragma unroll
                for (int v = 0; v < NV; ++v) x[v * 2 * SLAB] = out[v];
            }
            if (a.stage == 2) {
                const int cf = D.cf_coarse;
                const bool skip = ((cf & 1) && i == 0) || ((cf & 2) && i == BN - 1) || ((cf & 4) && j == 0) ||
                                  ((cf & 8) && j == BN - 1) || ((cf & 16) && k == 0) || ((cf & 32) && k == BN - 1);
                bool ok2;
                const double s = signal_rate(out, gamma, inv_dx, ok2);
                ok &= ok2;
                if (!skip) {
                    const unsigned long long sb = __double_as_longlong(s);
                    smax = sb > smax ? sb : smax;
                }
            }
        }
        // flux registers of x / y boundary faces of this plane
        if (tid < 32) {
            const int lane = tid & 15;
            if (tid < 16) {
                if (D.freg[0] >= 0) {
                    double *r = a.freg + size_t(D.freg[0]) * NV * REG + k * 16 + lane;
#pragma unroll
                    for (int v = 0; v < NV; ++v) r[v * REG] = double(sF[v][lane * 17]);
                }
                if (D.freg[1] >= 0) {
                    double *r = a.freg + size_t(D.freg[1]) * NV * REG + k * 16 + lane;
#pragma unroll
                    for (int v = 0; v < NV; ++v) r[v * REG] = double(sF[v][lane * 17 + 16]);
                }
            } else {
                if (D.freg[2] >= 0) {
                    double *r = a.freg + size_t(D.freg[2]) * NV * REG + k * 16 + lane;
#pragma unroll
                    for (int v = 0; v < NV; ++v) r[v * REG] = double(sF[v][NXF + lane]);
                }
                if (D.freg[3] >= 0) {
                    double *r = a.freg + size_t(D.freg[3]) * NV * REG + k * 16 + lane;
#pragma unroll
                    for (int v = 0; v < NV; ++v) r[v * REG] = double(sF[v][NXF + BN * 16 + lane]);
                }
            }
        }
        // slide the z window
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            W0[v] = W1[v]; W1[v] = W2[v]; W2[v] = W3[v]; Flo[v] = Fhi[v];
        }
    }
    // z flux register of the +z face (Flo now holds the flux of face 15+1/2)
    if (D.freg[5] >= 0) {
        double *r = a.freg + size_t(D.freg[5]) * NV * REG + j * 16 + i;
        r[0] = double(Flo[0]); r[1 * REG] = double(Flo[2]); r[2 * REG] = double(Flo[3]);
        r[3 * REG] = double(Flo[1]); r[4 * REG] = double(Flo[4]);
    }
    if (!ok) atomicOr(&mp.flags, 1);
    if (a.stage == 2) {
        smax = wave_max_u64(smax);
        if ((tid & 63) == 0) sMax[tid >> 6] = smax;
        __syncthreads();
        if (tid == 0) {
            unsigned long long m = sMax[0];
            for (int w = 1; w < 4; ++w) m = sMax[w] > m ? sMax[w] : m;
            a.smax[b] = m;
        }
    }
}

// ---------------------------------------------------------------------------
// ghost-slab cell index (c in [0, 512)) -> (g, a, b) and back

__device__ __forceinline__ void slab_coords(int d, int c, int &g, int &ta, int &tb) {
    if (d == 0) { g = c & 1; ta = (c >> 1) & 15; tb = c >> 5; }          // [k][j][g]
    else if (d == 1) { ta = c & 15; g = (c >> 4) & 1; tb = c >> 5; }     // [k][g][i]
    else { ta = c & 15; tb = (c >> 4) & 15; g = c >> 8; }                // [g][j][i]
}
__device__ __forceinline__ int slab_index(int d, int g, int ta, int tb) {
    if (d == 0) return (tb * 16 + ta) * 2 + g;
    if (d == 1) return (tb * 2 + g) * 16 + ta;
    return (g * 16 + tb) * 16 + ta;
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

// Restriction: coarse ghost = mean of its 8 fine children, summed pairwise
// ((c000+c100)+(c010+c110)) + ((c001+c101)+(c011+c111)) with x fastest.
__global__ __launch_bounds__(256) void k_restrict(const RestrictTask *tasks, const double *U, double *halo, int NV) {
    const RestrictTask t = tasks[blockIdx.x];
    const int d = t.face >> 1, side = t.face & 1;
    for (int c = threadIdx.x; c < SLAB; c += blockDim.x) {
        int g, ta, tb;
        slab_coords(d, c, g, ta, tb);
        const int q = (ta >> 3) + 2 * (tb >> 3);
        const int F = t.fine[q];
        int base[3];
        base[d] = side ? 2 * g : 12 + 2 * g;   // fine cells under coarse ghost layer g
        base[d == 0 ? 1 : 0] = 2 * (ta & 7);
        base[d == 2 ? 1 : 2] = 2 * (tb & 7);
        for (int v = 0; v < NV; ++v) {
            const double *u = U + (size_t(F) * NV + v) * CELLS;
            double ch[8];
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx)
                        ch[dx + 2 * dy + 4 * dz] = u[((base[2] + dz) * 16 + base[1] + dy) * 16 + base[0] + dx];
            const double s = ((ch[0] + ch[1]) + (ch[2] + ch[3])) + ((ch[4] + ch[5]) + (ch[6] + ch[7]));
            halo[(size_t(t.slot) * NV + v) * SLAB + c] = s * 0.125;
        }
    }
}

// Prolongation: fine ghost = parent + sum over x, y, z (in that order) of
// +/- (1/4) minmod(parent - left, right - parent) of the parent's axis neighbours.
__global__ __launch_bounds__(256) void k_prolong(const ProlongTask *tasks, const BlockDesc *desc, const double *U,
                                                 double *halo, int NV) {
    const ProlongTask t = tasks[blockIdx.x];
    const int d = t.face >> 1, side = t.face & 1;
    const int da = d == 0 ? 1 : 0, dbx = d == 2 ? 1 : 2;
    for (int c = threadIdx.x; c < SLAB; c += blockDim.x) {
        int g, ta, tb;
        slab_coords(d, c, g, ta, tb);
        int pc[3], sg[3];
        pc[d] = side ? 0 : BN - 1;      // coarse layer next to the face
        sg[d] = g ? 1 : -1;             // fine ghost layer g: low child for g = 0
        pc[da] = t.ta + (ta >> 1);
        sg[da] = (ta & 1) ? 1 : -1;
        pc[dbx] = t.tb + (tb >> 1);
        sg[dbx] = (tb & 1) ? 1 : -1;
        for (int v = 0; v < NV; ++v) {
            const double vc = block_value(desc, U, halo, NV, t.coarse, v, pc[0], pc[1], pc[2]);
            double val = vc;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                int m[3] = {pc[0], pc[1], pc[2]}, p[3] = {pc[0], pc[1], pc[2]};
                m[e] -= 1;
                p[e] += 1;
                const double vm = block_value(desc, U, halo, NV, t.coarse, v, m[0], m[1], m[2]);
                const double vp = block_value(desc, U, halo, NV, t.coarse, v, p[0], p[1], p[2]);
                const double q = 0.25 * minmod(vc - vm, vp - vc);
                val = sg[e] > 0 ? val + q : val - q;
            }
            halo[(size_t(t.slot) * NV + v) * SLAB + c] = val;
        }
    }
}

// Coarse-fine flux correction of one coarse block: for each coarse-fine face
// the coarse flux F_c is replaced by the mean of the 4 fine fluxes covering it,
// F_f = ((f00+f10)+(f01+f11))/4, i.e. U += w dt/dx (+/-)(F_c - F_f).
__global__ __launch_bounds__(256) void k_reflux(const RefluxTask *tasks, const BlockDesc *desc, MeshParams *mp,
                                                double *U, double *XE, const double *freg,
                                                unsigned long long *smax, int NV, int stage) {
    const RefluxTask t = tasks[blockIdx.x];
    const BlockDesc D = desc[t.block];
    MeshParams &P = mp[D.mesh];
    const double inv_dx = P.inv_dx1 * double(1 << (D.level - 1));
    const double w = (stage == 1 ? P.dt : 0.5 * P.dt) * inv_dx;
    const int c = threadIdx.x;
    const int ta = c & 15, tb = c >> 4;
    for (int n = 0; n < t.nface; ++n) {
        const int f = t.face[n], d = f >> 1, side = f & 1;
        const int q = (ta >> 3) + 2 * (tb >> 3);
        const double *fr = freg + size_t(t.fslot[n][q]) * NV * REG;
        const double *cr = freg + size_t(t.cslot[n]) * NV * REG;
        const int fa = 2 * (ta & 7), fb = 2 * (tb & 7);
        int x[3];
        x[d] = side ? BN - 1 : 0;
        x[d == 0 ? 1 : 0] = ta;
        x[d == 2 ? 1 : 2] = tb;
        const size_t cell = (size_t(x[2]) * 16 + x[1]) * 16 + x[0];
        for (int v = 0; v < NV; ++v) {
            const double *f = fr + v * REG;
            const double fm = ((f[fb * 16 + fa] + f[fb * 16 + fa + 1]) + (f[(fb + 1) * 16 + fa] + f[(fb + 1) * 16 + fa + 1])) * 0.25;
            const double diff = cr[v * REG + c] - fm;
            double *u = U + (size_t(t.block) * NV + v) * CELLS + cell;
            const double nu = side ? *u + w * diff : *u - w * diff;
            *u = nu;
            if (x[0] < 2 || x[0] >= BN - 2) {
                const int xs = x[0] >= BN - 2;
                XE[((size_t(t.block) * NV + v) * 2 + xs) * SLAB + (x[2] * 16 + x[1]) * 2 + (x[0] - (xs ? BN - 2 : 0))] = nu;
            }
        }
        __syncthreads();
    }
    if (stage == 2) {
        // signal rate of the corrected cells (left out of the stage-2 maximum)
        unsigned long long m = 0;
        bool ok = true;
        for (int n = 0; n < t.nface; ++n) {
            const int f = t.face[n], d = f >> 1, side = f & 1;
            int x[3];
            x[d] = side ? BN - 1 : 0;
            x[d == 0 ? 1 : 0] = ta;
            x[d == 2 ? 1 : 2] = tb;
            const size_t cell = (size_t(x[2]) * 16 + x[1]) * 16 + x[0];
            double u[5];
            for (int v = 0; v < 5; ++v) u[v] = U[(size_t(t.block) * NV + v) * CELLS + cell];
            bool ok2;
            const double s = signal_rate(u, P.gamma, inv_dx, ok2);
            ok &= ok2;
            const unsigned long long sb = __double_as_longlong(s);
            m = sb > m ? sb : m;
        }
        m = wave_max_u64(m);
        if ((c & 63) == 0) atomicMax(&smax[t.block], m);
        if (!ok) atomicOr(&P.flags, 1);
    }
}

// x-boundary columns of every row into XE (after an upload or external change).
__global__ __launch_bounds__(256) void k_xexport(const double *U, double *XE, int NV) {
    const int b = blockIdx.x;
    for (int e = threadIdx.x; e < NV * XE_CELLS; e += blockDim.x) {
        const int v = e / XE_CELLS, r = e - v * XE_CELLS;
        const int side = r / SLAB, s = r - side * SLAB;
        const int g = s & 1, row = s >> 1;   // row = k*16 + j
        const int x = side ? BN - 2 + g : g;
        XE[(size_t(b) * NV + v) * XE_CELLS + r] = U[(size_t(b) * NV + v) * CELLS + row * 16 + x];
    }
}

// per-block maximum signal rate of the current state
__global__ __launch_bounds__(256) void k_smax(const BlockDesc *desc, MeshParams *mp, const double *U,
                                              unsigned long long *smax, int NV) {
    __shared__ unsigned long long sMax[4];
    const int b = blockIdx.x;
    const BlockDesc D = desc[b];
    MeshParams &P = mp[D.mesh];
    const double inv_dx = P.inv_dx1 * double(1 << (D.level - 1));
    unsigned long long m = 0;
    bool ok = true;
    for (int c = threadIdx.x; c < CELLS; c += blockDim.x) {
        double u[5];
        for (int v = 0; v < 5; ++v) u[v] = U[(size_t(b) * NV + v) * CELLS + c];
        bool ok2;
        const double s = signal_rate(u, P.gamma, inv_dx, ok2);
        ok &= ok2;
        const unsigned long long sb = __double_as_longlong(s);
        m = sb > m ? sb : m;
    }
    m = wave_max_u64(m);
    if ((threadIdx.x & 63) == 0) sMax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = sMax[0];
        for (int w = 1; w < 4; ++w) r = sMax[w] > r ? sMax[w] : r;
        smax[b] = r;
    }
    if (!ok) atomicOr(&P.flags, 1);
}

// dt = cfl / max s over the mesh's blocks [first, first + n)
__global__ __launch_bounds__(256) void k_dt_finalize(MeshParams *mp, int mesh, const unsigned long long *smax,
                                                     int first, int n, int set_dt) {
    __shared__ unsigned long long sMax[4];
    unsigned long long m = 0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const unsigned long long v = smax[first + q];
        m = v > m ? v : m;
    }
    m = wave_max_u64(m);
    if ((threadIdx.x & 63) == 0) sMax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = sMax[0];
        for (int w = 1; w < 4; ++w) r = sMax[w] > r ? sMax[w] : r;
        mp[mesh].smax = r;
        if (set_dt) mp[mesh].dt = mp[mesh].cfl / __longlong_as_double(r);
    }
}

__global__ void k_set_dt(MeshParams *mp, int mesh, double dt) {
    if (threadIdx.x == 0) mp[mesh].dt = dt;
}

// permuted block copies between caller order and device order
__global__ __launch_bounds__(256) void k_permute(const double *src, double *dst, const int *map, int per_block,
                                                 int gather) {
    const int b = blockIdx.x;
    const int o = map[b];
    const double *s = src + size_t(gather ? o : b) * per_block;
    double *d = dst + size_t(gather ? b : o) * per_block;
    for (int e = threadIdx.x; e < per_block; e += blockDim.x) d[e] = s[e];
}

// face ghosts of every block as the update reads them: [block][face][var][512]
__global__ __launch_bounds__(256) void k_read_ghosts(const BlockDesc *desc, const double *U, const double *halo,
                                                     double *out, int NV) {
    const int b = blockIdx.x;
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
            out[((size_t(b) * 6 + f) * NV + v) * SLAB + c] = block_value(desc, U, halo, NV, b, v, x[0], x[1], x[2]);
    }
}

// ---------------------------------------------------------------------------
// launch wrappers (host)

hipError_t launch_stage(const StageArgs &a, int riemann, int precision, hipStream_t s) {
    dim3 grid(a.nblocks), block(256);
    if (precision == 0) {
        if (riemann == 0) hipLaunchKernelGGL((k_stage<0, double>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_stage<1, double>), grid, block, 0, s, a);
    } else {
        if (riemann == 0) hipLaunchKernelGGL((k_stage<0, float>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_stage<1, float>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_restrict(const RestrictTask *t, int n, const double *U, double *halo, int NV, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_restrict, dim3(n), dim3(256), 0, s, t, U, halo, NV);
    return hipGetLastError();
}

hipError_t launch_prolong(const ProlongTask *t, int n, const BlockDesc *desc, const double *U, double *halo, int NV,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prolong, dim3(n), dim3(256), 0, s, t, desc, U, halo, NV);
    return hipGetLastError();
}

hipError_t launch_reflux(const RefluxTask *t, int n, const BlockDesc *desc, MeshParams *mp, double *U, double *XE,
                         const double *freg, unsigned long long *smax, int NV, int stage, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reflux, dim3(n), dim3(256), 0, s, t, desc, mp, U, XE, freg, smax, NV, stage);
    return hipGetLastError();
}

hipError_t launch_xexport(const double *U, double *XE, int nblocks, int NV, hipStream_t s) {
    hipLaunchKernelGGL(k_xexport, dim3(nblocks), dim3(256), 0, s, U, XE, NV);
    return hipGetLastError();
}

hipError_t launch_smax(const BlockDesc *desc, MeshParams *mp, const double *U, unsigned long long *smax, int nblocks,
                       int NV, hipStream_t s) {
    hipLaunchKernelGGL(k_smax, dim3(nblocks), dim3(256), 0, s, desc, mp, U, smax, NV);
    return hipGetLastError();
}

hipError_t launch_dt_finalize(MeshParams *mp, int mesh, const unsigned long long *smax, int first, int n, int set_dt,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_dt_finalize, dim3(1), dim3(256), 0, s, mp, mesh, smax, first, n, set_dt);
    return hipGetLastError();
}

hipError_t launch_set_dt(MeshParams *mp, int mesh, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(64), 0, s, mp, mesh, dt);
    return hipGetLastError();
}

hipError_t launch_permute(const double *src, double *dst, const int *map, int nblocks, int per_block, int gather,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(nblocks), dim3(256), 0, s, src, dst, map, per_block, gather);
    return hipGetLastError();
}

hipError_t launch_read_ghosts(const BlockDesc *desc, const double *U, const double *halo, double *out, int nblocks,
                              int NV, hipStream_t s) {
    hipLaunchKernelGGL(k_read_ghosts, dim3(nblocks), dim3(256), 0, s, desc, U, halo, out, NV);
    return hipGetLastError();
}

} // namespace agile
