// device_math.hpp -- per-cell / per-face device arithmetic shared by the
// gfx950 kernels: the Euler update (AGILE 1.0, Sec. 2.3.1 equations;
// Table 1 solvers HLL, HLLC, LF), ideal MHD with GLM cleaning (Sec. 2.3.3)
// and special relativistic hydrodynamics (Sec. 2.3.4); minmod and van Leer
// slopes (Sec. 3.1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace agile {

// ---------------------------------------------------------------------------
// arithmetic helpers

// reciprocal: hardware estimate (relative error below 5e-8 on gfx950)
// refined by one Newton step, which squares the error: below 3e-15, measured
// at most 20 ulp over 2^-60 .. 2^60
__device__ __forceinline__ double rcp64(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
// square root of zero or a positive normal number: hardware reciprocal
// square root refined by two Goldschmidt steps and a final residual
// correction (~1 ulp); zero maps to zero (the iteration alone would give
// 0 * inf)
__device__ __forceinline__ double sqrt64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    return x == 0.0 ? 0.0 : fma(d, h, g);
}
__device__ __forceinline__ double rcpR(double x) { return rcp64(x); }
__device__ __forceinline__ float rcpR(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sqrtR(double x) { return sqrt64(x); }
__device__ __forceinline__ float sqrtR(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fminR(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float fminR(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double fmaxR(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ double absR(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float absR(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ float fmaxR(float a, float b) { return __builtin_fmaxf(a, b); }

// minmod(a, b) = median(a, b, 0): 0 unless a and b have the same sign, else
// the argument of smaller magnitude (a and b equal on ties).
__device__ __forceinline__ double minmod(double a, double b) {
    return __builtin_fmax(__builtin_fmin(a, b), __builtin_fmin(__builtin_fmax(a, b), 0.0));
}
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }

// van Leer's limited slope: the harmonic mean 2ab/(a+b) when a and b have the
// same strict sign, else 0.
template <typename R>
__device__ __forceinline__ R vanleer(R a, R b) {
    const bool same = (a > R(0) && b > R(0)) || (a < R(0) && b < R(0));
    return same ? (R(2) * a * b) * rcpR(a + b) : R(0);
}

// reconstruction slope: LIM 0 minmod, 1 van Leer
template <int LIM, typename R>
__device__ __forceinline__ R slope(R a, R b) {
    if (LIM == 1) return vanleer(a, b);
    return minmod(a, b);
}

// reciprocal square root of a positive normal number: hardware estimate
// refined by one Newton step (measured at most 36 ulp over 2^-60 .. 2^60)
__device__ __forceinline__ double rsq64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}
__device__ __forceinline__ double rsqR(double x) { return rsq64(x); }
__device__ __forceinline__ float rsqR(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Euler physics

// conserved -> primitives (rho, vx, vy, vz, p) with v = m (1/rho),
// p = (gamma-1)(e - rho v^2/2); returns whether rho > 0 and p > 0
__device__ __forceinline__ bool cons2prim(const double U[5], double gm1, double w[5]) {
    const double rho = U[0];
    const double r = rcp64(rho);
    const double vx = U[1] * r, vy = U[2] * r, vz = U[3] * r;
    const double vv = (vx * vx + vy * vy) + vz * vz;
    const double p = gm1 * (U[4] - 0.5 * rho * vv);
    w[0] = rho; w[1] = vx; w[2] = vy; w[3] = vz; w[4] = p;
    return rho > 0.0 && p > 0.0;
}

// Cell signal rate s = ((|vx|+c)/dx + (|vy|+c)/dx) + (|vz|+c)/dx with
// c = sqrt(gamma p / rho), evaluated operation by operation with IEEE
// division and square root and no contraction, so that the CFL maximum is
// the same number as on the CPU.
__device__ __forceinline__ double signal_rate(const double U[5], double gamma, double inv_dx, bool &ok) {
#pragma clang fp contract(off)
    const double rho = U[0];
    const double r = 1.0 / rho;
    const double vx = U[1] * r, vy = U[2] * r, vz = U[3] * r;
    const double vv = (vx * vx + vy * vy) + vz * vz;
    const double p = (gamma - 1.0) * (U[4] - 0.5 * rho * vv);
    ok = rho > 0.0 && p > 0.0;
    const double c = __builtin_sqrt(gamma * p / rho);
    double s = (__builtin_fabs(vx) + c) * inv_dx;
    s = s + (__builtin_fabs(vy) + c) * inv_dx;
    s = s + (__builtin_fabs(vz) + c) * inv_dx;
    return s;
}

// Conserved state and physical flux of a primitive state rotated to the face
// normal, (rho, u_n, u_t1, u_t2, p): mass rho u_n, momentum rho u u_n + p e_n,
// energy u_n (e + p) -- the Euler equations of Sec. 2.3.1.
template <typename R>
__device__ __forceinline__ void euler_UF(const R w[5], R igm1, R U[5], R F[5]) {
    const R rho = w[0], un = w[1], v1 = w[2], v2 = w[3], p = w[4];
    const R vv = (un * un + v1 * v1) + v2 * v2;
    const R e = p * igm1 + R(0.5) * rho * vv;
    const R mn = rho * un;
    U[0] = rho; U[1] = mn; U[2] = rho * v1; U[3] = rho * v2; U[4] = e;
    F[0] = mn; F[1] = mn * un + p; F[2] = U[2] * un; F[3] = U[3] * un; F[4] = un * (e + p);
}

// sound speed c = sqrt(gamma p / rho), written as gamma p / sqrt(gamma p rho)
template <typename R>
__device__ __forceinline__ R sound_speed(R rho, R p, R gamma) {
    const R gp = gamma * p;
    return gp * rsqR(gp * rho);
}

// HLL (RS = 0), HLLC (RS = 1) or local Lax-Friedrichs (RS = 2) flux across a
// face from rotated left / right primitive states, evaluated without branches.  Wave speeds of Davis:
// S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).
// HLL: with a = max(S_R, 0), b = min(S_L, 0),
//   F = (a F_L - b F_R + a b (U_R - U_L)) / (a - b),
// which equals F_L for S_L >= 0, F_R for S_R <= 0 and the two-wave HLL flux
// otherwise.
// HLLC (Toro, Sec. 10.4): contact speed
//   S* = (p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R)) / (rho_L (S_L - u_L) - rho_R (S_R - u_R)),
// upwind side K = L if S_L >= 0, R if S_R <= 0, else L iff S* >= 0; then
//   F = F_K in the supersonic cases, else
//   F*_K = (S*(S_K U_K - F_K) + S_K P_K D*)/(S_K - S*), D* = (0, 1, 0, 0, S*),
//   P_K = p_K + rho_K (S_K - u_K)(S* - u_K).
// Only side K's conserved state and flux are formed.
template <typename R>
__device__ __forceinline__ void riemann_srhd(const R wL[5], const R wR[5], R g, R igm1, R F[5]);

template <int RS, typename R>
__device__ __forceinline__ void riemann(const R wL[5], const R wR[5], R gamma, R igm1, R F[5]) {
    if (RS == 3) {   // SRHD states (rho, u, p): local Lax-Friedrichs
        riemann_srhd(wL, wR, gamma, igm1, F);
        return;
    }
    const R cL = sound_speed(wL[0], wL[4], gamma);
    const R cR = sound_speed(wR[0], wR[4], gamma);
    const R uL = wL[1], uR = wR[1];
    const R SL = fminR(uL - cL, uR - cR);
    const R SR = fmaxR(uL + cL, uR + cR);
    if (RS == 2) {
        // local Lax-Friedrichs: F = ((F_L + F_R) - s (U_R - U_L))/2 with the
        // larger |u| + c of the two states
        R UL[5], FL[5], UR[5], FRt[5];
        euler_UF(wL, igm1, UL, FL);
        euler_UF(wR, igm1, UR, FRt);
        const R sp = fmaxR(absR(uL) + cL, absR(uR) + cR);
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = R(0.5) * ((FL[v] + FRt[v]) - sp * (UR[v] - UL[v]));
    } else if (RS == 0) {
        R UL[5], FL[5], UR[5], FRt[5];
        euler_UF(wL, igm1, UL, FL);
        euler_UF(wR, igm1, UR, FRt);
        const R ap = fmaxR(SR, R(0)), bm = fminR(SL, R(0));
        const R inv = rcpR(ap - bm);
        const R ab = ap * bm;
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = ((ap * FL[v] - bm * FRt[v]) + ab * (UR[v] - UL[v])) * inv;
    } else {
        const R dL = wL[0] * (SL - uL), dR = wR[0] * (SR - uR);
        const R Ss = ((wR[4] - wL[4]) + (uL * dL - uR * dR)) * rcpR(dL - dR);
        const bool supL = SL >= R(0), supR = SR <= R(0);
        const bool left = supL || (!supR && Ss >= R(0));
        R w[5], U[5], Fk[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) w[v] = left ? wL[v] : wR[v];
        const R SK = left ? SL : SR;
        const R dK = left ? dL : dR;
        euler_UF(w, igm1, U, Fk);
        const R PK = w[4] + dK * (Ss - w[1]);
        const R inv = rcpR(SK - Ss);
        const R SP = SK * PK;
        const bool sup = supL || supR;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            R t = Ss * (SK * U[v] - Fk[v]);
            if (v == 1) t = t + SP;
            if (v == 4) t = t + SP * Ss;
            F[v] = sup ? Fk[v] : t * inv;
        }
    }
}


// ---------------------------------------------------------------------------
// special relativistic hydrodynamics (c = 1), nvar 5: (D, m, tau)
// primitives (rho, u, p) with u = Gamma v the spatial four-velocity, ideal
// gas h = 1 + g/(g-1) p/rho (Sec. 2.3.4)

// con2prim by a 1-D root in xi = Gamma^2 rho h: with e = tau + D,
//   1/Gamma^2 = 1 - m^2/xi^2, rho = D/Gamma, p(xi) = (g-1)/g (xi/Gamma^2 - D/Gamma),
//   f(xi) = xi - p(xi) - e increases on (|m|, g e], f(|m|) <= 0 < f(g e);
// Newton steps from xi = e kept inside the bracket (bisection otherwise)
// until a step moves xi by at most 1e-15 xi (at most 100).  IEEE division and
// square root without contraction: the same iterates as on any machine.  The
// CFL signal uses this form, so that dt is the same number everywhere.
__device__ __forceinline__ bool srhd_con2prim(const double U[5], double g, double w[5]) {
#pragma clang fp contract(off)
    const double D = U[0], e = U[4] + U[0];
    const double m2 = (U[1] * U[1] + U[2] * U[2]) + U[3] * U[3];
    const double mm = __builtin_sqrt(m2);
    const double gg = (g - 1.0) / g;
    double lo = mm, hi = g * e;
    if (!(D > 0.0) || !(hi > lo)) {
        for (int v = 0; v < 5; ++v) w[v] = 1.0;
        return false;
    }
    double x = e;
    if (!(x > lo)) x = 0.5 * (lo + hi);
    bool conv = false;
    for (int it = 0; it < 100 && !conv; ++it) {
        const double q = m2 / (x * x);
        const double g2 = 1.0 - q;
        const double ig = __builtin_sqrt(g2);
        const double G = 1.0 / ig;
        const double p = gg * (x * g2 - D * ig);
        const double f = (x - p) - e;
        const double fp = 1.0 - gg * ((1.0 + q) - D * G * q / x);
        if (f > 0.0) hi = x;
        else if (f < 0.0) lo = x;
        double xn = x - f / fp;
        // a step within the tolerance converges, also on a bracket end
        conv = __builtin_fabs(xn - x) <= 1e-15 * xn;
        if (!conv && !(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        x = xn;
    }
    const double g2 = 1.0 - m2 / (x * x);
    const double ig = __builtin_sqrt(g2);
    const double G = 1.0 / ig;
    const double rho = D * ig;
    const double p = gg * (x * g2 - D * ig);
    w[0] = rho;
    w[1] = (U[1] / x) * G;
    w[2] = (U[2] / x) * G;
    w[3] = (U[3] / x) * G;
    w[4] = p;
    return conv && rho > 0.0 && p > 0.0;
}

// reciprocal and reciprocal square root refined by two Newton steps
// (within about an ulp): the con2prim iteration below stops on its step
// size, which must stay above their rounding noise
__device__ __forceinline__ double rcp64x2(double x) {
    const double r = rcp64(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq64x2(double x) {
    const double y = rsq64(x);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// The same root for the flux path, where the primitives need not be the same
// bits as elsewhere: reciprocals instead of IEEE division and square root, a
// start nearer the root, and Newton stops after a step of at most 1e-9 xi.  Newton converges
// quadratically there, so that step leaves an error far below rounding (the
// result agrees with the 1e-15 iteration to a few ulp), and the stopping
// test stays clear of the arithmetic's noise.
__device__ __forceinline__ bool srhd_con2prim_fast(const double U[5], double g, double w[5]) {
    const double D = U[0], e = U[4] + U[0];
    const double m2 = (U[1] * U[1] + U[2] * U[2]) + U[3] * U[3];
    const double gg = (g - 1.0) / g;
    double lo = __builtin_sqrt(m2), hi = g * e;
    if (!(D > 0.0) || !(hi > lo)) {
        for (int v = 0; v < 5; ++v) w[v] = 1.0;
        return false;
    }
    // start: the root at rest, xi = e + (g-1)(e - D), with the pressure part
    // scaled by 1 - m^2/e^2 (one Newton step fewer than xi = e on moving gas)
    double x = e + ((g - 1.0) * (e - D)) * (1.0 - m2 * rcp64x2(e * e));
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    bool conv = false;
    for (int it = 0; it < 100 && !conv; ++it) {
        const double r = rcp64x2(x);
        const double q = (m2 * r) * r;
        const double g2 = 1.0 - q;
        const double G = rsq64x2(g2);
        const double ig = g2 * G;
        const double p = gg * (x * g2 - D * ig);
        const double f = (x - p) - e;
        const double fp = 1.0 - gg * ((1.0 + q) - ((D * G) * q) * r);
        if (f > 0.0) hi = x;
        else if (f < 0.0) lo = x;
        const double dx = f * rcp64x2(fp);
        double xn = x - dx;
        conv = __builtin_fabs(dx) <= 1e-9 * x;
        if (!conv && !(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        x = xn;
    }
    const double r = rcp64x2(x);
    const double g2 = 1.0 - (m2 * r) * r;
    const double G = rsq64x2(g2);
    const double ig = g2 * G;
    const double rho = D * ig;
    const double p = gg * (x * g2 - D * ig);
    const double rG = r * G;
    w[0] = rho;
    w[1] = U[1] * rG;
    w[2] = U[2] * rG;
    w[3] = U[3] * rG;
    w[4] = p;
    return conv && rho > 0.0 && p > 0.0;
}

// One reconstructed state (rho, u_n, u_t1, u_t2, p) at a face along the first
// velocity slot: its conserved values
//   D = Gamma rho, m = Gamma rho h u, tau = Gamma^2 rho h - p - D,
// its flux F = (D v_n, m v_n + p e_n, m_n - D v_n), and its largest
// |characteristic speed|
//   (|v_n| (1 - c_s^2) + sqrt(c_s^2 (1 - v^2)(1 - v^2 c_s^2 - v_n^2 (1 - c_s^2)))) / (1 - v^2 c_s^2),
// c_s^2 = g p / (rho h).  With s = 1/sqrt(1 + u^2): Gamma = (1 + u^2) s,
// v_n = u_n s, v^2 = u^2 s^2, so a state takes one reciprocal square root,
// two reciprocals and one square root.
template <typename R>
__device__ __forceinline__ R srhd_face_state(const R w[5], R ghat, R g, R U[5], R F[5]) {
    const R uu = (w[1] * w[1] + w[2] * w[2]) + w[3] * w[3];
    const R G2 = R(1) + uu;
    const R s = rsqR(G2);
    const R G = G2 * s;
    const R vn = w[1] * s;
    const R v2 = uu * (s * s);
    const R rhoh = w[0] + ghat * w[4];
    const R cs2 = (g * w[4]) * rcpR(rhoh);
    U[0] = G * w[0];
    const R Grh = G * rhoh;
    U[1] = Grh * w[1];
    U[2] = Grh * w[2];
    U[3] = Grh * w[3];
    U[4] = (G * Grh - w[4]) - U[0];
    F[0] = U[0] * vn;
    F[1] = U[1] * vn + w[4];
    F[2] = U[2] * vn;
    F[3] = U[3] * vn;
    F[4] = U[1] - F[0];
    R disc = (R(1) - v2) * ((R(1) - v2 * cs2) - (vn * vn) * (R(1) - cs2));
    disc = disc < R(0) ? R(0) : disc;
    return (absR(vn) * (R(1) - cs2) + sqrtR(cs2 * disc)) * rcpR(R(1) - v2 * cs2);
}

// local Lax-Friedrichs flux with the larger |characteristic speed| of the
// two reconstructed states (Table 1: the SRHD module offers LF)
template <typename R>
__device__ __forceinline__ void riemann_srhd(const R wL[5], const R wR[5], R g, R igm1, R F[5]) {
    R UL[5], FL[5], UR[5], FR[5];
    const R ghat = g * igm1;
    const R sL = srhd_face_state(wL, ghat, g, UL, FL);
    const R sR = srhd_face_state(wR, ghat, g, UR, FR);
    const R sp = fmaxR(sL, sR);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = R(0.5) * ((FL[v] + FR[v]) - sp * (UR[v] - UL[v]));
}

// cell signal rate sum_d a_d / dx of a conserved SRHD state: the flux path's
// con2prim, then the largest |speed| along each axis as in srhd_face_state.
// Every kernel that forms the CFL signal of an SRHD state (the dt reduction,
// the last RK stage, the flux correction) calls this one function with the
// library's per-expression contraction, so they agree bitwise; against IEEE
// evaluation the rate differs by a few ulp.
__device__ __forceinline__ double srhd_signal(const double U[5], double g, double inv_dx, bool &ok) {
    double w[5];
    ok = srhd_con2prim_fast(U, g, w);
    const double uu = (w[1] * w[1] + w[2] * w[2]) + w[3] * w[3];
    const double is = rsq64(1.0 + uu);
    const double v2 = uu * (is * is);
    const double rhoh = w[0] + (g / (g - 1.0)) * w[4];
    const double cs2 = (g * w[4]) * rcp64(rhoh);
    const double ic = rcp64(1.0 - v2 * cs2);
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double vn = __builtin_fabs(w[1 + d]) * is;
        double disc = (1.0 - v2) * ((1.0 - v2 * cs2) - (vn * vn) * (1.0 - cs2));
        disc = disc < 0.0 ? 0.0 : disc;
        const double a = (vn * (1.0 - cs2) + sqrt64(cs2 * disc)) * ic;
        s = d == 0 ? a * inv_dx : s + a * inv_dx;
    }
    return s;
}

// ---------------------------------------------------------------------------
// ideal MHD with GLM cleaning (Sec. 2.3.3), nvar 9: (rho, m, e, B, psi)

// conserved -> primitives (rho, v, p, B, psi) with
// p = (gamma-1)((e - rho v^2/2) - B^2/2); returns whether rho > 0 and p > 0
__device__ __forceinline__ bool mhd_cons2prim(const double U[9], double gm1, double w[9]) {
    const double rho = U[0];
    const double r = rcp64(rho);
    const double vx = U[1] * r, vy = U[2] * r, vz = U[3] * r;
    const double vv = (vx * vx + vy * vy) + vz * vz;
    const double bb = (U[5] * U[5] + U[6] * U[6]) + U[7] * U[7];
    const double p = gm1 * ((U[4] - 0.5 * rho * vv) - 0.5 * bb);
    w[0] = rho; w[1] = vx; w[2] = vy; w[3] = vz; w[4] = p;
    w[5] = U[5]; w[6] = U[6]; w[7] = U[7]; w[8] = U[8];
    return rho > 0.0 && p > 0.0;
}

// Cell signal rate s = sum_d (|v_d| + c_f,d)/dx (summed x, y, z) and the GLM
// speed candidate cm = max_d (|v_d| + c_f,d), with the fast speed
// c_f^2 = ((a^2 + b^2) + sqrt((a^2 + b^2)^2 - 4 a^2 b_d^2))/2, a^2 = gamma p/rho,
// b^2 = |B|^2/rho, b_d^2 = B_d^2/rho; IEEE operations without contraction, so
// that dt and c_h are the same numbers as on the CPU.
__device__ __forceinline__ double mhd_signal(const double U[9], double gamma, double inv_dx, double &cm, bool &ok) {
#pragma clang fp contract(off)
    const double rho = U[0];
    const double r = 1.0 / rho;
    const double v[3] = {U[1] * r, U[2] * r, U[3] * r};
    const double vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    const double bb = (U[5] * U[5] + U[6] * U[6]) + U[7] * U[7];
    const double p = (gamma - 1.0) * ((U[4] - 0.5 * rho * vv) - 0.5 * bb);
    ok = rho > 0.0 && p > 0.0;
    const double a2 = gamma * p / rho;
    const double b2 = bb / rho;
    const double ss = a2 + b2;
    double s = 0.0;
    cm = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double bd2 = U[5 + d] * U[5 + d] / rho;
        double disc = ss * ss - 4.0 * a2 * bd2;
        if (disc < 0.0) disc = 0.0;
        const double c = __builtin_sqrt(0.5 * (ss + __builtin_sqrt(disc)));
        const double a = __builtin_fabs(v[d]) + c;
        s = d == 0 ? a * inv_dx : s + a * inv_dx;
        cm = a > cm ? a : cm;
    }
    return s;
}

// MHD flux across a face from rotated primitive states (rho, u_n, u_t1, u_t2,
// p, B_n, B_t1, B_t2, psi).  GLM interface step of Dedner et al. (2002):
//   B_n* = (B_nL + B_nR)/2 - (psi_R - psi_L)/(2 c_h),
//   psi* = (psi_L + psi_R)/2 - c_h (B_nR - B_nL)/2,
// both sides take B_n*, the (B_n, psi) fluxes are (psi*, c_h^2 B_n*); HLL with
// Davis fast-speed bounds on the other seven components, in the clamped
// branch-free form F = ((a F_L - b F_R) + a b (U_R - U_L))/(a - b),
// a = max(S_R, 0), b = min(S_L, 0).  Physical flux along n: mass rho u_n,
// momentum rho u u_n + (p + B^2/2) e_n - B B_n, energy
// u_n (e + p + B^2/2) - B_n (u.B), induction u_n B - B_n u.
template <typename R>
__device__ __forceinline__ void mhd_hll(const R wL[9], const R wR[9], R gamma, R igm1, R ch, R inv2ch, R F[9]) {
    const R bn = R(0.5) * (wL[5] + wR[5]) - (wR[8] - wL[8]) * inv2ch;
    const R ps = R(0.5) * (wL[8] + wR[8]) - R(0.5) * ch * (wR[5] - wL[5]);
    R U[2][9], Fs[2][9], c[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const R *w = s ? wR : wL;
        const R rho = w[0], un = w[1], u1 = w[2], u2 = w[3], p = w[4], b1 = w[6], b2 = w[7];
        const R vv = (un * un + u1 * u1) + u2 * u2;
        const R bb = (bn * bn + b1 * b1) + b2 * b2;
        const R vb = (un * bn + u1 * b1) + u2 * b2;
        const R pt = p + R(0.5) * bb;
        const R e = (p * igm1 + R(0.5) * rho * vv) + R(0.5) * bb;
        const R mn = rho * un;
        U[s][0] = rho; U[s][1] = mn; U[s][2] = rho * u1; U[s][3] = rho * u2; U[s][4] = e;
        U[s][6] = b1; U[s][7] = b2;
        Fs[s][0] = mn;
        Fs[s][1] = mn * un + pt - bn * bn;
        Fs[s][2] = U[s][2] * un - b1 * bn;
        Fs[s][3] = U[s][3] * un - b2 * bn;
        Fs[s][4] = un * (e + pt) - bn * vb;
        Fs[s][6] = un * b1 - bn * u1;
        Fs[s][7] = un * b2 - bn * u2;
        const R r = rcpR(rho);
        const R a2 = gamma * p * r, B2 = bb * r, bd2 = bn * bn * r;
        const R sum = a2 + B2;
        const R disc = fmaxR(sum * sum - R(4) * a2 * bd2, R(0));
        c[s] = sqrtR(R(0.5) * (sum + sqrtR(disc)));
    }
    const R SL = fminR(wL[1] - c[0], wR[1] - c[1]);
    const R SR = fmaxR(wL[1] + c[0], wR[1] + c[1]);
    const R ap = fmaxR(SR, R(0)), bm = fminR(SL, R(0));
    const R inv = rcpR(ap - bm);
    const R ab = ap * bm;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        if (v == 5) continue;
        F[v] = ((ap * Fs[0][v] - bm * Fs[1][v]) + ab * (U[1][v] - U[0][v])) * inv;
    }
    F[5] = ps;
    F[8] = ch * ch * bn;
}

} // namespace agile
