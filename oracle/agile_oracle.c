/*
 * agile_oracle.c -- plain FP64 CPU oracle of the block-AMR finite-volume update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * What it computes (paper: AGILE 1.0, Porth et al.):
 *   - conservation law dU/dt + div F(U) = 0 (Sec. 2.3, first equation), no sources;
 *   - Euler system with the ideal-gas closure e = p/(gamma-1) + rho v^2/2
 *     (Sec. 2.3.1, mass/momentum/energy equations and the closure equation);
 *   - physical flux F_d = U v_d + (0, P e_d, P v_d) of the Euler equations
 *     (Sec. 2.3.1), P the pressure (plus B^2/2 and the magnetic stress and
 *     energy terms of Sec. 2.3.3 for MHD);
 *   - ideal MHD with GLM divergence cleaning (Sec. 2.3.3: momentum, energy
 *     and induction equations, the GLM equation and its exact exponential
 *     decay of psi by operator splitting);
 *   - PLM reconstruction with the minmod limiter (named in Sec. 4.5 for the
 *     Orszag-Tang run) or the van Leer limiter (the benchmark of Sec. 3.1);
 *   - HLL / HLLC / local Lax-Friedrichs fluxes (Table 1; LF is the benchmark
 *     flux of Sec. 3.1);
 *   - two ghost layers per block side (Sec. 3.1);
 *   - ghost fill across blocks: same-level copy, restriction and limited
 *     prolongation at 2:1 level jumps (Sec. 2.1.2 lists prolongation /
 *     restriction and ghost exchange as device work; Sec. 2.1.3 names the
 *     same-level / finer / coarser neighbour relations);
 *   - special relativistic hydrodynamics (the D, m, tau conservation laws of
 *     Sec. 2.3.4, ideal-gas enthalpy, primitives
 *     rho, four-velocity, p; con2prim by 1-D root finding in xi = Gamma^2 rho h;
 *     LF flux, the solver Table 1 lists for this module);
 *   - a global CFL time step (the "Set dt" node of the time-evolution flow
 *     chart, Sec. 2.1.2);
 *   - two- and three-stage SSP Runge-Kutta steps in Shu-Osher form (the
 *     paper's runs use an unnamed three-step RK, Sec. 3.1, read here as SSP-RK3).
 *
 * The paper does not write the limiter, Riemann solvers, RK scheme, CFL rule,
 * prolongation, restriction or coarse-fine flux correction as formulas.  Where
 * it is silent this file follows the named textbook method and the reading is
 * stated at the function.  Every reading is also listed in the design notes.
 *
 * Independence from the GPU path: ghost values are found by recursive point
 * location on the block tree (V_l(x) below), not by the task tables the HIP
 * library builds, and coarse-fine fluxes are replaced inside the divergence
 * rather than corrected afterwards.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math), so
 * that bitwise invariants (mirror symmetry, uniform-AMR == single grid) hold.
 *
 * Parity pins: see the oracle tests (exact Sod solution, conservation, block
 * decomposition invariance, free-stream, linear prolongation, second-order
 * convergence, mirror symmetry, HLLC contact, dt closed form, GLM decay).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 2          /* ghost layers per side (Sec. 3.1) */
#define MAXLEV 12
#define MAXVAR 9

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENONPHYSICAL = -5 };
enum { PHYS_EULER = 0, PHYS_MHD = 1, PHYS_SRHD = 2 };
enum { RS_HLL = 0, RS_HLLC = 1, RS_LF = 2 };
enum { LIM_MINMOD = 0, LIM_VANLEER = 1 };

/* conserved variable order: rho, m_x, m_y, m_z, e [, B_x, B_y, B_z, psi] */
enum { V_RHO = 0, V_MX = 1, V_E = 4, V_BX = 5, V_PSI = 8 };

typedef struct orc_mesh {
    int physics, riemann, nvar;
    int limiter;               /* slope limiter of the reconstruction (LIM_*) */
    int rk;                    /* Runge-Kutta stages: 2 or 3 (SSP) */
    double gamma, cfl, glm_alpha;
    int bn[3];                 /* interior cells per block axis */
    int base[3];               /* blocks per axis on level 1 */
    int max_level;
    double lo[3], hi[3];
    double dx1;                /* cubic cell size on level 1 */
    int nleaf;
    int *lev;                  /* [nleaf] */
    long *bidx;                /* [nleaf][3] block coordinates on its level */
    int pn[3];                 /* padded dims bn + 2*NG */
    long pvol;                 /* padded cells per variable */
    double *u;                 /* [nleaf][nvar][pvol] padded conserved state */
    long nbl[MAXLEV + 1][3];   /* blocks per axis on each level */
    int *lookup[MAXLEV + 1];   /* dense map block coords -> leaf index or -1 */
    double ch;                 /* GLM cleaning speed c_h = c_max of the step */
} orc_mesh;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */

static double nanv(void) { return nan(""); }

static long wrapl(long c, long n) {
    long r = c % n;
    return r < 0 ? r + n : r;
}

static int lookup_leaf(const orc_mesh *m, int l, const long b[3]) {
    if (l < 1 || l > m->max_level) return -1;
    const long *nb = m->nbl[l];
    return m->lookup[l][(b[2] * nb[1] + b[1]) * nb[0] + b[0]];
}

static long pidx(const orc_mesh *m, int i, int j, int k) {
    return ((long)(k + NG) * m->pn[1] + (j + NG)) * m->pn[0] + (i + NG);
}

static double *leaf_var(const orc_mesh *m, int leaf, int v) {
    return m->u + ((long)leaf * m->nvar + v) * m->pvol;
}

static double cell_size(const orc_mesh *m, int l) {
    return ldexp(m->dx1, -(l - 1));
}

/* minmod(a, b): zero unless a and b have the same strict sign, else the
 * argument of smaller magnitude; on a tie a is returned.  Sign tests rather
 * than a*b so that tiny products cannot underflow to zero. */
static double minmod(double a, double b) {
    if (a > 0.0 && b > 0.0) return (a <= b) ? a : b;
    if (a < 0.0 && b < 0.0) return (a >= b) ? a : b;
    return 0.0;
}

/* van Leer's limited slope of two one-sided differences: the harmonic mean
 * 2ab/(a+b) when a and b have the same strict sign, else zero. */
static double vanleer(double a, double b) {
    if ((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0)) return (2.0 * a * b) / (a + b);
    return 0.0;
}

/* reconstruction slope with the mesh's limiter (the prolongation keeps minmod) */
static double slope(const orc_mesh *m, double a, double b) {
    return m->limiter == LIM_VANLEER ? vanleer(a, b) : minmod(a, b);
}

/* ------------------------------------------------------------------ */
/* Ghost values by point location on the tree: V_l(c) is the value of the
 * level-l cell with integer coordinates c (periodic wrap on level l).
 *   - a level-l leaf holds c              -> its stored interior value;
 *   - c lies in a coarser leaf            -> limited linear prolongation from
 *                                            the parent cell on level l-1;
 *   - c is covered by finer leaves        -> mean of the 8 children on l+1.
 * Restriction and prolongation act on conserved variables (reading: the paper
 * does not say which variables; conserved ones keep both operations
 * conservative in exact arithmetic), except that the SRHD prolongation
 * interpolates primitives (prolong_value_srhd).                         */

static double V(const orc_mesh *m, int l, const long cin[3], int v);

/* minmod-limited linear prolongation (reading of the "prolongation" named in
 * Sec. 2.1.2): slope per axis from the parent's two axis neighbours, child
 * value = parent + (+/-1/4) slope per axis, added in x, y, z order.       */
static double prolong_value(const orc_mesh *m, int l, const long c[3], int v) {
    long C[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
    double vc = V(m, l - 1, C, v);
    double val = vc;
    for (int d = 0; d < 3; ++d) {
        long Cm[3] = {C[0], C[1], C[2]}, Cp[3] = {C[0], C[1], C[2]};
        Cm[d] -= 1;
        Cp[d] += 1;
        double sig = minmod(vc - V(m, l - 1, Cm, v), V(m, l - 1, Cp, v) - vc);
        double q = 0.25 * sig;
        val = (c[d] & 1) ? val + q : val - q;
    }
    return val;
}

static int srhd_con2prim(double g, const double *U, double *w, int *steps);
static void srhd_prim_to_cons(double g, const double *w, double *U);

/* SRHD: the same limited linear prolongation applied to the primitives
 * (rho, Gamma v, p) of the parent and its axis neighbours, and the child's
 * primitives converted back to (D, m, tau).  Reading: limited interpolation
 * of the conserved variables can give |m| > tau + D (no physical state)
 * next to a strong relativistic shock; minmod-limited primitives stay between
 * neighbouring values, so rho, p > 0 and every u is causal.  A parent stencil
 * with a non-physical cell gives NaN.                                    */
static double prolong_value_srhd(const orc_mesh *m, int l, const long c[3], int v) {
    const double g = m->gamma;
    long C[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
    double U[5], wc[5], w[5];
    for (int q = 0; q < 5; ++q) U[q] = V(m, l - 1, C, q);
    if (srhd_con2prim(g, U, wc, NULL) != ORC_OK) return NAN;
    for (int q = 0; q < 5; ++q) w[q] = wc[q];
    for (int d = 0; d < 3; ++d) {
        long Cm[3] = {C[0], C[1], C[2]}, Cp[3] = {C[0], C[1], C[2]};
        Cm[d] -= 1;
        Cp[d] += 1;
        double Um[5], Up[5], wm[5], wp[5];
        for (int q = 0; q < 5; ++q) {
            Um[q] = V(m, l - 1, Cm, q);
            Up[q] = V(m, l - 1, Cp, q);
        }
        if (srhd_con2prim(g, Um, wm, NULL) != ORC_OK || srhd_con2prim(g, Up, wp, NULL) != ORC_OK) return NAN;
        for (int q = 0; q < 5; ++q) {
            double sq = 0.25 * minmod(wc[q] - wm[q], wp[q] - wc[q]);
            w[q] = (c[d] & 1) ? w[q] + sq : w[q] - sq;
        }
    }
    srhd_prim_to_cons(g, w, U);
    return U[v];
}

/* restriction: volume mean of the 8 children, summed pairwise
 * ((c000+c100)+(c010+c110)) + ((c001+c101)+(c011+c111)), then times 1/8. */
static double restrict_value(const orc_mesh *m, int l, const long c[3], int v) {
    double ch[8];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                long f[3] = {2 * c[0] + dx, 2 * c[1] + dy, 2 * c[2] + dz};
                ch[dx + 2 * dy + 4 * dz] = V(m, l + 1, f, v);
            }
    double s = ((ch[0] + ch[1]) + (ch[2] + ch[3])) + ((ch[4] + ch[5]) + (ch[6] + ch[7]));
    return s * 0.125;
}

static double V(const orc_mesh *m, int l, const long cin[3], int v) {
    long c[3], b[3];
    for (int d = 0; d < 3; ++d) {
        c[d] = wrapl(cin[d], m->nbl[l][d] * m->bn[d]);
        b[d] = c[d] / m->bn[d];
    }
    int leaf = lookup_leaf(m, l, b);
    if (leaf >= 0) {
        const double *u = leaf_var(m, leaf, v);
        return u[pidx(m, (int)(c[0] - b[0] * m->bn[0]), (int)(c[1] - b[1] * m->bn[1]),
                      (int)(c[2] - b[2] * m->bn[2]))];
    }
    for (int L = l - 1; L >= 1; --L) {
        long bb[3];
        for (int d = 0; d < 3; ++d) bb[d] = (c[d] >> (l - L)) / m->bn[d];
        if (lookup_leaf(m, L, bb) >= 0)
            return m->physics == PHYS_SRHD ? prolong_value_srhd(m, l, c, v) : prolong_value(m, l, c, v);
    }
    return restrict_value(m, l, c, v);
}

/* Fill the two face-ghost layers of every leaf with V_l at the ghost cell
 * centres.  Edge and corner ghosts stay NaN: the dimension-by-dimension
 * update never reads them.                                                */
void orc_fill_ghosts(orc_mesh *m) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int leaf = 0; leaf < m->nleaf; ++leaf) {
        const int l = m->lev[leaf];
        const long *b = m->bidx + 3L * leaf;
        for (int d = 0; d < 3; ++d) {
            const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
            for (int side = 0; side < 2; ++side)
                for (int g = 0; g < NG; ++g) {
                    int n = side ? m->bn[d] + g : -NG + g;
                    for (int a2 = 0; a2 < m->bn[t2]; ++a2)
                        for (int a1 = 0; a1 < m->bn[t1]; ++a1) {
                            int loc[3];
                            loc[d] = n;
                            loc[t1] = a1;
                            loc[t2] = a2;
                            long c[3];
                            for (int e = 0; e < 3; ++e) c[e] = b[e] * m->bn[e] + loc[e];
                            long p = pidx(m, loc[0], loc[1], loc[2]);
                            for (int v = 0; v < m->nvar; ++v) leaf_var(m, leaf, v)[p] = V(m, l, c, v);
                        }
                }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Physics: primitive variables, physical flux, signal speeds.          */
/* Euler primitives: rho, v_x, v_y, v_z, p.
 * MHD primitives:   rho, v_x, v_y, v_z, p, B_x, B_y, B_z, psi.
 * SRHD primitives:  rho, u_x, u_y, u_z, p with u = Gamma v the spatial part
 * of the four-velocity (the primitive set of the relativistic section).   */

/* SRHD con2prim.  Reading of the root finding in xi = Gamma^2 rho h the paper
 * cites: with e = tau + D, |m| and the ideal gas h = 1 + g/(g-1) p/rho,
 *   1/Gamma^2 = 1 - m^2/xi^2,  rho = D/Gamma,
 *   p(xi) = (g-1)/g (xi/Gamma^2 - D/Gamma),
 *   f(xi) = xi - p(xi) - e = 0,
 *   f'(xi) = 1 - (g-1)/g (1 + m^2/xi^2 - D Gamma m^2/xi^3);
 * f increases on (|m|, g e] with f(|m|) <= 0 < f(g e), so Newton steps are
 * kept inside that bracket (bisection when a step leaves it), starting at
 * xi = e, until a step changes xi by at most 1e-15 xi (at most 100 steps). */
static int srhd_con2prim(double g, const double *U, double *w, int *steps) {
    const double D = U[0], e = U[4] + U[0];
    const double m2 = (U[1] * U[1] + U[2] * U[2]) + U[3] * U[3];
    const double mm = sqrt(m2);
    const double gg = (g - 1.0) / g;
    double lo = mm, hi = g * e;
    if (!(D > 0.0) || !(hi > lo)) return ORC_ENONPHYSICAL;
    double x = e;
    if (!(x > lo)) x = 0.5 * (lo + hi);
    int conv = 0, it = 0;
    for (; it < 100 && !conv; ++it) {
        const double q = m2 / (x * x);
        const double g2 = 1.0 - q;
        const double ig = sqrt(g2);
        const double G = 1.0 / ig;
        const double p = gg * (x * g2 - D * ig);
        const double f = (x - p) - e;
        const double fp = 1.0 - gg * ((1.0 + q) - D * G * q / x);
        if (f > 0.0) hi = x;
        else if (f < 0.0) lo = x;
        double xn = x - f / fp;
        /* a step within the tolerance is convergence, also when rounding
           leaves it on a bracket end (or f is exactly 0): bisecting there
           would throw the root away */
        conv = fabs(xn - x) <= 1e-15 * xn;
        if (!conv && !(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        x = xn;
    }
    if (steps) *steps = it;
    const double g2 = 1.0 - m2 / (x * x);
    const double ig = sqrt(g2);
    const double G = 1.0 / ig;
    const double rho = D * ig;
    const double p = gg * (x * g2 - D * ig);
    w[0] = rho;
    for (int a = 0; a < 3; ++a) w[1 + a] = (U[1 + a] / x) * G;
    w[4] = p;
    if (!conv || !(rho > 0.0) || !(p > 0.0)) return ORC_ENONPHYSICAL;
    return ORC_OK;
}

static int cons_to_prim(const orc_mesh *m, const double *U, double *w) {
    const double g = m->gamma;
    if (m->physics == PHYS_SRHD) return srhd_con2prim(g, U, w, NULL);
    double rho = U[V_RHO];
    double r = 1.0 / rho;
    double vx = U[1] * r, vy = U[2] * r, vz = U[3] * r;
    double vv = (vx * vx + vy * vy) + vz * vz;
    double p;
    if (m->physics == PHYS_EULER) {
        p = (g - 1.0) * (U[V_E] - 0.5 * rho * vv);
    } else {
        double bb = (U[5] * U[5] + U[6] * U[6]) + U[7] * U[7];
        p = (g - 1.0) * ((U[V_E] - 0.5 * rho * vv) - 0.5 * bb);
    }
    w[0] = rho; w[1] = vx; w[2] = vy; w[3] = vz; w[4] = p;
    if (m->physics == PHYS_MHD) {
        w[5] = U[5]; w[6] = U[6]; w[7] = U[7]; w[8] = U[8];
    }
    if (!(rho > 0.0) || !(p > 0.0)) return ORC_ENONPHYSICAL;
    return ORC_OK;
}

/* SRHD: Gamma = sqrt(1 + u^2), h = 1 + g/(g-1) p/rho,
 * D = Gamma rho, m = Gamma rho h u (= Gamma^2 rho h v), tau = Gamma^2 rho h - p - D. */
static void srhd_prim_to_cons(double g, const double *w, double *U) {
    const double uu = (w[1] * w[1] + w[2] * w[2]) + w[3] * w[3];
    const double G = sqrt(1.0 + uu);
    const double rhoh = w[0] + (g / (g - 1.0)) * w[4];
    U[0] = G * w[0];
    for (int a = 0; a < 3; ++a) U[1 + a] = (G * rhoh) * w[1 + a];
    U[4] = ((G * G) * rhoh - w[4]) - U[0];
}

static void prim_to_cons(const orc_mesh *m, const double *w, double *U) {
    const double g = m->gamma;
    if (m->physics == PHYS_SRHD) {
        srhd_prim_to_cons(g, w, U);
        return;
    }
    double rho = w[0];
    double vv = (w[1] * w[1] + w[2] * w[2]) + w[3] * w[3];
    U[0] = rho;
    U[1] = rho * w[1]; U[2] = rho * w[2]; U[3] = rho * w[3];
    if (m->physics == PHYS_EULER) {
        U[4] = w[4] / (g - 1.0) + 0.5 * rho * vv;
    } else {
        double bb = (w[5] * w[5] + w[6] * w[6]) + w[7] * w[7];
        U[4] = (w[4] / (g - 1.0) + 0.5 * rho * vv) + 0.5 * bb;
        U[5] = w[5]; U[6] = w[6]; U[7] = w[7]; U[8] = w[8];
    }
}

/* Physical flux along axis d from primitives, read off the conservation
 * laws of Sec. 2.3.1: every conserved quantity is carried with the normal
 * velocity, F_d = U v_d, and the pressure adds its force to the normal
 * momentum and its work to the energy, + (0, P e_d, P v_d).  For MHD
 * (Sec. 2.3.3) P is the total pressure p + B^2/2, the magnetic stress
 * -B B_d enters the momentum and -B_d (v.B) the energy, and the induction
 * flux is v_d B - B_d v; the normal B and psi components are set by the GLM
 * interface step, not here.  SRHD (Sec. 2.3.4): the same advective form with
 * the three-velocity, U = (D, m, tau).                                  */
static void phys_flux(const orc_mesh *m, const double *w, int d, double *F) {
    double U[MAXVAR];
    prim_to_cons(m, w, U);
    double vd, P;
    if (m->physics == PHYS_SRHD) {
        vd = w[1 + d] / sqrt(1.0 + ((w[1] * w[1] + w[2] * w[2]) + w[3] * w[3]));
        P = w[4];
    } else {
        vd = w[1 + d];
        P = w[4];
        if (m->physics == PHYS_MHD)
            P = P + 0.5 * ((w[5] * w[5] + w[6] * w[6]) + w[7] * w[7]);
    }
    for (int k = 0; k < 5; ++k) F[k] = U[k] * vd;
    F[1 + d] = F[1 + d] + P;
    F[4] = F[4] + P * vd;
    if (m->physics == PHYS_MHD) {
        const double *v = w + 1, *B = w + 5;
        const double vb = (v[0] * B[0] + v[1] * B[1]) + v[2] * B[2];
        for (int a = 0; a < 3; ++a) F[1 + a] = F[1 + a] - B[a] * B[d];
        F[4] = F[4] - B[d] * vb;
        for (int a = 0; a < 3; ++a) F[5 + a] = v[d] * B[a] - B[d] * v[a];
        F[5 + d] = 0.0;   /* replaced by the GLM flux psi* */
        F[8] = 0.0;       /* replaced by the GLM flux c_h^2 B_n* */
    }
}

/* sound speed (Euler) or fast magnetosonic speed along d (MHD):
 * c_f^2 = ( (a^2+b^2) + sqrt((a^2+b^2)^2 - 4 a^2 b_d^2) ) / 2,
 * a^2 = gamma p / rho, b^2 = |B|^2/rho, b_d^2 = B_d^2/rho.            */
/* SRHD: the largest |characteristic speed| along d,
 * max |lambda+-| = (|v_d| (1 - c_s^2) + c_s sqrt((1 - v^2)(1 - v^2 c_s^2 - v_d^2 (1 - c_s^2)))) / (1 - v^2 c_s^2),
 * c_s^2 = g p / (rho h) (the textbook eigenvalues of the SRHD flux Jacobian). */
static double srhd_speed(double g, const double *w, int d) {
    const double uu = (w[1] * w[1] + w[2] * w[2]) + w[3] * w[3];
    const double G2 = 1.0 + uu;
    const double v2 = uu / G2;
    const double vd = w[1 + d] / sqrt(G2);
    const double h = 1.0 + (g / (g - 1.0)) * (w[4] / w[0]);
    const double cs2 = (g * w[4]) / (w[0] * h);
    double disc = (1.0 - v2) * ((1.0 - v2 * cs2) - (vd * vd) * (1.0 - cs2));
    if (disc < 0.0) disc = 0.0;
    return (fabs(vd) * (1.0 - cs2) + sqrt(cs2) * sqrt(disc)) / (1.0 - v2 * cs2);
}

static double signal_speed(const orc_mesh *m, const double *w, int d) {
    double a2 = m->gamma * w[4] / w[0];
    if (m->physics == PHYS_EULER) return sqrt(a2);
    double bb = (w[5] * w[5] + w[6] * w[6]) + w[7] * w[7];
    double b2 = bb / w[0];
    double bd2 = w[5 + d] * w[5 + d] / w[0];
    double s = a2 + b2;
    double disc = s * s - 4.0 * a2 * bd2;
    if (disc < 0.0) disc = 0.0;
    return sqrt(0.5 * (s + sqrt(disc)));
}

/* Riemann flux at a face normal to axis d from left/right primitive states.
 * Wave-speed estimates of Davis: S_L = min(u_L - c_L, u_R - c_R),
 * S_R = max(u_L + c_L, u_R + c_R) (reading: the paper does not name them).
 * HLL: Harten-Lax-van Leer, three-case form (Toro 2009, Sec. 10.3).
 * HLLC: Toro 2009, Sec. 10.4, contact speed S* of Batten et al. and the
 * star flux written as F*_K = (S*(S_K U_K - F_K) + S_K P_K D*)/(S_K - S*),
 * D* = (0, e_d, S*), P_K = p_K + rho_K (S_K - u_K)(S* - u_K), taking P_K
 * from the side K that is used.
 * MHD: Dedner et al. (2002) GLM interface values for (B_d, psi), then HLL on
 * the remaining components with fast speeds (Table 1: mhd offers HLL).   */
static void riemann(const orc_mesh *m, const double *wL, const double *wR, int d, double *F) {
    const int nv = m->nvar;
    double wl[MAXVAR], wr[MAXVAR];
    memcpy(wl, wL, sizeof(double) * nv);
    memcpy(wr, wR, sizeof(double) * nv);
    double bn_star = 0.0, psi_star = 0.0;
    if (m->physics == PHYS_MHD) {
        const double ch = m->ch;
        double bL = wl[5 + d], bR = wr[5 + d], pL = wl[8], pR = wr[8];
        bn_star = 0.5 * (bL + bR) - (pR - pL) / (2.0 * ch);
        psi_star = 0.5 * (pL + pR) - 0.5 * ch * (bR - bL);
        wl[5 + d] = bn_star;
        wr[5 + d] = bn_star;
    }
    double cL = signal_speed(m, wl, d), cR = signal_speed(m, wr, d);
    double uL = wl[1 + d], uR = wr[1 + d];
    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);
    double UL[MAXVAR], UR[MAXVAR], FL[MAXVAR], FR[MAXVAR];
    prim_to_cons(m, wl, UL);
    prim_to_cons(m, wr, UR);
    phys_flux(m, wl, d, FL);
    phys_flux(m, wr, d, FR);

    if (m->physics == PHYS_SRHD) {
        /* local Lax-Friedrichs with the larger |characteristic speed| */
        double s = fmax(srhd_speed(m->gamma, wl, d), srhd_speed(m->gamma, wr, d));
        for (int v = 0; v < nv; ++v) F[v] = 0.5 * ((FL[v] + FR[v]) - s * (UR[v] - UL[v]));
    } else if (m->riemann == RS_LF) {
        /* local Lax-Friedrichs (Rusanov): one speed, the larger |u| + c of the
         * two states (the "tvdlf" family named in Table 1) */
        double s = fmax(fabs(uL) + cL, fabs(uR) + cR);
        for (int v = 0; v < nv; ++v) F[v] = 0.5 * ((FL[v] + FR[v]) - s * (UR[v] - UL[v]));
    } else if (SL >= 0.0) {
        memcpy(F, FL, sizeof(double) * nv);
    } else if (SR <= 0.0) {
        memcpy(F, FR, sizeof(double) * nv);
    } else if (m->riemann == RS_HLL || m->physics == PHYS_MHD) {
        for (int v = 0; v < nv; ++v)
            F[v] = ((SR * FL[v] - SL * FR[v]) + (SL * SR) * (UR[v] - UL[v])) / (SR - SL);
    } else {
        double dL = wl[0] * (SL - uL), dR = wr[0] * (SR - uR);
        double Ss = ((wr[4] - wl[4]) + (uL * dL - uR * dR)) / (dL - dR);
        const double *wK, *UK, *FK;
        double SK, dK;
        if (Ss >= 0.0) { wK = wl; UK = UL; FK = FL; SK = SL; dK = dL; }
        else           { wK = wr; UK = UR; FK = FR; SK = SR; dK = dR; }
        double PK = wK[4] + dK * (Ss - wK[1 + d]);
        double den = SK - Ss;
        for (int v = 0; v < 5; ++v) {
            double Dv = (v == 1 + d) ? 1.0 : (v == 4 ? Ss : 0.0);
            F[v] = (Ss * (SK * UK[v] - FK[v]) + (SK * PK) * Dv) / den;
        }
    }
    if (m->physics == PHYS_MHD) {
        F[5 + d] = psi_star;
        F[8] = (m->ch * m->ch) * bn_star;
    }
}

/* ------------------------------------------------------------------ */
/* neighbour classification of a leaf face: 0 same level, -1 coarser,
 * +1 finer (2:1 balance assumed).                                      */
static int face_relation(const orc_mesh *m, int leaf, int d, int side) {
    const int l = m->lev[leaf];
    long b[3] = {m->bidx[3L * leaf], m->bidx[3L * leaf + 1], m->bidx[3L * leaf + 2]};
    b[d] += side ? 1 : -1;
    b[d] = wrapl(b[d], m->nbl[l][d]);
    if (lookup_leaf(m, l, b) >= 0) return 0;
    if (l > 1) {
        long pb[3] = {b[0] >> 1, b[1] >> 1, b[2] >> 1};
        if (lookup_leaf(m, l - 1, pb) >= 0) return -1;
    }
    return 1;
}

/* per-leaf work arrays */
typedef struct {
    double *W;      /* [nvar][pvol] primitives */
    double *S;      /* [nvar][pvol] slopes along the current axis */
    double *F[3];   /* [nvar][faces] fluxes per axis */
} leaf_work;

static long nfaces(const orc_mesh *m, int d) {
    long n = 1;
    for (int e = 0; e < 3; ++e) n *= (e == d) ? m->bn[e] + 1 : m->bn[e];
    return n;
}

/* face index of (i,j,k) on axis d: i along d runs 0..bn[d] */
static long fidx(const orc_mesh *m, int d, int i, int j, int k) {
    int nx = m->bn[0] + (d == 0), ny = m->bn[1] + (d == 1);
    return ((long)k * ny + j) * nx + i;
}

/* Primitives on the interior and face ghosts, PLM slopes per axis, and the
 * Riemann flux at every face of the leaf (faces 0..bn along each axis).   */
static int leaf_fluxes(const orc_mesh *m, int leaf, leaf_work *wk) {
    const int nv = m->nvar;
    const int *bn = m->bn;
    int err = ORC_OK;
    for (int k = -NG; k < bn[2] + NG; ++k)
        for (int j = -NG; j < bn[1] + NG; ++j)
            for (int i = -NG; i < bn[0] + NG; ++i) {
                int out = (i < 0 || i >= bn[0]) + (j < 0 || j >= bn[1]) + (k < 0 || k >= bn[2]);
                long p = pidx(m, i, j, k);
                if (out > 1) {
                    for (int v = 0; v < nv; ++v) wk->W[v * m->pvol + p] = nanv();
                    continue;
                }
                double U[MAXVAR], w[MAXVAR];
                for (int v = 0; v < nv; ++v) U[v] = leaf_var(m, leaf, v)[p];
                if (cons_to_prim(m, U, w) != ORC_OK) err = ORC_ENONPHYSICAL;
                for (int v = 0; v < nv; ++v) wk->W[v * m->pvol + p] = w[v];
            }
    if (err) return err;
    for (int d = 0; d < 3; ++d) {
        const long st = (d == 0) ? 1 : (d == 1 ? m->pn[0] : (long)m->pn[0] * m->pn[1]);
        /* slopes at cells -1..bn[d] along d, interior across */
        for (int k = -1; k <= bn[2]; ++k)
            for (int j = -1; j <= bn[1]; ++j)
                for (int i = -1; i <= bn[0]; ++i) {
                    int loc[3] = {i, j, k};
                    int ok = 1;
                    for (int e = 0; e < 3; ++e)
                        if (e != d && (loc[e] < 0 || loc[e] >= bn[e])) ok = 0;
                    if (!ok) continue;
                    long p = pidx(m, i, j, k);
                    for (int v = 0; v < nv; ++v) {
                        const double *w = wk->W + v * m->pvol;
                        wk->S[v * m->pvol + p] = slope(m, w[p] - w[p - st], w[p + st] - w[p]);
                    }
                }
        long nf = nfaces(m, d);
        int nx = bn[0] + (d == 0), ny = bn[1] + (d == 1), nz = bn[2] + (d == 2);
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    long pr = pidx(m, i, j, k);      /* cell on the right of the face */
                    long pl = pr - st;               /* cell on the left */
                    double wL[MAXVAR], wR[MAXVAR], F[MAXVAR];
                    for (int v = 0; v < nv; ++v) {
                        const double *w = wk->W + v * m->pvol, *s = wk->S + v * m->pvol;
                        wL[v] = w[pl] + 0.5 * s[pl];
                        wR[v] = w[pr] - 0.5 * s[pr];
                    }
                    riemann(m, wL, wR, d, F);
                    long f = fidx(m, d, i, j, k);
                    for (int v = 0; v < nv; ++v) wk->F[d][v * nf + f] = F[v];
                }
    }
    return ORC_OK;
}

/* Coarse-fine flux correction (reading: the paper does not describe it; the
 * standard conservative treatment is used): on a coarse leaf face whose
 * neighbour region is finer, each coarse face flux is replaced by the mean
 * of the 4 fine face fluxes covering it, ((f00+f10)+(f01+f11))/4 with the
 * first index along the lower tangential axis.                          */
static void correct_fluxes(const orc_mesh *m, double **F) {
    const int nv = m->nvar;
    const int *bn = m->bn;
#pragma omp parallel for schedule(dynamic, 4)
    for (int leaf = 0; leaf < m->nleaf; ++leaf) {
        const int l = m->lev[leaf];
        const long *b = m->bidx + 3L * leaf;
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) {
                if (face_relation(m, leaf, d, side) != 1) continue;
                const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;   /* lower, upper tangential axes */
                long nf_c = nfaces(m, d);
                int fl = side ? bn[d] : 0;                                /* coarse local face index */
                long Xf = 2 * (b[d] * bn[d] + fl);                        /* fine face coordinate */
                long fine_cell_d = side ? Xf : Xf - 1;                    /* fine cell across the face */
                for (int a2 = 0; a2 < bn[t2]; ++a2)
                    for (int a1 = 0; a1 < bn[t1]; ++a1) {
                        double fsum[MAXVAR][4];
                        for (int q2 = 0; q2 < 2; ++q2)
                            for (int q1 = 0; q1 < 2; ++q1) {
                                long fc[3];
                                fc[d] = fine_cell_d;
                                fc[t1] = 2 * (b[t1] * bn[t1] + a1) + q1;
                                fc[t2] = 2 * (b[t2] * bn[t2] + a2) + q2;
                                long fb[3];
                                int floc[3];
                                for (int e = 0; e < 3; ++e) {
                                    fc[e] = wrapl(fc[e], m->nbl[l + 1][e] * bn[e]);
                                    fb[e] = fc[e] / bn[e];
                                    floc[e] = (int)(fc[e] - fb[e] * bn[e]);
                                }
                                int fleaf = lookup_leaf(m, l + 1, fb);
                                /* the fine leaf's face: its +d face if it lies below, else its -d face */
                                floc[d] = side ? 0 : bn[d];
                                long nf_f = nf_c;
                                long ff = fidx(m, d, floc[0], floc[1], floc[2]);
                                for (int v = 0; v < nv; ++v) fsum[v][q1 + 2 * q2] = F[3 * fleaf + d][v * nf_f + ff];
                            }
                        int loc[3];
                        loc[d] = fl;
                        loc[t1] = a1;
                        loc[t2] = a2;
                        long fc = fidx(m, d, loc[0], loc[1], loc[2]);
                        for (int v = 0; v < nv; ++v)
                            F[3 * leaf + d][v * nf_c + fc] =
                                ((fsum[v][0] + fsum[v][1]) + (fsum[v][2] + fsum[v][3])) * 0.25;
                    }
            }
    }
}

/* L(U) = -[(Fx+ - Fx-) + (Fy+ - Fy-) + (Fz+ - Fz-)] / dx on every interior
 * cell of every leaf, after filling ghosts from the current state.        */
static int compute_rhs(orc_mesh *m, double *L) {
    const int nv = m->nvar;
    const int *bn = m->bn;
    const long ncell = (long)bn[0] * bn[1] * bn[2];
    orc_fill_ghosts(m);
    double **F = (double **)calloc(3L * m->nleaf, sizeof(double *));
    if (!F) return ORC_ENOMEM;
    int err = ORC_OK;
#pragma omp parallel
    {
        leaf_work wk;
        wk.W = (double *)malloc(sizeof(double) * nv * m->pvol);
        wk.S = (double *)malloc(sizeof(double) * nv * m->pvol);
#pragma omp for schedule(dynamic, 2)
        for (int leaf = 0; leaf < m->nleaf; ++leaf) {
            for (int d = 0; d < 3; ++d) {
                F[3 * leaf + d] = (double *)malloc(sizeof(double) * nv * nfaces(m, d));
                wk.F[d] = F[3 * leaf + d];
            }
            int e = leaf_fluxes(m, leaf, &wk);
            if (e) {
#pragma omp critical
                err = e;
            }
        }
        free(wk.W);
        free(wk.S);
    }
    if (!err) {
        correct_fluxes(m, F);
#pragma omp parallel for schedule(static)
        for (int leaf = 0; leaf < m->nleaf; ++leaf) {
            const double dx = cell_size(m, m->lev[leaf]);
            long nf[3] = {nfaces(m, 0), nfaces(m, 1), nfaces(m, 2)};
            for (int v = 0; v < nv; ++v) {
                const double *fx = F[3 * leaf] + v * nf[0];
                const double *fy = F[3 * leaf + 1] + v * nf[1];
                const double *fz = F[3 * leaf + 2] + v * nf[2];
                double *Lv = L + ((long)leaf * nv + v) * ncell;
                for (int k = 0; k < bn[2]; ++k)
                    for (int j = 0; j < bn[1]; ++j)
                        for (int i = 0; i < bn[0]; ++i) {
                            double dfx = fx[fidx(m, 0, i + 1, j, k)] - fx[fidx(m, 0, i, j, k)];
                            double dfy = fy[fidx(m, 1, i, j + 1, k)] - fy[fidx(m, 1, i, j, k)];
                            double dfz = fz[fidx(m, 2, i, j, k + 1)] - fz[fidx(m, 2, i, j, k)];
                            Lv[((long)k * bn[1] + j) * bn[0] + i] = -((dfx + dfy) + dfz) / dx;
                        }
            }
        }
    }
    for (long q = 0; q < 3L * m->nleaf; ++q) free(F[q]);
    free(F);
    return err;
}

/* ------------------------------------------------------------------ */
/* public API                                                          */

static void set_err(char *err, int errlen, const char *msg) {
    if (err && errlen > 0) {
        strncpy(err, msg, (size_t)errlen - 1);
        err[errlen - 1] = 0;
    }
}

void orc_destroy(orc_mesh *m) {
    if (!m) return;
    for (int l = 0; l <= MAXLEV; ++l) free(m->lookup[l]);
    free(m->lev);
    free(m->bidx);
    free(m->u);
    free(m);
}

/* desc: nleaf rows of (level, ix, iy, iz); block coordinates on that level.
 * The leaves must tile the periodic domain without overlap; 2:1 face balance
 * is required for prolongation and flux correction.                     */
orc_mesh *orc_create(int physics, int riemann, double gamma, double cfl, double glm_alpha,
                     const int *bn, const int *base, const double *lo, const double *hi,
                     int max_level, int nleaf, const int *desc, char *err, int errlen) {
    if (physics != PHYS_EULER && physics != PHYS_MHD && physics != PHYS_SRHD) { set_err(err, errlen, "bad physics"); return NULL; }
    if (physics == PHYS_SRHD && riemann != RS_LF) { set_err(err, errlen, "SRHD takes the LF flux"); return NULL; }
    if (riemann != RS_HLL && riemann != RS_HLLC && riemann != RS_LF) { set_err(err, errlen, "bad riemann"); return NULL; }
    if (max_level < 1 || max_level > MAXLEV) { set_err(err, errlen, "bad max_level"); return NULL; }
    for (int d = 0; d < 3; ++d)
        if (bn[d] < 2 || (bn[d] & 1) || base[d] < 1) { set_err(err, errlen, "bad block dims"); return NULL; }
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    if (!m) return NULL;
    m->physics = physics;
    m->riemann = riemann;
    m->limiter = LIM_MINMOD;
    m->rk = 2;
    m->nvar = physics == PHYS_MHD ? 9 : 5;
    m->gamma = gamma;
    m->cfl = cfl;
    m->glm_alpha = glm_alpha;
    m->max_level = max_level;
    m->nleaf = nleaf;
    for (int d = 0; d < 3; ++d) {
        m->bn[d] = bn[d];
        m->base[d] = base[d];
        m->lo[d] = lo[d];
        m->hi[d] = hi[d];
        m->pn[d] = bn[d] + 2 * NG;
    }
    m->dx1 = (hi[0] - lo[0]) / (double)(base[0] * bn[0]);
    for (int d = 1; d < 3; ++d) {
        double dxd = (hi[d] - lo[d]) / (double)(base[d] * bn[d]);
        if (fabs(dxd - m->dx1) > 1e-14 * m->dx1) { set_err(err, errlen, "cells must be cubic"); orc_destroy(m); return NULL; }
    }
    m->pvol = (long)m->pn[0] * m->pn[1] * m->pn[2];
    for (int l = 1; l <= max_level; ++l) {
        long tot = 1;
        for (int d = 0; d < 3; ++d) {
            m->nbl[l][d] = (long)base[d] << (l - 1);
            tot *= m->nbl[l][d];
        }
        m->lookup[l] = (int *)malloc(sizeof(int) * tot);
        if (!m->lookup[l]) { orc_destroy(m); return NULL; }
        for (long q = 0; q < tot; ++q) m->lookup[l][q] = -1;
    }
    m->lev = (int *)malloc(sizeof(int) * (nleaf > 0 ? nleaf : 1));
    m->bidx = (long *)malloc(sizeof(long) * 3 * (nleaf > 0 ? nleaf : 1));
    if (!m->lev || !m->bidx) { orc_destroy(m); return NULL; }
    for (int q = 0; q < nleaf; ++q) {
        int l = desc[4 * q];
        if (l < 1 || l > max_level) { set_err(err, errlen, "bad level"); orc_destroy(m); return NULL; }
        m->lev[q] = l;
        long b[3];
        for (int d = 0; d < 3; ++d) {
            b[d] = desc[4 * q + 1 + d];
            if (b[d] < 0 || b[d] >= m->nbl[l][d]) { set_err(err, errlen, "block index out of range"); orc_destroy(m); return NULL; }
            m->bidx[3L * q + d] = b[d];
        }
        int *slot = &m->lookup[l][(b[2] * m->nbl[l][1] + b[1]) * m->nbl[l][0] + b[0]];
        if (*slot >= 0) { set_err(err, errlen, "duplicate block"); orc_destroy(m); return NULL; }
        *slot = q;
    }
    /* tiling: no leaf may have a leaf ancestor, and the leaf volumes must add
     * up to the domain (counted in finest-level blocks) */
    unsigned long long vol = 0, dom = (unsigned long long)base[0] * base[1] * base[2];
    for (int l = 1; l < max_level; ++l) dom *= 8ULL;
    for (int q = 0; q < nleaf; ++q) {
        int l = m->lev[q];
        for (int L = l - 1; L >= 1; --L) {
            long a[3];
            for (int d = 0; d < 3; ++d) a[d] = m->bidx[3L * q + d] >> (l - L);
            if (lookup_leaf(m, L, a) >= 0) { set_err(err, errlen, "overlapping blocks"); orc_destroy(m); return NULL; }
        }
        vol += 1ULL << (3 * (max_level - l));
    }
    if (vol != dom) { set_err(err, errlen, "blocks do not tile the domain"); orc_destroy(m); return NULL; }
    m->u = (double *)malloc(sizeof(double) * (long)(nleaf > 0 ? nleaf : 1) * m->nvar * m->pvol);
    if (!m->u) { orc_destroy(m); return NULL; }
    for (long q = 0; q < (long)nleaf * m->nvar * m->pvol; ++q) m->u[q] = nanv();
    return m;
}

int orc_nvar(const orc_mesh *m) { return m->nvar; }

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* u: [nleaf][nvar][bn2][bn1][bn0] interiors in the creation order. */
int orc_set_state(orc_mesh *m, const double *u) {
    const int *bn = m->bn;
    long q = 0;
    for (int leaf = 0; leaf < m->nleaf; ++leaf)
        for (int v = 0; v < m->nvar; ++v) {
            double *dst = leaf_var(m, leaf, v);
            for (int k = 0; k < bn[2]; ++k)
                for (int j = 0; j < bn[1]; ++j)
                    for (int i = 0; i < bn[0]; ++i) dst[pidx(m, i, j, k)] = u[q++];
        }
    return ORC_OK;
}

int orc_get_state(const orc_mesh *m, double *u) {
    const int *bn = m->bn;
    long q = 0;
    for (int leaf = 0; leaf < m->nleaf; ++leaf)
        for (int v = 0; v < m->nvar; ++v) {
            const double *src = leaf_var(m, leaf, v);
            for (int k = 0; k < bn[2]; ++k)
                for (int j = 0; j < bn[1]; ++j)
                    for (int i = 0; i < bn[0]; ++i) u[q++] = src[pidx(m, i, j, k)];
        }
    return ORC_OK;
}

/* Face ghosts after orc_fill_ghosts: [leaf][face][var][cells], faces ordered
 * -x,+x,-y,+y,-z,+z, cells of each 2-deep slab in (k, j, i) order with the
 * ghost layer index increasing with the coordinate.                      */
int orc_get_ghosts(const orc_mesh *m, double *g) {
    const int *bn = m->bn;
    long q = 0;
    for (int leaf = 0; leaf < m->nleaf; ++leaf)
        for (int f = 0; f < 6; ++f) {
            int d = f / 2, side = f % 2;
            int lo3[3] = {0, 0, 0}, hi3[3] = {bn[0], bn[1], bn[2]};
            lo3[d] = side ? bn[d] : -NG;
            hi3[d] = lo3[d] + NG;
            for (int v = 0; v < m->nvar; ++v) {
                const double *src = leaf_var(m, leaf, v);
                for (int k = lo3[2]; k < hi3[2]; ++k)
                    for (int j = lo3[1]; j < hi3[1]; ++j)
                        for (int i = lo3[0]; i < hi3[0]; ++i) g[q++] = src[pidx(m, i, j, k)];
            }
        }
    return ORC_OK;
}

/* Largest cell signal rate over all leaf interiors:
 * s = (|v_x|+c_x)/dx + (|v_y|+c_y)/dx + (|v_z|+c_z)/dx, summed in that order,
 * c = sqrt(gamma p / rho) (Euler) or the fast speed along each axis (MHD).
 * Reading of "Set dt": the paper gives CFL numbers but no rule; this is the
 * unsplit 3-D bound.  Also returns the GLM speed
 * c_max = max_cells max_d (|v_d| + c_d) used by the MHD module (Sec. 2.3.3). */
int orc_max_speed(orc_mesh *m, double *smax_out, double *cmax_out) {
    const int *bn = m->bn;
    double smax = 0.0, cmax = 0.0;
    int err = ORC_OK;
#pragma omp parallel for reduction(max : smax, cmax) schedule(static)
    for (int leaf = 0; leaf < m->nleaf; ++leaf) {
        const double dx = cell_size(m, m->lev[leaf]);
        for (int k = 0; k < bn[2]; ++k)
            for (int j = 0; j < bn[1]; ++j)
                for (int i = 0; i < bn[0]; ++i) {
                    long p = pidx(m, i, j, k);
                    double U[MAXVAR], w[MAXVAR];
                    for (int v = 0; v < m->nvar; ++v) U[v] = leaf_var(m, leaf, v)[p];
                    if (cons_to_prim(m, U, w) != ORC_OK) {
#pragma omp atomic write
                        err = ORC_ENONPHYSICAL;
                        continue;
                    }
                    double s = 0.0, cm = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        double a = m->physics == PHYS_SRHD ? srhd_speed(m->gamma, w, d)
                                                           : fabs(w[1 + d]) + signal_speed(m, w, d);
                        s = (d == 0) ? a / dx : s + a / dx;
                        if (a > cm) cm = a;
                    }
                    if (s > smax) smax = s;
                    if (cm > cmax) cmax = cm;
                }
    }
    if (smax_out) *smax_out = smax;
    if (cmax_out) *cmax_out = cmax;
    return err;
}

/* dt = CFL / max s; returns a negative error code for non-physical states. */
double orc_dt(orc_mesh *m) {
    double smax = 0.0;
    int e = orc_max_speed(m, &smax, NULL);
    if (e) return (double)e;
    return m->cfl / smax;
}

/* L(U) for the current state: [leaf][var][interior] (fills ghosts first). */
int orc_rhs(orc_mesh *m, double *L) {
    if (m->physics == PHYS_MHD) {
        double cmax = 0.0;
        int e = orc_max_speed(m, NULL, &cmax);
        if (e) return e;
        m->ch = cmax;
    }
    return compute_rhs(m, L);
}

/* exact GLM source split: psi <- psi * exp(-h c_h alpha / dx_l) */
static void glm_decay(orc_mesh *m, double h) {
    const int *bn = m->bn;
#pragma omp parallel for schedule(static)
    for (int leaf = 0; leaf < m->nleaf; ++leaf) {
        const double dx = cell_size(m, m->lev[leaf]);
        const double f = exp(-h * m->ch * m->glm_alpha / dx);
        double *psi = leaf_var(m, leaf, V_PSI);
        for (int k = 0; k < bn[2]; ++k)
            for (int j = 0; j < bn[1]; ++j)
                for (int i = 0; i < bn[0]; ++i) psi[pidx(m, i, j, k)] *= f;
    }
}

/* One SSP Runge-Kutta step (Shu-Osher form):
 *   RK2: U1 = Un + dt L(Un);   U^{n+1} = 1/2 (Un + (U1 + dt L(U1)));
 *   RK3: U1 as above, U2 = 3/4 Un + 1/4 (U1 + dt L(U1)),
 *        U^{n+1} = 1/3 Un + 2/3 (U2 + dt L(U2)).
 * MHD: c_h is taken from the state at the start of the step and psi decays
 * by exp(-dt/2 c_h alpha/dx) before and after the RK step (Strang split;
 * reading of "second-order operator splitting" in Sec. 2.3.3).           */
int orc_step(orc_mesh *m, double dt) {
    const int nv = m->nvar;
    const int *bn = m->bn;
    const long ncell = (long)bn[0] * bn[1] * bn[2];
    const long tot = (long)m->nleaf * nv * ncell;
    if (m->physics == PHYS_MHD) {
        double cmax = 0.0;
        int e = orc_max_speed(m, NULL, &cmax);
        if (e) return e;
        m->ch = cmax;
        glm_decay(m, 0.5 * dt);
    }
    double *U0 = (double *)malloc(sizeof(double) * (tot > 0 ? tot : 1));
    double *L = (double *)malloc(sizeof(double) * (tot > 0 ? tot : 1));
    if (!U0 || !L) { free(U0); free(L); return ORC_ENOMEM; }
    orc_get_state(m, U0);
    int e = compute_rhs(m, L);
    if (e) { free(U0); free(L); return e; }
#pragma omp parallel for schedule(static)
    for (int leaf = 0; leaf < m->nleaf; ++leaf)
        for (int v = 0; v < nv; ++v) {
            double *u = leaf_var(m, leaf, v);
            const long off = ((long)leaf * nv + v) * ncell;
            long q = 0;
            for (int k = 0; k < bn[2]; ++k)
                for (int j = 0; j < bn[1]; ++j)
                    for (int i = 0; i < bn[0]; ++i, ++q) u[pidx(m, i, j, k)] = U0[off + q] + dt * L[off + q];
        }
    if (m->rk == 3) {
        /* SSP-RK3 (Shu-Osher): U2 = 3/4 U + 1/4 (U1 + dt L(U1)),
         * U' = 1/3 U + 2/3 (U2 + dt L(U2)) */
        e = compute_rhs(m, L);
        if (e) { free(U0); free(L); return e; }
#pragma omp parallel for schedule(static)
        for (int leaf = 0; leaf < m->nleaf; ++leaf)
            for (int v = 0; v < nv; ++v) {
                double *u = leaf_var(m, leaf, v);
                const long off = ((long)leaf * nv + v) * ncell;
                long q = 0;
                for (int k = 0; k < bn[2]; ++k)
                    for (int j = 0; j < bn[1]; ++j)
                        for (int i = 0; i < bn[0]; ++i, ++q) {
                            long p = pidx(m, i, j, k);
                            u[p] = 0.75 * U0[off + q] + 0.25 * (u[p] + dt * L[off + q]);
                        }
            }
        e = compute_rhs(m, L);
        if (e) { free(U0); free(L); return e; }
#pragma omp parallel for schedule(static)
        for (int leaf = 0; leaf < m->nleaf; ++leaf)
            for (int v = 0; v < nv; ++v) {
                double *u = leaf_var(m, leaf, v);
                const long off = ((long)leaf * nv + v) * ncell;
                long q = 0;
                for (int k = 0; k < bn[2]; ++k)
                    for (int j = 0; j < bn[1]; ++j)
                        for (int i = 0; i < bn[0]; ++i, ++q) {
                            long p = pidx(m, i, j, k);
                            u[p] = (1.0 / 3.0) * U0[off + q] + (2.0 / 3.0) * (u[p] + dt * L[off + q]);
                        }
            }
    } else {
        e = compute_rhs(m, L);
        if (e) { free(U0); free(L); return e; }
#pragma omp parallel for schedule(static)
        for (int leaf = 0; leaf < m->nleaf; ++leaf)
            for (int v = 0; v < nv; ++v) {
                double *u = leaf_var(m, leaf, v);
                const long off = ((long)leaf * nv + v) * ncell;
                long q = 0;
                for (int k = 0; k < bn[2]; ++k)
                    for (int j = 0; j < bn[1]; ++j)
                        for (int i = 0; i < bn[0]; ++i, ++q) {
                            long p = pidx(m, i, j, k);
                            u[p] = 0.5 * (U0[off + q] + (u[p] + dt * L[off + q]));
                        }
            }
    }
    free(U0);
    free(L);
    if (m->physics == PHYS_MHD) glm_decay(m, 0.5 * dt);
    return ORC_OK;
}

/* reconstruction limiter (0 minmod, 1 van Leer) and Runge-Kutta stages (2 or 3) */
int orc_set_scheme(orc_mesh *m, int limiter, int rk) {
    if ((limiter != LIM_MINMOD && limiter != LIM_VANLEER) || (rk != 2 && rk != 3)) return ORC_EINVAL;
    m->limiter = limiter;
    m->rk = rk;
    return ORC_OK;
}

/* single face flux, exposed for closed-form tests of the Riemann solvers */
int orc_face_flux(orc_mesh *m, const double *wL, const double *wR, int d, double ch, double *F) {
    m->ch = ch;
    riemann(m, wL, wR, d, F);
    return ORC_OK;
}

double orc_get_ch(const orc_mesh *m) { return m->ch; }

/* ------------------------------------------------------------------ */
/* AMR error estimation and data transfer for a regrid (the "AMR error
 * estimator" and "AMR Coarsen Refine" nodes of the flow charts, Fig. 1 and
 * Fig. 2; the estimator follows Loehner's scheme, which Sec. 4.3 names).
 *
 * Reading of the estimator (the paper names the scheme, not its formula):
 * Loehner's normalised second difference of variable v per cell, summed over
 * the three axes without cross terms (face neighbours only),
 *   E = sqrt( sum_d a_d^2 / sum_d b_d^2 ),
 *   a_d = (u_+ - u) - (u - u_-),
 *   b_d = (|u_+ - u| + |u - u_-|) + eps ((|u_+| + 2|u|) + |u_-|),
 * u_+/- the axis neighbours (face ghosts at a block side), sums in x, y, z
 * order; 0 <= E <= 1, and E = 0 where v is zero on the whole stencil
 * (both sums vanish).  The block value is the maximum over its cells.     */
int orc_lohner(orc_mesh *m, int v, double eps, double *out) {
    if (v < 0 || v >= m->nvar || !(eps > 0.0)) return ORC_EINVAL;
    orc_fill_ghosts(m);
    const int *bn = m->bn;
    const long st[3] = {1, m->pn[0], (long)m->pn[0] * m->pn[1]};
#pragma omp parallel for schedule(dynamic, 4)
    for (int leaf = 0; leaf < m->nleaf; ++leaf) {
        const double *u = leaf_var(m, leaf, v);
        double emax = 0.0;
        for (int k = 0; k < bn[2]; ++k)
            for (int j = 0; j < bn[1]; ++j)
                for (int i = 0; i < bn[0]; ++i) {
                    const long p = pidx(m, i, j, k);
                    double num = 0.0, den = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        const double up = u[p + st[d]], u0 = u[p], um = u[p - st[d]];
                        const double a = (up - u0) - (u0 - um);
                        const double b = (fabs(up - u0) + fabs(u0 - um)) + eps * ((fabs(up) + 2.0 * fabs(u0)) + fabs(um));
                        num = num + a * a;
                        den = den + b * b;
                    }
                    /* den = 0 only where v vanishes on the whole stencil: E = 0 */
                    const double e = den > 0.0 ? sqrt(num / den) : 0.0;
                    if (e > emax) emax = e;
                }
        out[leaf] = emax;
    }
    return ORC_OK;
}

/* State of a new block list sampled from this mesh: every cell of a new
 * leaf (level l, block coordinates b) takes V_l at its centre -- the stored
 * value where the leaf is unchanged, limited linear prolongation from the
 * parent where a leaf was refined, the mean of the 8 children where an octet
 * was coarsened.  blocks: [n][4] = (level, bx, by, bz); out:
 * [n][nvar][bn2][bn1][bn0].                                              */
int orc_remap(const orc_mesh *m, long n, const int *blocks, double *out) {
    const int *bn = m->bn;
    const long per = (long)bn[0] * bn[1] * bn[2];
    for (long q = 0; q < n; ++q) {
        const int l = blocks[4 * q];
        if (l < 1 || l > m->max_level) return ORC_EINVAL;
        for (int d = 0; d < 3; ++d)
            if (blocks[4 * q + 1 + d] < 0 || blocks[4 * q + 1 + d] >= m->nbl[l][d]) return ORC_EINVAL;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (long q = 0; q < n; ++q) {
        const int l = blocks[4 * q];
        for (int v = 0; v < m->nvar; ++v) {
            double *o = out + (q * m->nvar + v) * per;
            long idx = 0;
            for (int k = 0; k < bn[2]; ++k)
                for (int j = 0; j < bn[1]; ++j)
                    for (int i = 0; i < bn[0]; ++i) {
                        const long c[3] = {(long)blocks[4 * q + 1] * bn[0] + i, (long)blocks[4 * q + 2] * bn[1] + j,
                                           (long)blocks[4 * q + 3] * bn[2] + k};
                        o[idx++] = V(m, l, c, v);
                    }
        }
    }
    return ORC_OK;
}

/* primitives of n conserved states ([n][nvar] each) with the mesh's physics;
 * returns the first error (non-physical state) or ORC_OK                 */
/* Newton steps the SRHD con2prim takes for each of n conserved states (0
   for a state it rejects before iterating) */
int orc_srhd_newton_steps(const orc_mesh *m, long n, const double *U, int *steps) {
    if (m->physics != PHYS_SRHD) return ORC_EINVAL;
    double w[5];
    for (long q = 0; q < n; ++q) {
        steps[q] = 0;
        srhd_con2prim(m->gamma, U + q * 5, w, steps + q);
    }
    return ORC_OK;
}

int orc_cons_to_prim(const orc_mesh *m, long n, const double *U, double *w) {
    int rc = ORC_OK;
    for (long q = 0; q < n; ++q) {
        const int r = cons_to_prim(m, U + q * m->nvar, w + q * m->nvar);
        if (r != ORC_OK && rc == ORC_OK) rc = r;
    }
    return rc;
}
