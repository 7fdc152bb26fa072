/*
 * CPU FP64 oracle of the per-leaf hydro step (arXiv 2107.10987, section IV-B).
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use this file.  It is a plain, slow, scalar rendering of the
 * method, written for a reader to check against the paper by eye; it shares no
 * code, header, table or constant generator with the GPU library.  Build with
 * contraction off (-ffp-contract=off) so every operation rounds as written.
 *
 * Method (section IV-B): finite volumes on 8^3 leaves; the seven evolved
 * fields are reconstructed at 26 points of each cell (6 face centres, 12 edge
 * centres, 8 corners) by PPM (Colella & Woodward 1984) applied along the 13
 * lines through the cell centre that pass through those points, giving a value
 * at each end; the central-upwind flux of Kurganov & Tadmor turns the left and
 * right values at each face point into a point flux; a Newton-Cotes rule over
 * the 3x3 points of a face gives the face flux.  The evolved set is mass,
 * momenta and gas energy in a frame rotating about z (section I), plus the
 * entropy tracer of Bryan et al.'s dual-energy formalism and one passive
 * species.  Time integration is two-stage SSP Runge-Kutta (the paper's
 * production runs use three stages, section V-A2).
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *  - PPM: CW84 interface formula with monotonised-central slopes and the CW84
 *    monotonicity constraint; no contact steepening, no flattening; applied to
 *    each conserved field along each line in the line's own index.
 *  - Face points pair the two cells sharing the face, each reconstructed
 *    towards the same point.
 *  - Point flux: F = (F(UL)+F(UR))/2 - a (UR-UL)/2, a = max over both sides
 *    of |u_n| + c, with u the velocity relative to the rotating grid.
 *  - Rotating frame: inertial momenta in rotating coordinates, source -Omega x s,
 *    energy flux E u_n + p v_n, rotation axis z through x = y = 0.
 *  - Dual energy: e = E - |s|^2/(2 rho); where e < eta1 E the tracer gives
 *    e = tau^gamma; after each full step tau = e^(1/gamma) where e > eta2 E.
 *  - Ghosts: periodic wrap or zero-gradient outflow at the leaf's own level,
 *    injection from a coarser leaf, mean of the 2^3 children of a finer one.
 */
#include "hydro_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { NX = 8, GW = 3, PB = 14, NFLD = 7, NCELL = 512, NPAD = 2744 };
enum { RB = 10 };            /* cells -1..8 per axis carry reconstructed values */
#define MAXLEV 24

static long pidx(int i, int j, int k) { return ((long)(k + GW) * PB + (j + GW)) * PB + (i + GW); }
static int dir27(int dx, int dy, int dz) { return 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1); }
static int dir26(int dx, int dy, int dz) { int k = dir27(dx, dy, dz); return k < 13 ? k : k - 1; }
static long ridx(int i, int j, int k) { return ((long)(k + 1) * RB + (j + 1)) * RB + (i + 1); }

/* One direction of each of the 13 lines through a cell centre and the 26
 * points: face normals, face diagonals and body diagonals. */
static const int LINE[13][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1},
    {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

/* 2D Newton-Cotes (Simpson) weights (1,4,1)/6 x (1,4,1)/6 over a face. */
static const double SIMPSON[3][3] = {
    {1.0 / 36.0, 4.0 / 36.0, 1.0 / 36.0},
    {4.0 / 36.0, 16.0 / 36.0, 4.0 / 36.0},
    {1.0 / 36.0, 4.0 / 36.0, 1.0 / 36.0}};

/* ------------------------------------------------------------------------ */
/* PPM along one line (CW84 eqs. 1.6-1.10, section IV-B)                   */
/* ------------------------------------------------------------------------ */

/* Monotonised-central slope of the middle of three values: the centred
 * difference, bounded by twice each one-sided difference, zero at an extremum. */
static double limited_slope(double qm, double q0, double qp)
{
    double dl = q0 - qm;
    double dr = qp - q0;
    double d = 0.5 * (qp - qm);
    if (dl * dr > 0.0) {
        double m = fabs(d);
        double a = 2.0 * fabs(dl);
        double b = 2.0 * fabs(dr);
        if (a < m) m = a;
        if (b < m) m = b;
        return copysign(m, d);
    }
    return 0.0;
}

void oracle_ppm(const double q[5], double *left, double *right)
{
    const double sixth = 1.0 / 6.0;
    double sm = limited_slope(q[0], q[1], q[2]);
    double s0 = limited_slope(q[1], q[2], q[3]);
    double sp = limited_slope(q[2], q[3], q[4]);
    /* interface values of the parabola through the cell averages */
    double R = q[2] + 0.5 * (q[3] - q[2]) - (sp - s0) * sixth;
    double L = q[1] + 0.5 * (q[2] - q[1]) - (s0 - sm) * sixth;
    /* monotonicity: flat at a local extremum, otherwise pull the far edge in
     * so the parabola has no interior extremum */
    if ((R - q[2]) * (q[2] - L) <= 0.0) {
        L = q[2];
        R = q[2];
    } else {
        double D = R - L;
        double M6 = 6.0 * (q[2] - 0.5 * (L + R));
        if (D * M6 > D * D)
            L = 3.0 * q[2] - 2.0 * R;
        else if (D * M6 < -(D * D))
            R = 3.0 * q[2] - 2.0 * L;
    }
    *left = L;
    *right = R;
}

/* ------------------------------------------------------------------------ */
/* Point flux: central-upwind (Kurganov-Tadmor) with dual-energy pressure  */
/* ------------------------------------------------------------------------ */

static double side_flux(int n, const double U[7], const double xq[3], const oracle_phys *ph,
                        double F[7])
{
    double rho = U[0], E = U[4], tau = U[5];
    double rinv = 1.0 / rho;
    double v[3], u[3];
    v[0] = U[1] * rinv;
    v[1] = U[2] * rinv;
    v[2] = U[3] * rinv;
    /* velocity relative to the grid rotating at omega about z: u = v - omega x x */
    u[0] = v[0] + ph->omega * xq[1];
    u[1] = v[1] - ph->omega * xq[0];
    u[2] = v[2];
    double ek = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * rinv;
    double eint = E - ek;
    if (eint < ph->eta1 * E) eint = pow(tau, ph->gamma);
    double p = (ph->gamma - 1.0) * eint;
    double cs = sqrt(ph->gamma * p * rinv);
    double un = u[n];
    F[0] = rho * un;
    F[1] = U[1] * un;
    F[2] = U[2] * un;
    F[3] = U[3] * un;
    F[1 + n] = F[1 + n] + p;
    F[4] = E * un + p * v[n];
    F[5] = tau * un;
    F[6] = U[6] * un;
    return fabs(un) + cs;
}

double oracle_point_flux(int n, const double UL[7], const double UR[7], const double xq[3],
                         const oracle_phys *ph, double F[7])
{
    double FL[7], FR[7];
    double sl = side_flux(n, UL, xq, ph, FL);
    double sr = side_flux(n, UR, xq, ph, FR);
    /* a side without a real sound speed (rho <= 0, or a negative or non-finite
     * pressure) has no signal speed: the maximum is then undefined and the
     * point flux is NaN, so the stage reports a non-physical result */
    double a = (isnan(sl) || isnan(sr)) ? (double)NAN : (sl > sr ? sl : sr);
    for (int f = 0; f < NFLD; ++f)
        F[f] = 0.5 * (FL[f] + FR[f]) - 0.5 * a * (UR[f] - UL[f]);
    return a;
}

/* ------------------------------------------------------------------------ */
/* Ghost layers from the octree                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nb[3], bc[3], n, lmax;
    int prolong; /* 1: linear-limited prolongation of ghosts from coarser leaves */
    const int *level, *coord;
    long dim[MAXLEV][3];
    int *slot[MAXLEV]; /* leaf index of each level-l slot, -1 if none */
} tree_t;

void *oracle_tree_create(const int nb[3], const int bc[3], int n, const int *level,
                         const int *coord)
{
    tree_t *t = (tree_t *)calloc(1, sizeof(tree_t));
    if (!t) return NULL;
    memcpy(t->nb, nb, sizeof(t->nb));
    memcpy(t->bc, bc, sizeof(t->bc));
    t->n = n;
    t->level = level;
    t->coord = coord;
    t->lmax = 0;
    for (int i = 0; i < n; ++i)
        if (level[i] > t->lmax) t->lmax = level[i];
    if (t->lmax >= MAXLEV) { free(t); return NULL; }
    for (int l = 0; l <= t->lmax; ++l) {
        long cnt = 1;
        for (int a = 0; a < 3; ++a) {
            t->dim[l][a] = (long)nb[a] << l;
            cnt *= t->dim[l][a];
        }
        t->slot[l] = (int *)malloc(sizeof(int) * cnt);
        for (long s = 0; s < cnt; ++s) t->slot[l][s] = -1;
    }
    for (int i = 0; i < n; ++i) {
        int l = level[i];
        const int *c = coord + 3 * i;
        long s = ((long)c[2] * t->dim[l][1] + c[1]) * t->dim[l][0] + c[0];
        t->slot[l][s] = i;
    }
    return t;
}

void oracle_tree_destroy(void *tp)
{
    tree_t *t = (tree_t *)tp;
    if (!t) return;
    for (int l = 0; l <= t->lmax; ++l) free(t->slot[l]);
    free(t);
}

/* Value of the level-l cell g (global cell coordinates at level l, inside the
 * box): the cell of the leaf covering it when that leaf is at level <= l
 * (injection from a coarser leaf), else the mean of its 2^3 children. */
static int cell_value(const tree_t *t, const double *U, int l, const long g[3], double out[7])
{
    for (int lc = (l < t->lmax ? l : t->lmax); lc >= 0; --lc) {
        long c[3], s[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = g[a] >> (l - lc);
            s[a] = c[a] / NX;
        }
        int leaf = t->slot[lc][(s[2] * t->dim[lc][1] + s[1]) * t->dim[lc][0] + s[0]];
        if (leaf >= 0) {
            long cell = ((c[2] - NX * s[2]) * NX + (c[1] - NX * s[1])) * NX + (c[0] - NX * s[0]);
            for (int f = 0; f < NFLD; ++f) out[f] = U[((long)leaf * NFLD + f) * NCELL + cell];
            return 0;
        }
    }
    if (l + 1 > t->lmax) return -1;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0}, tmp[7];
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                long h[3] = {2 * g[0] + ox, 2 * g[1] + oy, 2 * g[2] + oz};
                if (cell_value(t, U, l + 1, h, tmp)) return -1;
                for (int f = 0; f < NFLD; ++f) acc[f] = acc[f] + tmp[f];
            }
    for (int f = 0; f < NFLD; ++f) out[f] = acc[f] * 0.125;
    return 0;
}

void oracle_tree_set_prolong(void *tp, int on)
{
    ((tree_t *)tp)->prolong = on;
}

/* Level of the leaf covering level-l cell g when that leaf is at level <= l,
 * else -1 (the cell is refined). */
static int covering_level(const tree_t *t, int l, const long g[3])
{
    for (int lc = (l < t->lmax ? l : t->lmax); lc >= 0; --lc) {
        long s[3];
        for (int a = 0; a < 3; ++a) s[a] = (g[a] >> (l - lc)) / NX;
        if (t->slot[lc][(s[2] * t->dim[lc][1] + s[1]) * t->dim[lc][0] + s[0]] >= 0) return lc;
    }
    return -1;
}

static double minmod(double a, double b)
{
    if (!(a * b > 0.0)) return 0.0;
    return fabs(a) <= fabs(b) ? a : b;
}

/* Ghost value of level-l cell g.  Without prolongation (and wherever the cell
 * is not covered by a coarser leaf) it is cell_value's.  With it, a cell inside
 * the cell C of a coarser leaf takes the linear reconstruction of C at its
 * centre: U_C + sum over axes of (offset of the centre from C's, in units of
 * C's size) x minmod(U_{C+e} - U_C, U_C - U_{C-e}), the neighbours taken at C's
 * level by the same rules (wrap or clamp, injection, mean of finer cells), and
 * the three terms added in x, y, z order.  The paper's AMR (section IV-B)
 * leaves the coarse-to-fine ghost interpolation unspecified; this is the
 * usual conservative, monotonicity-preserving choice. */
static int ghost_value(const tree_t *t, const double *U, int l, const long g[3], double out[7])
{
    if (!t->prolong) return cell_value(t, U, l, g, out);
    const int lc = covering_level(t, l, g);
    if (lc < 0 || lc == l) return cell_value(t, U, l, g, out);
    const int d = l - lc;
    long C[3];
    double frac[3];
    for (int a = 0; a < 3; ++a) {
        C[a] = g[a] >> d;
        frac[a] = ((double)(g[a] - (C[a] << d)) + 0.5) / (double)(1L << d) - 0.5;
    }
    double uc[7];
    if (cell_value(t, U, lc, C, uc)) return -1;
    for (int f = 0; f < NFLD; ++f) out[f] = uc[f];
    for (int a = 0; a < 3; ++a) {
        double um[7], up[7];
        long cm[3] = {C[0], C[1], C[2]}, cp[3] = {C[0], C[1], C[2]};
        const long ncell = (long)NX * t->dim[lc][a];
        cm[a] = C[a] - 1;
        cp[a] = C[a] + 1;
        if (t->bc[a] == 0) {
            cm[a] = (cm[a] + ncell) % ncell;
            cp[a] = cp[a] % ncell;
        } else {
            if (cm[a] < 0) cm[a] = 0;
            if (cp[a] >= ncell) cp[a] = ncell - 1;
        }
        if (cell_value(t, U, lc, cm, um) || cell_value(t, U, lc, cp, up)) return -1;
        for (int f = 0; f < NFLD; ++f) out[f] = out[f] + frac[a] * minmod(up[f] - uc[f], uc[f] - um[f]);
    }
    return 0;
}

int oracle_fill_padded(const void *tp, const double *U, int l0, int l1, double *P)
{
    const tree_t *t = (const tree_t *)tp;
    for (int leaf = l0; leaf < l1; ++leaf) {
        double *B = P + (long)(leaf - l0) * NFLD * NPAD;
        int l = t->level[leaf];
        const int *co = t->coord + 3 * leaf;
        for (int k = -GW; k < NX + GW; ++k)
            for (int j = -GW; j < NX + GW; ++j)
                for (int i = -GW; i < NX + GW; ++i) {
                    double v[7];
                    int loc[3] = {i, j, k};
                    int inside = (i >= 0 && i < NX && j >= 0 && j < NX && k >= 0 && k < NX);
                    if (inside) {
                        long cell = ((long)k * NX + j) * NX + i;
                        for (int f = 0; f < NFLD; ++f)
                            v[f] = U[((long)leaf * NFLD + f) * NCELL + cell];
                    } else {
                        long g[3];
                        for (int a = 0; a < 3; ++a) {
                            long ncell = (long)NX * t->dim[l][a];
                            g[a] = (long)NX * co[a] + loc[a];
                            if (g[a] < 0 || g[a] >= ncell) {
                                if (t->bc[a] == 0)
                                    g[a] = ((g[a] % ncell) + ncell) % ncell;
                                else
                                    g[a] = g[a] < 0 ? 0 : ncell - 1;
                            }
                        }
                        if (ghost_value(t, U, l, g, v)) return -1;
                    }
                    for (int f = 0; f < NFLD; ++f) B[(long)f * NPAD + pidx(i, j, k)] = v[f];
                }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction, fluxes and L(U) of one leaf                              */
/* ------------------------------------------------------------------------ */

/* V[ridx(cell)][dir26][f] for cells -1..8 per axis (interior plus the ghost
 * cells that share a face with the leaf, and some unused ones). */
static void reconstruct_block(const double *P, double *V)
{
    for (int k = -1; k <= NX; ++k)
        for (int j = -1; j <= NX; ++j)
            for (int i = -1; i <= NX; ++i)
                for (int ln = 0; ln < 13; ++ln) {
                    const int *d = LINE[ln];
                    int kp = dir26(d[0], d[1], d[2]);
                    int km = dir26(-d[0], -d[1], -d[2]);
                    for (int f = 0; f < NFLD; ++f) {
                        double q[5], L, R;
                        for (int m = -2; m <= 2; ++m)
                            q[m + 2] = P[(long)f * NPAD + pidx(i + m * d[0], j + m * d[1], k + m * d[2])];
                        oracle_ppm(q, &L, &R);
                        V[(ridx(i, j, k) * 26 + kp) * NFLD + f] = R;
                        V[(ridx(i, j, k) * 26 + km) * NFLD + f] = L;
                    }
                }
}

void oracle_reconstruct_values(const double *P, double *V) { reconstruct_block(P, V); }

void oracle_leaf_reconstruct(const double *P, double *out)
{
    double *V = (double *)malloc(sizeof(double) * RB * RB * RB * 26 * NFLD);
    reconstruct_block(P, V);
    for (int f = 0; f < NFLD; ++f)
        for (int k = 0; k < NX; ++k)
            for (int j = 0; j < NX; ++j)
                for (int i = 0; i < NX; ++i)
                    for (int d = 0; d < 26; ++d)
                        out[(((long)f * NCELL) + (k * NX + j) * NX + i) * 26 + d] =
                            V[(ridx(i, j, k) * 26 + d) * NFLD + f];
    free(V);
}

/* Face fluxes of one leaf, Fn[n][face 0..8 along n][t1][t2][f] with (t1, t2)
 * the other two axes in increasing order; returns the max signal speed. */
double oracle_leaf_fluxes(const double *P, double dx, const double origin[3], const oracle_phys *ph,
                          double *Fn)
{
    double *V = (double *)malloc(sizeof(double) * RB * RB * RB * 26 * NFLD);
    reconstruct_block(P, V);
    double smax = oracle_leaf_fluxes_from_values(V, dx, origin, ph, Fn);
    free(V);
    return smax;
}

double oracle_leaf_fluxes_from_values(const double *V, double dx, const double origin[3],
                                      const oracle_phys *ph, double *Fn)
{
    double smax = 0.0;
    for (int n = 0; n < 3; ++n) {
        int t1 = (n == 0) ? 1 : 0;
        int t2 = (n == 2) ? 1 : 2;
        for (int fi = 0; fi <= NX; ++fi)
            for (int c1 = 0; c1 < NX; ++c1)
                for (int c2 = 0; c2 < NX; ++c2) {
                    int B[3], A[3];
                    B[n] = fi;
                    B[t1] = c1;
                    B[t2] = c2;
                    for (int a = 0; a < 3; ++a) A[a] = B[a];
                    A[n] = fi - 1;
                    double xB[3];
                    for (int a = 0; a < 3; ++a) xB[a] = origin[a] + (double)B[a] * dx;
                    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
                    /* the old scheme (section IV-B, last sentence) evaluates the
                     * flux at the face centre only, with weight one */
                    const int span = ph->centre_only ? 0 : 1;
                    for (int a = -span; a <= span; ++a)
                        for (int b = -span; b <= span; ++b) {
                            int dB[3], dA[3];
                            dB[n] = -1;
                            dB[t1] = a;
                            dB[t2] = b;
                            dA[n] = 1;
                            dA[t1] = a;
                            dA[t2] = b;
                            const double *UL = V + (ridx(A[0], A[1], A[2]) * 26 + dir26(dA[0], dA[1], dA[2])) * NFLD;
                            const double *UR = V + (ridx(B[0], B[1], B[2]) * 26 + dir26(dB[0], dB[1], dB[2])) * NFLD;
                            double xq[3], F[7];
                            for (int c = 0; c < 3; ++c) xq[c] = xB[c] + 0.5 * (double)dB[c] * dx;
                            double s = oracle_point_flux(n, UL, UR, xq, ph, F);
                            if (s > smax) smax = s;
                            const double w = ph->centre_only ? 1.0 : SIMPSON[a + 1][b + 1];
                            for (int f = 0; f < NFLD; ++f) acc[f] = acc[f] + w * F[f];
                        }
                    double *dst = Fn + ((((long)n * 9 + fi) * NX + c1) * NX + c2) * NFLD;
                    for (int f = 0; f < NFLD; ++f) dst[f] = acc[f];
                }
    }
    return smax;
}

void oracle_leaf_rhs(const double *P, double dx, const double origin[3], const oracle_phys *ph,
                     double *dU, double *amax)
{
    double *V = (double *)malloc(sizeof(double) * RB * RB * RB * 26 * NFLD);
    reconstruct_block(P, V);
    oracle_leaf_rhs_from_values(V, P, dx, origin, ph, dU, amax);
    free(V);
}

/* L(U) from the face fluxes Fn: flux divergence plus the rotating-frame
 * source (Omega sy, -Omega sx) of the cell values in P. */
static void rhs_from_fluxes(const double *Fn, const double *P, double dx, const oracle_phys *ph, double *dU)
{
    double idx = 1.0 / dx;
#define FX(i, j, k, f) Fn[((((long)0 * 9 + (i)) * NX + (j)) * NX + (k)) * NFLD + (f)]
#define FY(i, j, k, f) Fn[((((long)1 * 9 + (j)) * NX + (i)) * NX + (k)) * NFLD + (f)]
#define FZ(i, j, k, f) Fn[((((long)2 * 9 + (k)) * NX + (i)) * NX + (j)) * NFLD + (f)]
    for (int k = 0; k < NX; ++k)
        for (int j = 0; j < NX; ++j)
            for (int i = 0; i < NX; ++i) {
                long c = ((long)k * NX + j) * NX + i;
                for (int f = 0; f < NFLD; ++f) {
                    double d = (FX(i + 1, j, k, f) - FX(i, j, k, f)) + (FY(i, j + 1, k, f) - FY(i, j, k, f)) +
                               (FZ(i, j, k + 1, f) - FZ(i, j, k, f));
                    dU[(long)f * NCELL + c] = -d * idx;
                }
                double sx = P[1L * NPAD + pidx(i, j, k)];
                double sy = P[2L * NPAD + pidx(i, j, k)];
                dU[1L * NCELL + c] = dU[1L * NCELL + c] + ph->omega * sy;
                dU[2L * NCELL + c] = dU[2L * NCELL + c] - ph->omega * sx;
            }
#undef FX
#undef FY
#undef FZ
}

void oracle_leaf_rhs_from_values(const double *V, const double *P, double dx, const double origin[3],
                                 const oracle_phys *ph, double *dU, double *amax)
{
    double *Fn = (double *)malloc(sizeof(double) * 3 * 9 * NX * NX * NFLD);
    *amax = oracle_leaf_fluxes_from_values(V, dx, origin, ph, Fn);
    rhs_from_fluxes(Fn, P, dx, ph, dU);
    free(Fn);
}

/* ------------------------------------------------------------------------ */
/* Stages of the two-stage SSP Runge-Kutta step                             */
/* ------------------------------------------------------------------------ */

/* Dual-energy tracer resync of one cell after a full step. */
static void resync(double *u[7], const oracle_phys *ph)
{
    double rho = *u[0], E = *u[4];
    double rinv = 1.0 / rho;
    double ek = 0.5 * ((*u[1]) * (*u[1]) + (*u[2]) * (*u[2]) + (*u[3]) * (*u[3])) * rinv;
    double eint = E - ek;
    if (eint > ph->eta2 * E) *u[5] = pow(eint, 1.0 / ph->gamma);
}

/* Shu-Osher coefficients of stage s (1-based) of the SSP Runge-Kutta
 * integrator of the given order: Uout = a Un + b (Uin + dt L(Uin)). */
static int ssp_coeffs(int order, int stage, double *a, double *b)
{
    if (order == 2 && stage == 2) { *a = 0.5; *b = 0.5; return 0; }
    if (order == 3 && stage == 2) { *a = 0.75; *b = 0.25; return 0; }
    if (order == 3 && stage == 3) { *a = 1.0 / 3.0; *b = 2.0 / 3.0; return 0; }
    if (stage == 1 && (order == 2 || order == 3)) { *a = 0.0; *b = 1.0; return 0; }
    return -2;
}

/* The leaves one level finer across face (n, s) of `leaf`, s = -1 or +1.
 * Returns 1 with ch[o1 + 2 o2] = the child whose offsets along the two other
 * axes (in increasing axis order) are o1, o2, when the region next to the
 * face, at the leaf's level, is split into leaves of the next level; 0 when
 * a leaf of the same or a coarser level covers it, or beyond an outflow
 * boundary; -1 when those children are not leaves (tree not 2:1 balanced). */
static int finer_across(const tree_t *t, int leaf, int n, int s, int ch[4])
{
    const int l = t->level[leaf];
    long q[3];
    for (int a = 0; a < 3; ++a) q[a] = t->coord[3 * leaf + a];
    q[n] += s;
    if (q[n] < 0 || q[n] >= t->dim[l][n]) {
        if (t->bc[n] != 0) return 0;
        q[n] = (q[n] + t->dim[l][n]) % t->dim[l][n];
    }
    for (int lc = l; lc >= 0; --lc) {
        long r[3];
        for (int a = 0; a < 3; ++a) r[a] = q[a] >> (l - lc);
        if (t->slot[lc][(r[2] * t->dim[lc][1] + r[1]) * t->dim[lc][0] + r[0]] >= 0) return 0;
    }
    if (l + 1 > t->lmax) return -1;
    const int t1 = (n == 0) ? 1 : 0, t2 = (n == 2) ? 1 : 2;
    for (int o2 = 0; o2 < 2; ++o2)
        for (int o1 = 0; o1 < 2; ++o1) {
            long r[3];
            r[n] = 2 * q[n] + (s > 0 ? 0 : 1);
            r[t1] = 2 * q[t1] + o1;
            r[t2] = 2 * q[t2] + o2;
            const int c = t->slot[l + 1][(r[2] * t->dim[l + 1][1] + r[1]) * t->dim[l + 1][0] + r[0]];
            if (c < 0) return -1;
            ch[o1 + 2 * o2] = c;
        }
    return 1;
}

static int plain_values(const double *P, void *ctx, double *V)
{
    (void)ctx;
    reconstruct_block(P, V);
    return 0;
}

/* Face fluxes Fn of one leaf for the state U: ghost fill, point values from
 * `values` (which returns its count of fallback cells), fluxes. */
static int fluxes_of_leaf(const tree_t *t, const double *U, int leaf, const double *dx,
                          const double *origin, const oracle_phys *ph, oracle_values_fn values,
                          void *ctx, double *P, double *V, double *Fn, double *smax, int *nfb)
{
    if (oracle_fill_padded(t, U, leaf, leaf + 1, P)) return -1;
    const int nf = values(P, ctx, V);
    if (nfb) *nfb = nf;
    *smax = oracle_leaf_fluxes_from_values(V, dx[leaf], origin + 3L * leaf, ph, Fn);
    return 0;
}

/* Flux correction at coarse/fine faces.  The paper runs the scheme on an
 * AMR octree (section IV-B) without saying how fluxes are matched where a
 * leaf meets finer ones; the reading here is the usual conservative one: the
 * coarse face flux through a face shared with four finer cells is the mean
 * of those cells' own face fluxes (each a flux density over a quarter of the
 * coarse face), so what leaves the fine cells enters the coarse cell. */
static int reflux_fluxes(const tree_t *t, const double *U, int leaf, const double *dx,
                         const double *origin, const oracle_phys *ph, oracle_values_fn values, void *ctx,
                         double *P, double *V, double *Fc, double *Fn)
{
    for (int n = 0; n < 3; ++n)
        for (int side = 0; side < 2; ++side) {
            int ch[4];
            const int r = finer_across(t, leaf, n, side ? 1 : -1, ch);
            if (r < 0) return -1;
            if (r == 0) continue;
            const int fi = side ? NX : 0;   /* this leaf's face on the shared plane */
            const int fc = side ? 0 : NX;   /* the children's face on it */
            for (int o2 = 0; o2 < 2; ++o2)
                for (int o1 = 0; o1 < 2; ++o1) {
                    double sm;
                    if (fluxes_of_leaf(t, U, ch[o1 + 2 * o2], dx, origin, ph, values, ctx, P, V, Fc, &sm, NULL))
                        return -1;
                    for (int c1 = 4 * o1; c1 < 4 * o1 + 4; ++c1)
                        for (int c2 = 4 * o2; c2 < 4 * o2 + 4; ++c2) {
                            const int a = 2 * (c1 - 4 * o1), b = 2 * (c2 - 4 * o2);
                            for (int f = 0; f < NFLD; ++f) {
#define FC(u, v) Fc[((((long)n * 9 + fc) * NX + (a + (u))) * NX + (b + (v))) * NFLD + f]
                                const double m = ((FC(0, 0) + FC(1, 0)) + (FC(0, 1) + FC(1, 1))) * 0.25;
#undef FC
                                Fn[((((long)n * 9 + fi) * NX + c1) * NX + c2) * NFLD + f] = m;
                            }
                        }
                }
        }
    return 0;
}

int oracle_stage(const void *t, int stage, double dt, const double *Uin, const double *Un,
                 const double *dx, const double *origin, const oracle_phys *ph, int l0, int l1,
                 double *Uout, double *amax)
{
    return oracle_stage_rk(t, 2, stage, dt, Uin, Un, dx, origin, ph, l0, l1, Uout, amax);
}

int oracle_stage_rk(const void *t, int order, int stage, double dt, const double *Uin, const double *Un,
                    const double *dx, const double *origin, const oracle_phys *ph, int l0, int l1,
                    double *Uout, double *amax)
{
    return oracle_stage_with(t, order, stage, dt, Uin, Un, dx, origin, ph, l0, l1, Uout, amax,
                             plain_values, NULL, NULL);
}

int oracle_stage_with(const void *tp, int order, int stage, double dt, const double *Uin,
                      const double *Un, const double *dx, const double *origin, const oracle_phys *ph,
                      int l0, int l1, double *Uout, double *amax, oracle_values_fn values, void *ctx,
                      int *fallback)
{
    const tree_t *t = (const tree_t *)tp;
    double ca, cb;
    if (ssp_coeffs(order, stage, &ca, &cb)) return -2;
    const long nfx = 3L * 9 * NX * NX * NFLD;
    double *P = (double *)malloc(sizeof(double) * NFLD * NPAD);
    double *P2 = (double *)malloc(sizeof(double) * NFLD * NPAD);
    double *V = (double *)malloc(sizeof(double) * RB * RB * RB * 26 * NFLD);
    double *Fn = (double *)malloc(sizeof(double) * nfx);
    double *Fc = (double *)malloc(sizeof(double) * nfx);
    double *dU = (double *)malloc(sizeof(double) * NFLD * NCELL);
    int rc = 0;
    for (int leaf = l0; leaf < l1 && rc == 0; ++leaf) {
        rc = fluxes_of_leaf(t, Uin, leaf, dx, origin, ph, values, ctx, P, V, Fn, &amax[leaf],
                            fallback ? &fallback[leaf] : NULL);
        if (rc) break;
        if (ph->reflux && (rc = reflux_fluxes(t, Uin, leaf, dx, origin, ph, values, ctx, P2, V, Fc, Fn)))
            break;
        rhs_from_fluxes(Fn, P, dx[leaf], ph, dU);
        const long base = (long)leaf * NFLD * NCELL;
        for (long e = 0; e < NFLD * NCELL; ++e) {
            double u = Uin[base + e];
            if (stage == 1)
                Uout[base + e] = u + dt * dU[e];
            else
                Uout[base + e] = ca * Un[base + e] + cb * (u + dt * dU[e]);
        }
        if (stage == order)
            for (long c = 0; c < NCELL; ++c) {
                double *u[7];
                for (int f = 0; f < NFLD; ++f) u[f] = Uout + base + (long)f * NCELL + c;
                resync(u, ph);
            }
    }
    free(dU);
    free(Fc);
    free(Fn);
    free(V);
    free(P2);
    free(P);
    return rc;
}

int oracle_signal_speed(const void *t, const double *U, const double *dx, const double *origin,
                        const oracle_phys *ph, int l0, int l1, double *amax)
{
    double *P = (double *)malloc(sizeof(double) * NFLD * NPAD);
    double *dU = (double *)malloc(sizeof(double) * NFLD * NCELL);
    int rc = 0;
    for (int leaf = l0; leaf < l1; ++leaf) {
        rc = oracle_fill_padded(t, U, leaf, leaf + 1, P);
        if (rc) break;
        oracle_leaf_rhs(P, dx[leaf], origin + 3L * leaf, ph, dU, &amax[leaf]);
    }
    free(dU);
    free(P);
    return rc;
}

int oracle_reconstruct(const void *t, const double *U, int l0, int l1, double *out)
{
    double *P = (double *)malloc(sizeof(double) * NFLD * NPAD);
    int rc = 0;
    for (int leaf = l0; leaf < l1; ++leaf) {
        rc = oracle_fill_padded(t, U, leaf, leaf + 1, P);
        if (rc) break;
        oracle_leaf_reconstruct(P, out + (long)(leaf - l0) * NFLD * NCELL * 26);
    }
    free(P);
    return rc;
}
