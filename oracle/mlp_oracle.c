/*
 * CPU oracle of the learned reconstruction: TEST INFRASTRUCTURE.
 *
 * A small network replaces PPM where it is safe to.  For each cell and field
 * the 3x3x3 neighbourhood is normalised, x_k = (q_{c+o_k} - q_c) / sigma with
 * sigma = max |q_nb - q_c|, and joined to a one-hot field id (34 inputs); two
 * hidden layers of 64 with tanh-GELU give 26 outputs y_d, and the point value
 * is q_c + sigma * y_d in FP64.  A flat neighbourhood (sigma = 0) passes q_c
 * through exactly.  The plain limiter then acts on the predicted values
 * (clamp between the cell and each neighbour, PPM monotonicity constraint per
 * line; the results are kept as q_c plus a binary32 offset), and every row
 * is checked in FP64 on those values: each value must lie
 * between the cell and its neighbour in that direction, each line's pair of
 * end values must satisfy the PPM monotonicity conditions, and rho, E, tau
 * must stay positive and X non-negative; a cell any of whose fields fails is
 * reconstructed by plain PPM instead, so the fluxes, the update and the
 * conservation stay those of the FP64 scheme.
 *
 * The network runs here in FP64.  With `emulate` set, inputs, weights,
 * activations and back-propagated operands are rounded to bfloat16 and
 * pre-activations to binary32 exactly where the GPU kernels round them, so
 * the two can be compared closely; with `emulate` clear everything stays
 * FP64 (the finite-difference gradient check uses that mode).
 *
 * Parameter vector (float32 masters, 8090 values): W1[64][34], b1[64],
 * W2[64][64], b2[64], W3[26][64], b3[26].
 */
#include "hydro_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { IN = 34, HID = 64, OUT = 26, NPAR = 8090 };
enum { OW1 = 0, OB1 = 2176, OW2 = 2240, OB2 = 6336, OW3 = 6400, OB3 = 8064 };
enum { NXC = 8, GWC = 3, PBC = 14, NFC = 7, NPADC = 2744, RBC = 10 };

static const double GELU_C = 0.7978845608028654;   /* sqrt(2/pi) */
static const double GELU_A = 0.044715;

/* binary64 -> binary32 -> bfloat16, round to nearest even at each step */
double oracle_bf16(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) {
        u += 0x7fffu + ((u >> 16) & 1u);
        u &= 0xffff0000u;
    }
    memcpy(&f, &u, 4);
    return (double)f;
}

static double f32(double v) { return (double)(float)v; }

static double gelu(double z) { return 0.5 * z * (1.0 + tanh(GELU_C * (z + GELU_A * z * z * z))); }

static double gelu_grad(double z)
{
    double t = tanh(GELU_C * (z + GELU_A * z * z * z));
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z);
}

/* Forward pass of B rows; caches (may be NULL) receive the pre-activations
 * and activations of both hidden layers for the backward pass. */
void oracle_mlp_forward(const float *par, int emulate, const double *x, int B, double *y, double *z1c,
                        double *a1c, double *z2c, double *a2c)
{
    double W1[HID * IN], W2[HID * HID], W3[OUT * HID];
    for (int i = 0; i < HID * IN; ++i) W1[i] = emulate ? oracle_bf16(par[OW1 + i]) : par[OW1 + i];
    for (int i = 0; i < HID * HID; ++i) W2[i] = emulate ? oracle_bf16(par[OW2 + i]) : par[OW2 + i];
    for (int i = 0; i < OUT * HID; ++i) W3[i] = emulate ? oracle_bf16(par[OW3 + i]) : par[OW3 + i];
    for (int b = 0; b < B; ++b) {
        double xin[IN], z1[HID], a1[HID], z2[HID], a2[HID];
        for (int i = 0; i < IN; ++i) xin[i] = emulate ? oracle_bf16(x[(long)b * IN + i]) : x[(long)b * IN + i];
        for (int h = 0; h < HID; ++h) {
            double acc = 0.0;
            for (int i = 0; i < IN; ++i) acc += W1[h * IN + i] * xin[i];
            z1[h] = emulate ? f32(acc + (double)par[OB1 + h]) : acc + (double)par[OB1 + h];
            a1[h] = emulate ? oracle_bf16(gelu(z1[h])) : gelu(z1[h]);
        }
        for (int h = 0; h < HID; ++h) {
            double acc = 0.0;
            for (int k = 0; k < HID; ++k) acc += W2[h * HID + k] * a1[k];
            z2[h] = emulate ? f32(acc + (double)par[OB2 + h]) : acc + (double)par[OB2 + h];
            a2[h] = emulate ? oracle_bf16(gelu(z2[h])) : gelu(z2[h]);
        }
        for (int o = 0; o < OUT; ++o) {
            double acc = 0.0;
            for (int k = 0; k < HID; ++k) acc += W3[o * HID + k] * a2[k];
            y[(long)b * OUT + o] = emulate ? f32(acc + (double)par[OB3 + o]) : acc + (double)par[OB3 + o];
        }
        if (z1c) memcpy(z1c + (long)b * HID, z1, sizeof z1);
        if (a1c) memcpy(a1c + (long)b * HID, a1, sizeof a1);
        if (z2c) memcpy(z2c + (long)b * HID, z2, sizeof z2);
        if (a2c) memcpy(a2c + (long)b * HID, a2, sizeof a2);
    }
}

/* Mean-square loss over B rows and 26 outputs and its gradient with respect
 * to every parameter (grad[8090]).  Returns the loss. */
double oracle_mlp_loss_grad(const float *par, int emulate, const double *x, const double *t, int B,
                            double *grad)
{
    double *y = (double *)malloc(sizeof(double) * B * OUT);
    double *z1 = (double *)malloc(sizeof(double) * B * HID), *a1 = (double *)malloc(sizeof(double) * B * HID);
    double *z2 = (double *)malloc(sizeof(double) * B * HID), *a2 = (double *)malloc(sizeof(double) * B * HID);
    oracle_mlp_forward(par, emulate, x, B, y, z1, a1, z2, a2);
    double W2[HID * HID], W3[OUT * HID];
    for (int i = 0; i < HID * HID; ++i) W2[i] = emulate ? oracle_bf16(par[OW2 + i]) : par[OW2 + i];
    for (int i = 0; i < OUT * HID; ++i) W3[i] = emulate ? oracle_bf16(par[OW3 + i]) : par[OW3 + i];
    memset(grad, 0, sizeof(double) * NPAR);
    double loss = 0.0;
    const double scale = 2.0 / ((double)B * OUT);
    for (int b = 0; b < B; ++b) {
        double dy[OUT], dyq[OUT], da2[HID], dz2[HID], dz2q[HID], da1[HID], dz1[HID], dz1q[HID], xin[IN];
        for (int o = 0; o < OUT; ++o) {
            double r = y[(long)b * OUT + o] - t[(long)b * OUT + o];
            loss += r * r;
            dy[o] = emulate ? f32(scale * r) : scale * r;
            dyq[o] = emulate ? oracle_bf16(dy[o]) : dy[o];
        }
        for (int h = 0; h < HID; ++h) {
            double acc = 0.0;
            for (int o = 0; o < OUT; ++o) acc += dyq[o] * W3[o * HID + h];
            da2[h] = emulate ? f32(acc) : acc;
            dz2[h] = da2[h] * gelu_grad(z2[(long)b * HID + h]);
            if (emulate) dz2[h] = f32(dz2[h]);
            dz2q[h] = emulate ? oracle_bf16(dz2[h]) : dz2[h];
        }
        for (int k = 0; k < HID; ++k) {
            double acc = 0.0;
            for (int h = 0; h < HID; ++h) acc += dz2q[h] * W2[h * HID + k];
            da1[k] = emulate ? f32(acc) : acc;
            dz1[k] = da1[k] * gelu_grad(z1[(long)b * HID + k]);
            if (emulate) dz1[k] = f32(dz1[k]);
            dz1q[k] = emulate ? oracle_bf16(dz1[k]) : dz1[k];
        }
        for (int i = 0; i < IN; ++i) xin[i] = emulate ? oracle_bf16(x[(long)b * IN + i]) : x[(long)b * IN + i];
        for (int o = 0; o < OUT; ++o) {
            for (int k = 0; k < HID; ++k) grad[OW3 + o * HID + k] += dyq[o] * a2[(long)b * HID + k];
            grad[OB3 + o] += dy[o];
        }
        for (int h = 0; h < HID; ++h) {
            for (int k = 0; k < HID; ++k) grad[OW2 + h * HID + k] += dz2q[h] * a1[(long)b * HID + k];
            grad[OB2 + h] += dz2[h];
        }
        for (int h = 0; h < HID; ++h) {
            for (int i = 0; i < IN; ++i) grad[OW1 + h * IN + i] += dz1q[h] * xin[i];
            grad[OB1 + h] += dz1[h];
        }
    }
    free(y); free(z1); free(a1); free(z2); free(a2);
    return loss / ((double)B * OUT);
}

/* One Adam update of float32 masters (step t >= 1). */
void oracle_adam(float *par, const double *grad, double *m, double *v, int t, double lr, double b1,
                 double b2, double eps, int n)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        par[i] = (float)((double)par[i] - lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps));
    }
}

/* ------------------------------------------------------------------------ */
/* Features, learned values and the FP64 check                              */
/* ------------------------------------------------------------------------ */

static long pix(int i, int j, int k) { return ((long)(k + GWC) * PBC + (j + GWC)) * PBC + (i + GWC); }
static int d26(int dx, int dy, int dz) { int q = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1); return q < 13 ? q : q - 1; }
static long rix(int i, int j, int k) { return ((long)(k + 1) * RBC + (j + 1)) * RBC + (i + 1); }

static const int LINES[13][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1},
    {0, 1, 1}, {0, 1, -1}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

/* Neighbourhood of field f at cell (i,j,k): nb[27] in dir27 order (centre at
 * 13), sigma and the 34 network inputs.  Returns 1 if the neighbourhood is
 * flat (sigma = 0, inputs untouched). */
int oracle_mlp_features(const double *P, int i, int j, int k, int f, double nb[27], double *sigma,
                        double x[34])
{
    const double *q = P + (long)f * NPADC;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                nb[9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)] = q[pix(i + dx, j + dy, k + dz)];
    double qc = nb[13], s = 0.0;
    for (int o = 0; o < 27; ++o) {
        double a = fabs(nb[o] - qc);
        if (a > s) s = a;
    }
    *sigma = s;
    if (s == 0.0) return 1;
    double r = 1.0 / s;
    for (int o = 0; o < 27; ++o) x[o] = (nb[o] - qc) * r;
    for (int g = 0; g < NFC; ++g) x[27 + g] = (g == f) ? 1.0 : 0.0;
    return 0;
}

/* FP64 acceptance test of the 26 values of one row of field f. */
int oracle_mlp_row_ok(const double nb[27], const double val[26], int f)
{
    double qc = nb[13];
    if (f == 0) {
        /* the network's error is a few percent of sigma; where the density
         * spans more than a factor 8 over the neighbourhood, the low side's
         * point values (and the velocities s / rho formed from them) would
         * carry relative errors of order one */
        double lo = nb[0], hi = nb[0];
        for (int o = 1; o < 27; ++o) {
            if (nb[o] < lo) lo = nb[o];
            if (nb[o] > hi) hi = nb[o];
        }
        if (!(hi <= 8.0 * lo)) return 0;
    }
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                double qn = nb[9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)];
                double v = val[d26(dx, dy, dz)];
                double lo = qc < qn ? qc : qn, hi = qc < qn ? qn : qc;
                if (!(v >= lo && v <= hi)) return 0;
                if ((f == 0 || f == 4 || f == 5) && !(v > 0.0)) return 0;
                if (f == 6 && !(v >= 0.0)) return 0;
            }
    for (int ln = 0; ln < 13; ++ln) {
        const int *d = LINES[ln];
        double R = val[d26(d[0], d[1], d[2])], L = val[d26(-d[0], -d[1], -d[2])];
        if (L == qc && R == qc) continue;
        if (!((R - qc) * (qc - L) > 0.0)) return 0;
        /* no interior extremum: |M6| <= |D|.  The PPM correction puts a pair
         * exactly on this boundary and M6 cancels when |D| << |q|, so allow
         * the rounding of M6: 1e-13 |D| (|L| + |q| + |R|) */
        double D = R - L, M6 = 6.0 * (qc - 0.5 * (L + R));
        double lim = D * D + 1e-13 * fabs(D) * (fabs(L) + fabs(qc) + fabs(R));
        if (D * M6 > lim || D * M6 < -lim) return 0;
    }
    return 1;
}

/* Binary32 rounding toward zero: the nearest binary32 (the C conversion
 * rounds to nearest), moved one unit toward zero where it came out larger in
 * magnitude than x. */
static float rz32(double x)
{
    float f = (float)x;
    if (fabs((double)f) > fabs(x)) f = nextafterf(f, 0.0f);
    return f;
}

/* The plain limiter applied to one row of predicted values: each value is
 * clamped between the cell and its neighbour in that direction, then each
 * line's pair goes through the PPM monotonicity constraint (flatten at an
 * extremum, else pull the far end in).  The limited values are kept as
 * binary32 offsets from q_c, so the point value is q_c + offset: the offset
 * of an end the constraint leaves is its difference from q_c rounded toward
 * zero (toward the cell value, so a clamped end stays within its bounds);
 * a pulled-in end, 3 q_c - 2 R, takes -2 times the other end's rounded
 * offset, which keeps the pair on the constraint's boundary; a flattened
 * pair has offsets zero.  Values that already satisfy both limits change
 * only by that rounding; a NaN stays NaN and fails the check afterwards. */
void oracle_mlp_limit(const double nb[27], double val[26])
{
    double qc = nb[13];
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!dx && !dy && !dz) continue;
                double qn = nb[9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)];
                double lo = qc < qn ? qc : qn, hi = qc < qn ? qn : qc;
                double *v = &val[d26(dx, dy, dz)];
                if (*v < lo) *v = lo;
                if (*v > hi) *v = hi;
            }
    for (int ln = 0; ln < 13; ++ln) {
        const int *d = LINES[ln];
        double *R = &val[d26(d[0], d[1], d[2])], *L = &val[d26(-d[0], -d[1], -d[2])];
        float oR = 0.0f, oL = 0.0f;
        if (!((*R - qc) * (qc - *L) <= 0.0)) {
            int pullL = 0, pullR = 0;
            double D = *R - *L, M6 = 6.0 * (qc - 0.5 * (*L + *R));
            if (D * M6 > D * D)
                pullL = 1;
            else if (D * M6 < -(D * D))
                pullR = 1;
            float fr = rz32(*R - qc), fl = rz32(*L - qc);
            oR = pullR ? -2.0f * fl : fr;
            oL = pullL ? -2.0f * fr : fl;
        }
        *R = qc + (double)oR;
        *L = qc + (double)oL;
    }
}

/* The learned reconstruction of every cell -1..8 of one padded block, row by
 * row and before any fallback.  For cell c (rix order, 10^3 cells) and field
 * f: flat[c*7+f] = 1 where sigma = 0 (the 26 values are q_c, the network is
 * not evaluated and y is left untouched); else y[(c*7+f)*26+d] are the
 * network's outputs (bfloat16-emulating forward), val[(c*7+f)*26+d] the
 * point values q_c + sigma y_d after the plain limiter, and ok[c*7+f] the
 * row's FP64 verdict.  A cell falls back to plain PPM when any of its seven
 * rows fails.  y may be NULL. */
void oracle_learned_rows(const double *P, const float *par, double *y, double *val, unsigned char *ok,
                         unsigned char *flat)
{
    for (int k = -1; k <= NXC; ++k)
        for (int j = -1; j <= NXC; ++j)
            for (int i = -1; i <= NXC; ++i) {
                const long c = rix(i, j, k);
                for (int f = 0; f < NFC; ++f) {
                    const long row = c * NFC + f;
                    double nb[27], s, x[34], yr[26];
                    double *v = val + row * 26;
                    if (oracle_mlp_features(P, i, j, k, f, nb, &s, x)) {
                        for (int d = 0; d < 26; ++d) v[d] = nb[13];
                        flat[row] = 1;
                        ok[row] = 1;
                        continue;
                    }
                    flat[row] = 0;
                    oracle_mlp_forward(par, 1, x, 1, yr, NULL, NULL, NULL, NULL);
                    if (y) memcpy(y + row * 26, yr, sizeof yr);
                    for (int d = 0; d < 26; ++d) v[d] = nb[13] + s * yr[d];
                    oracle_mlp_limit(nb, v);
                    ok[row] = (unsigned char)oracle_mlp_row_ok(nb, v, f);
                }
            }
}

/* Point-value table (oracle_reconstruct_values layout) of one padded block
 * by the learned reconstruction with plain-PPM fallback.  The fluxes need the
 * interior and the face-adjacent ghost cells; *needed and *fallback count the
 * interior cells and those of them that fell back (a ghost cell is counted in
 * its own block).  Every cell -1..8 gets values so the table is complete. */
void oracle_learned_values(const double *P, const float *par, double *V, int *needed, int *fallback)
{
    const long ncell = (long)RBC * RBC * RBC;
    double *Vp = (double *)malloc(sizeof(double) * ncell * 26 * NFC);
    double *val = (double *)malloc(sizeof(double) * ncell * NFC * 26);
    unsigned char *ok = (unsigned char *)malloc((size_t)ncell * NFC);
    unsigned char *flat = (unsigned char *)malloc((size_t)ncell * NFC);
    oracle_reconstruct_values(P, Vp);
    oracle_learned_rows(P, par, NULL, val, ok, flat);
    int nn = 0, nf = 0;
    for (int k = -1; k <= NXC; ++k)
        for (int j = -1; j <= NXC; ++j)
            for (int i = -1; i <= NXC; ++i) {
                int outside = (i < 0 || i >= NXC) + (j < 0 || j >= NXC) + (k < 0 || k >= NXC);
                const long c = rix(i, j, k);
                int cell_ok = 1;
                for (int f = 0; f < NFC; ++f) cell_ok &= ok[c * NFC + f];
                if (outside == 0) {
                    ++nn;
                    nf += !cell_ok;
                }
                for (int d = 0; d < 26; ++d)
                    for (int f = 0; f < NFC; ++f)
                        V[(c * 26 + d) * NFC + f] =
                            cell_ok ? val[(c * NFC + f) * 26 + d] : Vp[(c * 26 + d) * NFC + f];
            }
    free(Vp);
    free(val);
    free(ok);
    free(flat);
    if (needed) *needed = nn;
    if (fallback) *fallback = nf;
}

/* One SSP-RK2 stage of leaves [l0, l1) with the learned reconstruction;
 * otherwise as oracle_stage.  fallback[l] counts leaf l's interior cells that
 * fell back. */
static int learned_values(const double *P, void *ctx, double *V)
{
    int nn, nf;
    oracle_learned_values(P, (const float *)ctx, V, &nn, &nf);
    return nf;
}

int oracle_stage_learned(const void *t, const float *par, int stage, double dt, const double *Uin,
                         const double *Un, const double *dx, const double *origin, const oracle_phys *ph,
                         int l0, int l1, double *Uout, double *amax, int *fallback)
{
    return oracle_stage_with(t, 2, stage, dt, Uin, Un, dx, origin, ph, l0, l1, Uout, amax,
                             learned_values, (void *)par, fallback);
}
