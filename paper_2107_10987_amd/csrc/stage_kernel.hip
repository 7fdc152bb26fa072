// Fused hydro stage kernel for gfx950 (FP64).
//
// One workgroup advances one 8^3 leaf through one Runge-Kutta stage
// (arXiv 2107.10987, section IV-B):
//   1. gather the leaf and its three ghost layers into LDS as a 14^3 x 7
//      structure-of-arrays block (153,664 B): interior cells by coalesced
//      loads, ghost cells through the ghost map (copy, or mean of 2x2x2);
//   2. every thread owns one face of each axis (576 faces per axis, 576
//      threads): for the 9 points of the face it reconstructs the left and
//      right states by PPM along the line through each cell centre that
//      passes through the point, forms the central-upwind point flux and
//      accumulates the Simpson-weighted face flux in registers;
//   3. the face fluxes replace the dead input block in LDS;
//   4. one thread per cell takes the flux divergence, adds the rotating-frame
//      source, applies the stage combine and the dual-energy resync, and
//      stores; the leaf's maximum signal speed is reduced with wave shuffles.
// Reconstructed point values never leave the chip.
//
// Arithmetic is compiled with FP contraction off so limiter decisions and
// results round exactly as the expressions are written.

#include "hydro_common.h"
#include "mlp_common.h"

#include <math.h>

using namespace hydro;

namespace {

constexpr int NT = FACES_PER_AXIS;  // 576 threads: one face per axis each
constexpr int SX_ = 1, SY_ = PB, SZ_ = PB * PB;

__constant__ uint16_t c_ghost_pad[NG];  // padded index of each ghost slot

__device__ __forceinline__ int pidx(int i, int j, int k) {
    return ((k + GW) * PB + (j + GW)) * PB + (i + GW);
}

// pow for the dual-energy switch at face points, which only fires where the
// internal energy is a tiny fraction of the total, and for the tracer resync
// (once per cell and step).  Kept out of line: inlined, its polynomial
// constants are hoisted out of the walk's loops into registers for the whole
// kernel and spilled (a scratch write stream of ~170 B per lane per launch).
__device__ __attribute__((noinline)) double pow_cold(double x, double y) { return pow(x, y); }

// tau^gamma of the dual-energy switch.  For gamma = 5/3 (the double nearest
// it), tau^(5/3) = tau^2 tau^(-1/3) with the cube root by two Newton steps,
// y <- y (4 - a y^3) / 3, from a single-precision estimate of a^(-1/3), where
// tau = m 2^e, e = 3k + r and a = m 2^r in [0.5, 4): within a few ulp of the
// exact power, several times cheaper than pow; other exponents and tau
// outside [2^-330, 2^330] take pow_cold.  Inlined: a wave whose lanes hit the
// switch (leaves behind a strong shock) runs it at every face point, and the
// call's overhead made those leaves, which set the launch's length, 9% slower.
__device__ __forceinline__ double pow_tau(double x, double g) {
    if (g == 5.0 / 3.0 && x >= 0x1p-330 && x <= 0x1p+330) {
        int e;
        const double m = frexp(x, &e);
        const int k = (e >= 0 ? e : e - 2) / 3;   // floor(e / 3)
        const double a = ldexp(m, e - 3 * k);
        double y = (double)__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf((float)a) * (1.0f / 3.0f));
        y = y * (4.0 - a * y * y * y) * (1.0 / 3.0);
        y = y * (4.0 - a * y * y * y) * (1.0 / 3.0);
        return x * x * ldexp(y, -k);
    }
    return pow_cold(x, g);
}

// Monotonised-central slope of the middle value (zero at an extremum),
// computed as m sign dl + m sign dr with m = min(|q+ - q-| / 4, |dl|, |dr|):
// scaling by 2 commutes exactly with min, so 2 m is min(|q+ - q-| / 2,
// 2 |dl|, 2 |dr|) bit for bit; the sum is 2m (exact) with the common sign
// where dl and dr agree, +0 where they differ, and a zero of the right sign
// where a difference is zero (m is then zero), so neither the two doublings
// nor a select nor a multiply are needed.
__device__ __forceinline__ double mc_slope(double qm, double q0, double qp) {
    const double dl = q0 - qm;
    const double dr = qp - q0;
    const double d = 0.25 * (qp - qm);
    // all three operands are finite and non-negative, so fmin (one FP64
    // instruction) selects exactly what the comparisons would
    const double m = fmin(fmin(fabs(d), fabs(dl)), fabs(dr));
    return copysign(m, dl) + copysign(m, dr);
}

// PPM on five values q0..q4 along a line, with the CW84 limiter: left (toward
// q1) and right (toward q3) interface values of the middle cell.
__device__ __forceinline__ void ppm_vals(double q0, double q1, double q2, double q3, double q4,
                                         double &left, double &right) {
    const double sixth = 1.0 / 6.0;
    const double sm = mc_slope(q0, q1, q2);
    const double s0 = mc_slope(q1, q2, q3);
    const double sp = mc_slope(q2, q3, q4);
    // the interface and constraint arithmetic may fuse multiply-adds (results
    // within an ulp or two of the uncontracted expressions)
    {
#pragma clang fp contract(fast)
        double R = q2 + 0.5 * (q3 - q2) - (sp - s0) * sixth;
        double L = q1 + 0.5 * (q2 - q1) - (s0 - sm) * sixth;
        if ((R - q2) * (q2 - L) <= 0.0) {
            L = q2;
            R = q2;
        } else {
            const double D = R - L;
            const double M6 = 6.0 * (q2 - 0.5 * (L + R));
            if (D * M6 > D * D)
                L = 3.0 * q2 - 2.0 * R;
            else if (D * M6 < -(D * D))
                R = 3.0 * q2 - 2.0 * L;
        }
        left = L;
        right = R;
    }
}

// PPM on the five values q(c + m*st), m = -2..2: left (-st end) and right
// (+st end) interface values of the middle cell.
__device__ __forceinline__ void ppm_both(const double *q, int c, int st, double &left,
                                         double &right) {
    ppm_vals(q[c - 2 * st], q[c - st], q[c], q[c + st], q[c + 2 * st], left, right);
}

// Value at the +st end when `plus`, else at the -st end.
__device__ __forceinline__ double ppm_end(const double *q, int c, int st, bool plus) {
    double L, R;
    ppm_both(q, c, st, L, R);
    return plus ? R : L;
}

// Value of every field at direction (dx,dy,dz) of padded cell c.  The line
// through the cell is walked in its canonical orientation (first non-zero
// component positive) so both ends of a line round identically wherever
// they are used.
__device__ __forceinline__ void point_state(const double *P, int c, int dx, int dy, int dz,
                                            double U[NF]) {
    const bool plus = (dx != 0) ? (dx > 0) : ((dy != 0) ? (dy > 0) : (dz > 0));
    int st = dx * SX_ + dy * SY_ + dz * SZ_;
    st = plus ? st : -st;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        U[f] = ppm_end(P + f * NP, c, st, plus);
        __builtin_amdgcn_sched_barrier(0);   // bound the loads in flight (register pressure)
    }
}

// Reciprocal and square root for the flux: the hardware estimates refined by
// Newton steps (within an ulp of the correctly rounded results, a few
// instructions instead of the IEEE sequences).  Valid states have positive
// normal density and non-negative pressure (zero returns zero); where a
// reconstructed state has zero or infinite density the refinement gives NaN
// instead of an infinity, and the stage reports the non-physical result
// either way.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ double sqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    const double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    return x == 0.0 ? x : g;
}

// Euler flux along axis n (run-time) of one reconstructed state; returns |u_n| + c.
// The dual-energy switch is evaluated without contraction, exactly as
// written; the flux arithmetic after it may fuse multiply-adds.
__device__ __forceinline__ double side_flux_rt(int n, const double U[NF], double xq, double yq,
                                               const Phys &ph, double F[NF]) {
    const double rho = U[RHO], E = U[EGAS], tau = U[TAU];
    const double rinv = rcp_nr(rho);
    const double v0 = U[SX] * rinv, v1 = U[SY] * rinv, v2 = U[SZ] * rinv;
    const double ek = 0.5 * (U[SX] * U[SX] + U[SY] * U[SY] + U[SZ] * U[SZ]) * rinv;
    double eint = E - ek;
    if (eint < ph.eta1 * E) eint = pow_tau(tau, ph.gamma);
    {
#pragma clang fp contract(fast)
        // axis n as weights 0 / 1 (uniform): sums in place of selects,
        // adding exact zeros
        const double ex = n == 0 ? 1.0 : 0.0, ey = n == 1 ? 1.0 : 0.0, ez = n == 2 ? 1.0 : 0.0;
        const double vn = ex * v0 + ey * v1 + ez * v2;
        // velocity relative to the grid rotating about z: u = v - omega x r
        const double ux = v0 + ph.omega * yq;
        const double uy = v1 - ph.omega * xq;
        const double un = ex * ux + ey * uy + ez * v2;
        const double p = (ph.gamma - 1.0) * eint;
        const double cs = sqrt_nr(ph.gamma * p * rinv);
        F[RHO] = rho * un;
        F[SX] = U[SX] * un + ex * p;
        F[SY] = U[SY] * un + ey * p;
        F[SZ] = U[SZ] * un + ez * p;
        F[EGAS] = E * un + p * vn;
        F[TAU] = tau * un;
        F[SPC] = U[SPC] * un;
        return fabs(un) + cs;
    }
}

// Euler flux along axis N of one reconstructed state; returns |u_N| + c.
template <int N>
__device__ __forceinline__ double side_flux(const double U[NF], double xq, double yq,
                                            const Phys &ph, double F[NF]) {
    const double rho = U[RHO], E = U[EGAS], tau = U[TAU];
    const double rinv = rcp_nr(rho);
    const double v0 = U[SX] * rinv, v1 = U[SY] * rinv, v2 = U[SZ] * rinv;
    const double vn = (N == 0) ? v0 : ((N == 1) ? v1 : v2);
    // velocity relative to the grid rotating about z: u = v - omega x r
    const double un = (N == 0) ? (v0 + ph.omega * yq) : ((N == 1) ? (v1 - ph.omega * xq) : v2);
    const double ek = 0.5 * (U[SX] * U[SX] + U[SY] * U[SY] + U[SZ] * U[SZ]) * rinv;
    double eint = E - ek;
    if (eint < ph.eta1 * E) eint = pow_tau(tau, ph.gamma);
    const double p = (ph.gamma - 1.0) * eint;
    const double cs = sqrt_nr(ph.gamma * p * rinv);
    F[RHO] = rho * un;
    F[SX] = U[SX] * un;
    F[SY] = U[SY] * un;
    F[SZ] = U[SZ] * un;
    F[1 + N] = F[1 + N] + p;
    F[EGAS] = E * un + p * vn;
    F[TAU] = tau * un;
    F[SPC] = U[SPC] * un;
    return fabs(un) + cs;
}

// Simpson-weighted flux through the face of axis N owned by this thread.
template <int N>
__device__ __forceinline__ void face_flux(const double *P, int r, double dx, const double org[3],
                                          const Phys &ph, bool centre_only, double acc[NF],
                                          double &smax) {
    constexpr int T1 = (N == 0) ? 1 : 0;
    constexpr int T2 = (N == 2) ? 1 : 2;
    constexpr int E0 = (N == 0) ? NX + 1 : NX;
    constexpr int E1 = (N == 1) ? NX + 1 : NX;
    // face r: cell B = (i,j,k) on the high side, A = B - e_N
    const int i = r % E0;
    const int j = (r / E0) % E1;
    const int k = r / (E0 * E1);
    const int cB = pidx(i, j, k);
    constexpr int SN = (N == 0) ? SX_ : ((N == 1) ? SY_ : SZ_);
    const int cA = cB - SN;
    const double xB[3] = {org[0] + (double)i * dx, org[1] + (double)j * dx,
                          org[2] + (double)k * dx};
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0.0;
    const double wts[3] = {1.0 / 36.0, 4.0 / 36.0, 1.0 / 36.0};
    const double wc[3] = {4.0 / 36.0, 16.0 / 36.0, 4.0 / 36.0};
    const int span = centre_only ? 0 : 1;
    for (int a = -span; a <= span; ++a) {
#pragma unroll 1
        for (int b = -span; b <= span; ++b) {
            int dA[3], dB[3];
            dA[N] = 1;
            dB[N] = -1;
            dA[T1] = a;
            dB[T1] = a;
            dA[T2] = b;
            dB[T2] = b;
            double UL[NF], UR[NF], FL[NF], FR[NF];
            point_state(P, cA, dA[0], dA[1], dA[2], UL);
            point_state(P, cB, dB[0], dB[1], dB[2], UR);
            const double xq = xB[0] + 0.5 * (double)dB[0] * dx;
            const double yq = xB[1] + 0.5 * (double)dB[1] * dx;
            const double sl = side_flux<N>(UL, xq, yq, ph, FL);
            const double sr = side_flux<N>(UR, xq, yq, ph, FR);
            // a NaN speed (a side without a real sound speed) makes the
            // point flux NaN, so the stage reports the non-physical state
            const double s = fmax(sl, sr) + 0.0 * (sl + sr);
            smax = s > smax ? s : smax;
            const double w = centre_only ? 1.0 : ((a == 0) ? wc[b + 1] : wts[b + 1]);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double Fq = 0.5 * (FL[f] + FR[f]) - 0.5 * s * (UR[f] - UL[f]);
                acc[f] = acc[f] + w * Fq;
            }
        }
    }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

// Ghost-padded 14^3 block of block b into LDS (NTH threads cooperate): its
// 8^3 cells from U, its ghost cells through the ghost map (a copy, or the mean
// of the 2x2x2 cells of a finer leaf, summed in z, y, x order, or a
// prolongation row).  The loads are issued in two waves: first every load
// whose address is known (the block's own cells, the ghost-map entries and
// their padded positions), then the copied ghost values, all into registers
// before any LDS store, so that each thread waits on memory about twice
// rather than once per ghost cell.  Threads past the end of a range load and
// store the last element again (the same value to the same place).
template <int NTH>
__device__ __forceinline__ void gather_block(double *P, const double *U, const int32_t *gm, int b,
                                             int ts, int lg, const int32_t *prolong, int n_prolong,
                                             int tid) {
    const double *Ub = U + block_base(b, ts, lg);
    const size_t fs = (size_t)1 << (3 * lg);
    constexpr int NI = (LEAF_STRIDE + NTH - 1) / NTH;
    constexpr int NGI = (NG + NTH - 1) / NTH;
    const int32_t *g = gm + (size_t)b * NG;
    double v[NI];
    int srcs[NGI], pads[NGI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = min(tid + i * NTH, LEAF_STRIDE - 1);
        const int f = e >> 9, c = e & (NC - 1);
        v[i] = Ub[f * fs + block_cell(c, lg)];
    }
#pragma unroll
    for (int i = 0; i < NGI; ++i) {
        const int sl = min(tid + i * NTH, NG - 1);
        srcs[i] = g[sl];
        pads[i] = c_ghost_pad[sl];
    }
    // copied ghost values (the common case) straight into registers; means
    // and prolongation rows are formed after
    const int E = 1 << lg, E2 = E * E;
    double gv[NGI][NF];
#pragma unroll
    for (int i = 0; i < NGI; ++i) {
        if (srcs[i] >= 0) {
            const double *q = U + src_offset(srcs[i], lg);
#pragma unroll
            for (int f = 0; f < NF; ++f) gv[i][f] = q[f * fs];
        }
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = min(tid + i * NTH, LEAF_STRIDE - 1);
        const int f = e >> 9, c = e & (NC - 1);
        P[f * NP + pidx(c & 7, (c >> 3) & 7, c >> 6)] = v[i];
    }
#pragma unroll
    for (int i = 0; i < NGI; ++i) {
        const int src = srcs[i];
        if (src >= 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) P[f * NP + pads[i]] = gv[i][f];
        } else if (src < -PROLONG_BASE) {
#pragma unroll 1
            for (int f = 0; f < NF; ++f) P[f * NP + pads[i]] = ghost_value(U, src, f, lg, prolong, n_prolong);
        } else {
            const double *q = U + src_offset(-src - 1, lg);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double *qf = q + f * fs;
                double acc = 0.0;
                acc = acc + qf[0];
                acc = acc + qf[1];
                acc = acc + qf[E];
                acc = acc + qf[E + 1];
                acc = acc + qf[E2];
                acc = acc + qf[E2 + 1];
                acc = acc + qf[E2 + E];
                acc = acc + qf[E2 + E + 1];
                P[f * NP + pads[i]] = acc * 0.125;
            }
        }
    }
}

// Cell size and centre of cell (0,0,0) of block b.
__device__ __forceinline__ void block_geometry(const StageArgs &a, int b, double &dx, double &ox,
                                               double &oy, double &oz) {
    const int leaf = b >> a.ts, t = b & ((1 << a.ts) - 1);
    dx = a.dx[leaf];
    ox = a.origin[3 * leaf] + (double)(8 * (t & 1)) * dx;
    oy = a.origin[3 * leaf + 1] + (double)(8 * ((t >> 1) & 1)) * dx;
    oz = a.origin[3 * leaf + 2] + (double)(8 * (t >> 2)) * dx;
}

// Whether interior cell c lies on one of the faces set in mask (bit
// 2 axis + side, side 1 = the +axis face).
__device__ __forceinline__ bool corrected_cell(int mask, int c) {
    const int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    return ((mask & 1) && i == 0) || ((mask & 2) && i == NX - 1) || ((mask & 4) && j == 0) ||
           ((mask & 8) && j == NX - 1) || ((mask & 16) && k == 0) || ((mask & 32) && k == NX - 1);
}

// Keep the Simpson flux F of boundary face (axis n, index fn in 0..8 along
// n, face cell t1 + 8 t2) when the leaf's flags ask for it.
__device__ __forceinline__ void store_bflux(const StageArgs &a, int leaf, int n, int fn, int t12,
                                            const double F[NF]) {
    if (fn != 0 && fn != NX) return;
    const int phi = 2 * n + (fn == NX ? 1 : 0);
    if (!(a.face_flags[leaf] & (0x101 << phi))) return;
    double *o = a.bflux + (size_t)leaf * BFLUX_STRIDE + phi * NF * NX * NX + t12;
#pragma unroll
    for (int f = 0; f < NF; ++f) o[f * NX * NX] = F[f];
}

// Flux divergence sum dsum (per field, over the three axes) -> L(U), the
// rotating-frame source, the stage combine, the tracer resync and the store
// of one interior cell whose stage input is u; non-physical results are
// reported in a.status.
__device__ __forceinline__ void finish_cell_u(const StageArgs &a, int leaf, int c, double dx, double dt,
                                              const double dsum[NF], const double u[NF]) {
    // leaf: the block; its cell c lives at base in U, fields fs apart
    const double idx = 1.0 / dx;
    const size_t base = block_base(leaf, a.ts, a.lg) + block_cell(c, a.lg);
    const size_t fs = (size_t)1 << (3 * a.lg);
    double L[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) L[f] = -dsum[f] * idx;
    // rotating-frame source -Omega x s
    L[SX] = L[SX] + a.ph.omega * u[SY];
    L[SY] = L[SY] - a.ph.omega * u[SX];
    double o[NF];
    if (a.stage == 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) o[f] = u[f] + dt * L[f];
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) o[f] = a.ca * a.Un[base + f * fs] + a.cb * (u[f] + dt * L[f]);
    }
    // cells on a face the coarse/fine correction changes get their resync
    // after the correction, in the reflux pass
    const int cmask = a.face_flags ? (a.face_flags[leaf] & 63) : 0;
    if (a.last && !(cmask && corrected_cell(cmask, c))) {
        // dual-energy resync of the tracer after the full step
        const double rinv = 1.0 / o[RHO];
        const double ek = 0.5 * (o[SX] * o[SX] + o[SY] * o[SY] + o[SZ] * o[SZ]) * rinv;
        const double eint = o[EGAS] - ek;
        if (eint > a.ph.eta2 * o[EGAS]) o[TAU] = pow_cold(eint, 1.0 / a.ph.gamma);
    }
    bool bad = !(o[RHO] > 0.0);
    int badf = bad ? RHO : -1;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        a.Uout[base + f * fs] = o[f];
        if (!isfinite(o[f]) && !bad) {
            bad = true;
            badf = f;
        }
    }
    if (bad && atomicCAS(&a.status->flag, 0, 1) == 0) {
        const int lf = leaf >> a.ts;
        a.status->leaf = lf;
        a.status->cell = (int)(base - ((size_t)lf * NF << (3 * a.lg)));   // index within the leaf
        a.status->field = badf;
    }
}

// The same, with the cell's stage input read from HBM.
__device__ __forceinline__ void finish_cell(const StageArgs &a, int leaf, int c, double dx,
                                            double dt, const double dsum[NF]) {
    const size_t base = block_base(leaf, a.ts, a.lg) + block_cell(c, a.lg);
    const size_t fs = (size_t)1 << (3 * a.lg);
    double u[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) u[f] = a.Uin[base + f * fs];
    finish_cell_u(a, leaf, c, dx, dt, dsum, u);
}

// Time step of this launch: from device memory when the step is driven
// on the device (graph replay), else the host value.
__device__ __forceinline__ double stage_dt(const StageArgs &a) {
    return a.dt_dev ? *a.dt_dev : a.dt;
}

// Maximum of the per-wave maxima in red[0..nw) -> a.amax[leaf].
__device__ __forceinline__ void store_amax(const StageArgs &a, int leaf, const double *red, int nw) {
    double m = red[0];
    for (int w = 1; w < nw; ++w) m = red[w] > m ? red[w] : m;
    if (a.amax_accumulate) {
        const double old = a.amax[leaf];
        m = old > m ? old : m;
    }
    a.amax[leaf] = m;
}

__global__ void __launch_bounds__(NT) stage_kernel(StageArgs a) {
    __shared__ double P[NF * NP];
    const int leaf = a.leaf0 + xcd_leaf(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;

    gather_block<NT>(P, a.Uin, a.gmap, leaf, a.ts, a.lg, a.prolong, a.n_prolong, tid);
    __syncthreads();

    double dx, org[3];
    block_geometry(a, leaf, dx, org[0], org[1], org[2]);
    double F0[NF], F1[NF], F2[NF];
    double smax = 0.0;
    face_flux<0>(P, tid, dx, org, a.ph, a.centre_only, F0, smax);
    face_flux<1>(P, tid, dx, org, a.ph, a.centre_only, F1, smax);
    face_flux<2>(P, tid, dx, org, a.ph, a.centre_only, F2, smax);
    if (a.bflux) {
        // face r of axis 0: (i, j, k) = (r % 9, r / 9 % 8, r / 72); axis 1:
        // (r % 8, r / 8 % 9, r / 72); axis 2: (r % 8, r / 8 % 8, r / 64)
        store_bflux(a, leaf, 0, tid % 9, (tid / 9) % 8 + 8 * (tid / 72), F0);
        store_bflux(a, leaf, 1, (tid / 8) % 9, tid % 8 + 8 * (tid / 72), F1);
        store_bflux(a, leaf, 2, tid / 64, tid % 64, F2);
    }
    __syncthreads();  // the input block is dead from here on

    double *Fl = P;                      // [f][axis][576]
    double *red = P + NF * NFACE;        // per-wave maxima
    if (a.stage != 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            Fl[(f * 3 + 0) * NT + tid] = F0[f];
            Fl[(f * 3 + 1) * NT + tid] = F1[f];
            Fl[(f * 3 + 2) * NT + tid] = F2[f];
        }
    }
    const double wm = wave_max(smax);
    if ((tid & 63) == 0) red[tid >> 6] = wm;
    __syncthreads();

    if (a.stage != 0 && tid < NC) {
        const int c = tid;
        const int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
        const int rx0 = i + 9 * (j + 8 * k), rx1 = rx0 + 1;
        const int ry0 = i + 8 * (j + 9 * k), ry1 = ry0 + 8;
        const int rz0 = i + 8 * (j + 8 * k), rz1 = rz0 + 64;
        double dsum[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double *Ff = Fl + f * 3 * NT;
            dsum[f] = (Ff[rx1] - Ff[rx0]) + (Ff[NT + ry1] - Ff[NT + ry0]) +
                      (Ff[2 * NT + rz1] - Ff[2 * NT + rz0]);
        }
        finish_cell(a, leaf, c, dx, stage_dt(a), dsum);
    }
    if (tid == 0 && a.amax) store_amax(a, leaf, red, NT / 64);
}


// ---------------------------------------------------------------------------
// Column-walk schedule.
//
// For axis n, the faces normal to n lie on 64 columns of cells along n.  A
// column is held by 10 consecutive lanes, one per cell -1..8 along n (six
// columns per wave; the 192 columns of the three axes are 32 tasks for the
// leaf's 12 waves).  For each of the nine lines through
// a cell that cross a face of axis n (directions e_n + a t1 + b t2), a lane
// runs PPM once and keeps both ends: the end pointing to -n serves the face
// below the cell, and the end pointing to +n is passed one lane up to serve
// the face above it.  The lines are taken in pairs {e_n + a t1 + b t2,
// e_n - a t1 - b t2}, which are exactly the lines the two points (a,b) and
// (-a,-b) of a face need.  Each lane then owns the flux of the face below
// its cell, and one more lane shift gives the flux difference of its cell.
// A line is reconstructed once per axis it crosses (1.71x the minimal PPM
// work of a leaf, against 3x for one face per thread).
// ---------------------------------------------------------------------------

constexpr int NTC = 768;            // 12 waves x 64 lanes: three per SIMD
constexpr int COLS_PER_WAVE = 6;    // 6 columns x 10 cells = 60 lanes

// Both ends of the line through padded cell c along d = (dx,dy,dz) for all
// fields: pos = value at +d, neg = value at -d.  The stencil is walked along
// d itself, which the column walk always gives pointing to +n of its axis;
// the same line met in another axis pass may be walked the other way, which
// rounds its ends differently by at most an ulp (every face flux is still
// computed once and used by both of its cells).
__device__ __forceinline__ void line_ends(const double *P, int c, int dx, int dy, int dz,
                                          double pos[NF], double neg[NF]) {
    const int st = dx * SX_ + dy * SY_ + dz * SZ_;
    const double *q = P + c;
    double a0 = q[-2 * st], a1 = q[-st], a2 = q[0], a3 = q[st], a4 = q[2 * st];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        // the next field's stencil is loaded while this one is reconstructed
        double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0, b4 = 0.0;
        if (f + 1 < NF) {
            const double *qn = q + (f + 1) * NP;
            b0 = qn[-2 * st];
            b1 = qn[-st];
            b2 = qn[0];
            b3 = qn[st];
            b4 = qn[2 * st];
        }
        double L, R;
        ppm_vals(a0, a1, a2, a3, a4, L, R);
        pos[f] = R;
        neg[f] = L;
        // keep the scheduler from hoisting further fields' stencil loads:
        // all seven at once cost ~70 VGPRs and force spills at 12 waves per CU
        __builtin_amdgcn_sched_barrier(0);
        a0 = b0;
        a1 = b1;
        a2 = b2;
        a3 = b3;
        a4 = b4;
    }
}

// Where a lane's point values come from: plain PPM, or (learned
// reconstruction, cell passed the FP64 check) the inference pre-pass.
struct ValSrc {
    const float2 *off;     // this cell's values as offsets from its own value: both ends
                           // (+d, -d) of line l of field f at off[(13 f + l) * 896], or
                           // null for plain PPM
};

// Line (0..12) of each 3x3x3 direction index, + 16 at the line's -d end.
__constant__ mlp::LineOfDir c_line_of = mlp::make_line_of_dir();

// Offsets of the two ends of the line through a cell in direction
// (dx, dy, dz): o.x at +d, o.y at -d of that direction.
__device__ __forceinline__ float2 line_offsets(const float2 *off, int f, int dx, int dy, int dz) {
    const int lt = c_line_of.v[9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)];
    const float2 v = off[(size_t)(f * 13 + (lt & 15)) * mlp::NSLOT];
    return (lt & 16) ? float2{v.y, v.x} : v;
}


template <bool LEARNED>
__device__ __forceinline__ void line_vals(const double *P, int c, int dx, int dy, int dz,
                                          const ValSrc &src, double pos[NF], double neg[NF]) {
    if (LEARNED && src.off) {
        float2 o[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) o[f] = line_offsets(src.off, f, dx, dy, dz);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double qc = P[f * NP + c];
            pos[f] = qc + (double)o[f].x;
            neg[f] = qc + (double)o[f].y;
        }
    } else {
        line_ends(P, c, dx, dy, dz, pos, neg);
    }
}

// Both lines of a pair, d1 and d2: with learned values, every offset of the
// pair is loaded before any is used, so the loads of the two lines are in
// flight together.
template <bool LEARNED>
__device__ __forceinline__ void pair_vals(const double *P, int c, int x1, int y1, int z1, int x2, int y2, int z2,
                                          const ValSrc &src, double pos1[NF], double neg1[NF], double pos2[NF],
                                          double neg2[NF]) {
    if (LEARNED && src.off) {
        float2 o1[NF], o2[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            o1[f] = line_offsets(src.off, f, x1, y1, z1);
            o2[f] = line_offsets(src.off, f, x2, y2, z2);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double qc = P[f * NP + c];
            pos1[f] = qc + (double)o1[f].x;
            neg1[f] = qc + (double)o1[f].y;
            pos2[f] = qc + (double)o2[f].x;
            neg2[f] = qc + (double)o2[f].y;
        }
    } else {
        line_ends(P, c, x1, y1, z1, pos1, neg1);
        line_ends(P, c, x2, y2, z2, pos2, neg2);
    }
}

// Whole-wave lane shifts by one (DPP wave_shr:1 / wave_shl:1, two 32-bit
// moves, no LDS): lane l receives lane l - 1 (up) or l + 1 (down); lanes 0 and
// 63, which have no source, keep their own value.
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double shfl_up1(double v) { return dpp_shift<0x138>(v); }
__device__ __forceinline__ double shfl_down1(double v) { return dpp_shift<0x130>(v); }

// Central-upwind flux at one face point of axis n, Simpson weight w added
// into acc; returns the signal speed.
__device__ __forceinline__ double point_flux_acc(int n, const double UL[NF], const double UR[NF],
                                                 double xq, double yq, const Phys &ph, double w,
                                                 double acc[NF]) {
    double FL[NF], FR[NF];
    const double sl = side_flux_rt(n, UL, xq, yq, ph, FL);
    const double sr = side_flux_rt(n, UR, xq, yq, ph, FR);
    // fmax drops a NaN operand; adding 0 (sl + sr) restores it, so a side
    // without a real sound speed (rho <= 0, p < 0) makes the point flux NaN
    // and the stage reports the non-physical state
    const double s = fmax(sl, sr) + 0.0 * (sl + sr);
    {
#pragma clang fp contract(fast)
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double Fq = 0.5 * (FL[f] + FR[f]) - 0.5 * s * (UR[f] - UL[f]);
            acc[f] = acc[f] + w * Fq;
        }
    }
    return s;
}

// Flux difference F(face above) - F(face below) along axis N (run-time, so
// one copy of the walk serves all three axes) of this lane's cell, for
// column `col` and cell index `cell` in -1..8.  LEARNED: the learned
// reconstruction's values where the pre-pass passed the cell (a separate
// instantiation, so that the plain walk carries none of its registers).
template <bool LEARNED>
__device__ __forceinline__ void column_axis(int N, const double *P, int col, int cell, double dx,
                                            double ox, double oy, double oz, const Phys &ph,
                                            const StageArgs &a, int leaf, bool live, double dsum[NF],
                                            double &smax) {
    const int c1 = col & 7, c2 = col >> 3;
    // cell B on the walk, in (x, y, z): axis N takes `cell`, t1 < t2 take c1, c2
    const int bi = (N == 0) ? cell : c1;
    const int bj = (N == 1) ? cell : ((N == 0) ? c1 : c2);
    const int bk = (N == 2) ? cell : c2;
    const int cB = pidx(bi, bj, bk);
    ValSrc src{nullptr};
    if (LEARNED && a.mlp_off) {
        int blk = leaf, slot = mlp::slot_of(bi, bj, bk);
        if (slot >= NC && a.mlp_alias) {
            // a ghost-slab cell whose row another block of this launch holds
            // (the pre-pass may have skipped this block's copy)
            const int al = a.mlp_alias[(size_t)leaf * (mlp::NSLOT - NC) + slot - NC];
            const int tb = al / mlp::NSLOT;
            if (al >= 0 && tb >= a.leaf0 && tb < a.leaf0 + a.nleaf) {
                blk = tb;
                slot = al - tb * mlp::NSLOT;
            }
        }
        if (a.mlp_ok[(size_t)blk * mlp::NSLOT + slot])
            src.off = (const float2 *)a.mlp_off + (size_t)blk * NF * 13 * mlp::NSLOT + slot;
    }
    const double xB = ox + (double)bi * dx;
    const double yB = oy + (double)bj * dx;
    (void)oz;
    const bool face = cell >= 0;     // lanes of cells 0..8 own the face below them
    double acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0.0;
    // direction e_N + a t1 + b t2 in (x, y, z)
    auto dirx = [N](int a, int b) { return (N == 0) ? 1 : a; };
    auto diry = [N](int a, int b) { return (N == 1) ? 1 : ((N == 0) ? a : b); };
    auto dirz = [N](int a, int b) { return (N == 2) ? 1 : b; };
    // point positions x(B) + d_B dx / 2, d_B = -e_N + a t1 + b t2
    auto qx = [&](int a, int b) { return xB + 0.5 * (double)((N == 0) ? -1 : a) * dx; };
    auto qy = [&](int a, int b) { return yB + 0.5 * (double)((N == 1) ? -1 : ((N == 0) ? a : b)) * dx; };
    {   // the face-normal line serves the face centre
        double pos[NF], neg[NF], prev[NF];
        line_vals<LEARNED>(P, cB, dirx(0, 0), diry(0, 0), dirz(0, 0), src, pos, neg);
#pragma unroll
        for (int f = 0; f < NF; ++f) prev[f] = shfl_up1(pos[f]);
        if (face) {
            const double w0 = a.centre_only ? 1.0 : 16.0 / 36.0;
            const double s = point_flux_acc(N, prev, neg, qx(0, 0), qy(0, 0), ph, w0, acc);
            smax = s > smax ? s : smax;
        }
    }
    // line pairs {(a,b), (-a,-b)} for (a,b) = (1,0), (0,1), (1,1), (1,-1)
    const int npairs = a.centre_only ? 0 : 4;
#pragma unroll 1
    for (int p = 0; p < npairs; ++p) {
        const int ta = (p == 1) ? 0 : 1;
        const int tb = (p == 0) ? 0 : ((p == 3) ? -1 : 1);
        const double w = (p < 2) ? 4.0 / 36.0 : 1.0 / 36.0;
        double pos1[NF], neg1[NF], pos2[NF], neg2[NF];
        pair_vals<LEARNED>(P, cB, dirx(ta, tb), diry(ta, tb), dirz(ta, tb), dirx(-ta, -tb), diry(-ta, -tb),
                           dirz(-ta, -tb), src, pos1, neg1, pos2, neg2);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            pos1[f] = shfl_up1(pos1[f]);
            pos2[f] = shfl_up1(pos2[f]);
        }
        if (face) {
            // point (a,b): left = +end of line (a,b) below, right = -end of line (-a,-b) here
            double s = point_flux_acc(N, pos1, neg2, qx(ta, tb), qy(ta, tb), ph, w, acc);
            smax = s > smax ? s : smax;
            // point (-a,-b): left = +end of line (-a,-b) below, right = -end of line (a,b) here
            s = point_flux_acc(N, pos2, neg1, qx(-ta, -tb), qy(-ta, -tb), ph, w, acc);
            smax = s > smax ? s : smax;
        }
    }
    if (a.bflux && live) store_bflux(a, leaf, N, cell, col, acc);
#pragma unroll
    for (int f = 0; f < NF; ++f) dsum[f] = shfl_down1(acc[f]) - acc[f];
}

// Lane geometry of the column walk.  A leaf's 3 x 64 columns are numbered
// axis-major (column g walks axis g / 64); task t covers columns first + 6t ..
// first + 6t + 5 of a range [first, first + count), one per ten lanes, so the
// lanes of one wave may walk different axes.  Each lane gets its axis, column,
// cell -1..8, and whether it holds a real column (the four spare lanes and
// columns past the range reuse valid cells of the range's first column).
struct ColLane {
    int axis, col, cell, c1, c2;
    bool live;
    __device__ ColLane(int lane, int t, int first, int count) {
        const int slot = lane / 10;
        int g = first + t * COLS_PER_WAVE + slot;
        live = slot < COLS_PER_WAVE && g < first + count;
        g = live ? g : first;
        axis = g / (NX * NX);
        col = g - axis * NX * NX;
        cell = lane - 10 * slot - 1;
        c1 = col & 7;
        c2 = col >> 3;
    }
};

// Flux differences along this lane's axis N of one leaf into that axis's
// workspace slice of W (linear cell index); folds the lane's signal speeds
// into smax.
template <bool LEARNED>
__device__ __forceinline__ void col_axis_to_ws(int N, const StageArgs &a, const double *P,
                                               const ColLane &L, int leaf, double *W, double &smax) {
    double dx, ox, oy, oz;
    block_geometry(a, leaf, dx, ox, oy, oz);
    double d[NF];
    double sm = 0.0;
    column_axis<LEARNED>(N, P, L.col, L.cell, dx, ox, oy, oz, a.ph, a, leaf, L.live, d, sm);
    smax = L.live && sm > smax ? sm : smax;
    if (L.live && L.cell >= 0 && L.cell < NX && a.stage != 0) {
        const int c = (N == 0) ? (L.c2 * NX + L.c1) * NX + L.cell
                    : (N == 1) ? (L.c2 * NX + L.cell) * NX + L.c1
                               : (L.cell * NX + L.c2) * NX + L.c1;
#pragma unroll
        for (int f = 0; f < NF; ++f) W[(N * NF + f) * NC + c] = d[f];
    }
}

// The final pass of a leaf: sum the three axes' differences from W and
// finish every interior cell, whose stage input is still in the LDS block P
// (only a few corner ghost cells may have been overwritten by then).
__device__ __forceinline__ void col_finish_leaf(const StageArgs &a, int leaf, const double *W,
                                                const double *P, int tid, int nt) {
    if (a.stage == 0) return;
    const double dx = a.dx[leaf >> a.ts];
    const double dt = stage_dt(a);
    for (int c = tid; c < NC; c += nt) {
        const int pc = pidx(c & 7, (c >> 3) & 7, c >> 6);
        double dsum[NF], u[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            dsum[f] = (W[(0 * NF + f) * NC + c] + W[(1 * NF + f) * NC + c]) + W[(2 * NF + f) * NC + c];
            u[f] = P[f * NP + pc];
        }
        finish_cell_u(a, leaf, c, dx, dt, dsum, u);
    }
}

// The columns [first, first + count) of a leaf as six-column tasks: a wave
// takes task w (its index) first and then the next task from the counter in
// LDS (which starts at the wave count), so the tasks spread evenly over the
// SIMDs whatever the order the waves run in.  Columns of one axis write that
// axis's slice of W only, so no barrier separates the axes.
template <bool LEARNED>
__device__ __forceinline__ void walk_columns(const StageArgs &a, const double *P, int leaf,
                                             double *W, int first, int count, int *next_task,
                                             int tid, double &smax) {
    const int lane = tid & 63;
    const int ntask = (count + COLS_PER_WAVE - 1) / COLS_PER_WAVE;
    int task = tid >> 6;
#pragma unroll 1
    while (task < ntask) {
        const ColLane L(lane, task, first, count);
        col_axis_to_ws<LEARNED>(L.axis, a, P, L, leaf, W, smax);
        int t = 0;
        if (lane == 0) t = atomicAdd(next_task, 1);
        task = __builtin_amdgcn_readfirstlane(t);
    }
}

// Maximum over the workgroup's waves of smax, left in red[0 .. NTC/64);
// red may alias the input block (the barriers retire it first).
__device__ __forceinline__ void block_max(double smax, double *red, int tid) {
    const double wm = wave_max(smax);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = wm;
    __syncthreads();
}

// One leaf per workgroup, all three axes, then the leaf is finished from
// the three slices.
template <bool LEARNED>
__global__ void __launch_bounds__(NTC) stage_kernel_col(StageArgs a) {
    __shared__ double P[NF * NP];
    __shared__ int next_task;
    const int leaf = a.leaf0 + xcd_leaf(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    if (tid == 0) next_task = NTC / 64;
    gather_block<NTC>(P, a.Uin, a.gmap, leaf, a.ts, a.lg, a.prolong, a.n_prolong, tid);
    __syncthreads();
    double *W = a.dscr + (size_t)leaf * 3 * NF * NC;
    double smax = 0.0;
    walk_columns<LEARNED>(a, P, leaf, W, 0, 3 * NX * NX, &next_task, tid, smax);
    __syncthreads();   // every slice of W is written
    col_finish_leaf(a, leaf, W, P, tid, NTC);
    block_max(smax, P, tid);
    if (tid == 0 && a.amax) store_amax(a, leaf, P, NTC / 64);
}

// Persistent workgroups over a queue of (leaf, tile) items.  With one tile a
// workgroup does whole leaves; with three, an item is one axis of a leaf and
// the workgroup that completes a leaf's last axis finishes the leaf, so a
// small batch spreads over three times as many compute units.  Whole leaves
// come from one counter (a fast compute unit takes more of them).  Axis
// items are split into one contiguous (Morton) range per XCD, each with its
// own counter: a workgroup takes items from its XCD's range, so the three
// axis items of a leaf, which write and read the same workspace slices, and
// its neighbours' ghost cells stay in one L2; when that range is empty it
// takes the next items of the other ranges in turn (measured: tiled launches
// 6-8% faster than with one counter, whole-leaf launches 3-10% slower).  The
// last workgroup to leave resets the counters for the next launch.
__device__ __forceinline__ int next_item(int *queue, int items, int xcd) {
    const int q = items / NXCD, r = items % NXCD;
    for (int k = 0; k < NXCD; ++k) {
        const int x = (xcd + k) & (NXCD - 1);
        const int len = q + (x < r ? 1 : 0);
        // a device-coherent read skips exhausted ranges without an atomic
        if (__hip_atomic_load(&queue[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len) continue;
        const int i = atomicAdd(&queue[x], 1);
        if (i < len) return x * q + (x < r ? x : r) + i;
    }
    return items;
}
template <bool LEARNED>
__global__ void __launch_bounds__(NTC) stage_kernel_col_persistent(StageArgs a) {
    __shared__ double P[NF * NP];
    __shared__ int item_s, last_s, next_task;
    const int tid0 = threadIdx.x;
    const int T = a.tiles;
    const int items = a.nleaf * T;
    for (;;) {
        // a per-iteration copy of the thread index the compiler cannot see
        // through: what the body derives from it is recomputed each item
        // instead of hoisted out of the loop and kept live across the walk
        int tid = tid0;
        asm volatile("" : "+v"(tid));
        if (tid == 0) {
            item_s = T == 1 ? atomicAdd(&a.queue[0], 1) : next_item(a.queue, items, (int)(blockIdx.x % NXCD));
            next_task = NTC / 64;
        }
        __syncthreads();
        const int item = item_s;
        if (item >= items) break;
        const int leaf = a.leaf0 + item / T;
        const int tile = item - (item / T) * T;
        gather_block<NTC>(P, a.Uin, a.gmap, leaf, a.ts, a.lg, a.prolong, a.n_prolong, tid);
        __syncthreads();
        double *W = a.dscr + (size_t)leaf * 3 * NF * NC;
        double smax = 0.0;
        // one tile: all 192 columns; three: the 64 columns of axis `tile`
        walk_columns<LEARNED>(a, P, leaf, W, T == 1 ? 0 : tile * NX * NX, T == 1 ? 3 * NX * NX : NX * NX,
                     &next_task, tid, smax);
        if (T == 1) {
            __syncthreads();   // every slice of W is written
            col_finish_leaf(a, leaf, W, P, tid, NTC);
            block_max(smax, P, tid);
            if (tid == 0 && a.amax) store_amax(a, leaf, P, NTC / 64);
        } else {
            block_max(smax, P, tid);
            if (tid == 0) {
                double m = P[0];
                for (int w = 1; w < NTC / 64; ++w) m = P[w] > m ? P[w] : m;
                a.tile_amax[(size_t)leaf * 3 + tile] = m;
                __threadfence();   // publish W and the tile maximum device-wide
                last_s = atomicAdd(&a.leaf_done[leaf], 1) == T - 1;
                if (last_s) {
                    __threadfence();
                    a.leaf_done[leaf] = 0;
                }
            }
            __syncthreads();
            if (last_s) {
                __threadfence();   // see the other tiles' W
                col_finish_leaf(a, leaf, W, P, tid, NTC);
                if (tid == 0 && a.amax) {
                    double *r = P;   // reuse: the three tile maxima
                    r[0] = a.tile_amax[(size_t)leaf * 3 + 0];
                    r[1] = a.tile_amax[(size_t)leaf * 3 + 1];
                    r[2] = a.tile_amax[(size_t)leaf * 3 + 2];
                    store_amax(a, leaf, r, 3);
                }
            }
        }
        __syncthreads();   // LDS, item_s and next_task are reused by the next item
    }
    if (tid0 == 0) {
        __threadfence();
        if (atomicAdd(&a.queue[NXCD], 1) == (int)gridDim.x - 1) {
            for (int x = 0; x <= NXCD; ++x) a.queue[x] = 0;
            __threadfence();
        }
    }
}

// Flux correction of one coarse leaf after a stage: for each face shared
// with four finer leaves, the stage used the leaf's own flux Fc through the
// face; the conservative flux is the mean Ff of the finer faces' fluxes, so
// the face cell's L(U) changes by -(Ff - Fc)/dx on a +axis face and by
// +(Ff - Fc)/dx on a -axis face, and the stage output by cb dt times that.
// Faces are taken one after another (a cell on an edge or corner can sit on
// two or three of them); then the corrected cells get the tracer resync the
// stage kernel left out, and the non-physical check.
constexpr int NTR = NF * NX * NX;   // 448 threads: (field, face cell)

__global__ void __launch_bounds__(NTR) reflux_kernel(RefluxArgs r) {
    const int32_t *e = r.entries + (size_t)blockIdx.x * REFLUX_ENTRY;
    const int leaf = e[0], mask = e[1];
    const int tid = threadIdx.x;
    const int f = tid >> 6, t12 = tid & 63;
    const int t1 = t12 & 7, t2 = t12 >> 3;
    const double dt = r.dt_dev ? *r.dt_dev : r.dt;
    const double idx = 1.0 / r.dx[leaf >> r.ts];
    // the entry's block (an 8^3 tile of a leaf of 2^lg cells per edge)
    double *Ul = r.U + block_base(leaf, r.ts, r.lg);
    const size_t fs = (size_t)1 << (3 * r.lg);
    for (int phi = 0; phi < NBFACE; ++phi) {
        if (!((mask >> phi) & 1)) continue;   // uniform over the workgroup
        const int n = phi >> 1, side = phi & 1;
        const int child = e[2 + 4 * phi + (t1 >> 2) + 2 * (t2 >> 2)];
        const int cphi = 2 * n + (1 - side);   // the finer leaves' face on the shared plane
        const double *Fch = r.bflux + (size_t)child * BFLUX_STRIDE + (cphi * NF + f) * NX * NX;
        const int a0 = 2 * (t1 & 3), b0 = 2 * (t2 & 3);
        const double Ff = ((Fch[a0 + NX * b0] + Fch[a0 + 1 + NX * b0]) +
                           (Fch[a0 + NX * (b0 + 1)] + Fch[a0 + 1 + NX * (b0 + 1)])) * 0.25;
        const double Fc = r.bflux[(size_t)leaf * BFLUX_STRIDE + (phi * NF + f) * NX * NX + t12];
        const double dF = Ff - Fc;
        const double dL = (side ? -dF : dF) * idx;
        const int cn = side ? NX - 1 : 0;
        const int i = (n == 0) ? cn : t1;
        const int j = (n == 1) ? cn : ((n == 0) ? t1 : t2);
        const int k = (n == 2) ? cn : t2;
        double *u = Ul + f * fs + block_cell((k * NX + j) * NX + i, r.lg);
        *u = *u + r.cb * (dt * dL);
        __syncthreads();
    }
    for (int c = tid; c < NC; c += NTR) {
        if (!corrected_cell(mask, c)) continue;
        double *uc = Ul + block_cell(c, r.lg);
        double o[NF];
#pragma unroll
        for (int g = 0; g < NF; ++g) o[g] = uc[g * fs];
        if (r.last) {
            const double rinv = 1.0 / o[RHO];
            const double ek = 0.5 * (o[SX] * o[SX] + o[SY] * o[SY] + o[SZ] * o[SZ]) * rinv;
            const double eint = o[EGAS] - ek;
            if (eint > r.ph.eta2 * o[EGAS]) {
                o[TAU] = pow(eint, 1.0 / r.ph.gamma);
                uc[TAU * fs] = o[TAU];
            }
        }
        bool bad = !(o[RHO] > 0.0);
        int badf = bad ? RHO : -1;
#pragma unroll
        for (int g = 0; g < NF; ++g)
            if (!isfinite(o[g]) && !bad) {
                bad = true;
                badf = g;
            }
        if (bad && atomicCAS(&r.status->flag, 0, 1) == 0) {
            const int lf = leaf >> r.ts;
            r.status->leaf = lf;
            r.status->cell = (int)(uc - r.U - ((size_t)lf * NF << (3 * r.lg)));   // index within the leaf
            r.status->field = badf;
        }
    }
}

// Reconstructed values at the 26 points of every interior cell.
__global__ void __launch_bounds__(NT) reconstruct_kernel(const double *U, const int32_t *gm,
                                                         const int32_t *prolong, int n_prolong,
                                                         double *out) {
    __shared__ double P[NF * NP];
    const int leaf = blockIdx.x;
    gather_block<NT>(P, U, gm, leaf, 0, 3, prolong, n_prolong, threadIdx.x);
    __syncthreads();
    double *o = out + (size_t)leaf * NF * NC * 26;
    for (int e = threadIdx.x; e < NC * 26; e += NT) {
        const int c = e / 26;
        int d = e - c * 26;
        const int d27 = d < 13 ? d : d + 1;
        const int dx = d27 % 3 - 1, dy = (d27 / 3) % 3 - 1, dz = d27 / 9 - 1;
        double v[NF];
        point_state(P, pidx(c & 7, (c >> 3) & 7, c >> 6), dx, dy, dz, v);
#pragma unroll
        for (int f = 0; f < NF; ++f) o[((size_t)f * NC + c) * 26 + d] = v[f];
    }
}

}  // namespace

hipError_t hydro_upload_ghost_table(const uint16_t *table) {
    return hipMemcpyToSymbol(HIP_SYMBOL(c_ghost_pad), table, sizeof(uint16_t) * NG);
}

hipError_t hydro_launch_stage(const StageArgs &a, hipStream_t s) {
    if (a.nleaf <= 0) return hipSuccess;
    switch (a.kernel) {
    case KERNEL_FACE:
        hipLaunchKernelGGL(stage_kernel, dim3(a.nleaf), dim3(NT), 0, s, a);
        break;
    case KERNEL_COLUMN:
        if (a.mlp_off)
            hipLaunchKernelGGL(stage_kernel_col<true>, dim3(a.nleaf), dim3(NTC), 0, s, a);
        else
            hipLaunchKernelGGL(stage_kernel_col<false>, dim3(a.nleaf), dim3(NTC), 0, s, a);
        break;
    default: {   // persistent column walk
        const int items = a.nleaf * a.tiles;
        const int grid = items < a.grid_limit ? items : a.grid_limit;
        if (a.mlp_off)
            hipLaunchKernelGGL(stage_kernel_col_persistent<true>, dim3(grid), dim3(NTC), 0, s, a);
        else
            hipLaunchKernelGGL(stage_kernel_col_persistent<false>, dim3(grid), dim3(NTC), 0, s, a);
    }
    }
    return hipGetLastError();
}

// Training pairs of the learned reconstruction from the plain one: for each
// interior cell and field, the normalised 3x3x3 neighbourhood with the field's
// one-hot id (X [.][34], FP32 of the FP64 values) and the plain PPM values at
// the 26 points in the same normalisation (T [.][26]); rows are
// [leaf][cell][field], and valid = 0 marks flat neighbourhoods (sigma = 0).
__global__ void __launch_bounds__(NT) pairs_kernel(const double *U, const int32_t *gm,
                                                   const int32_t *prolong, int n_prolong, float *X,
                                                   float *T, uint8_t *valid) {
    __shared__ double P[NF * NP];
    const int leaf = blockIdx.x;
    gather_block<NT>(P, U, gm, leaf, 0, 3, prolong, n_prolong, threadIdx.x);
    __syncthreads();
    for (int e = threadIdx.x; e < NC * NF; e += NT) {
        const int c = e / NF, f = e - (e / NF) * NF;
        const int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
        const int pc = pidx(i, j, k);
        const double *q = P + f * NP;
        const double qc = q[pc];
        double sigma = 0.0;
        for (int o = 0; o < 27; ++o) {
            const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            const double d = fabs(q[pc + dx * SX_ + dy * SY_ + dz * SZ_] - qc);
            sigma = d > sigma ? d : sigma;
        }
        const size_t row = ((size_t)leaf * NC + c) * NF + f;
        valid[row] = sigma > 0.0 ? 1 : 0;
        const double rs = sigma > 0.0 ? 1.0 / sigma : 0.0;
        for (int o = 0; o < 27; ++o) {
            const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            X[row * 34 + o] = (float)((q[pc + dx * SX_ + dy * SY_ + dz * SZ_] - qc) * rs);
        }
        for (int g = 0; g < NF; ++g) X[row * 34 + 27 + g] = (g == f) ? 1.f : 0.f;
        for (int o = 0; o < 27; ++o) {
            if (o == 13) continue;
            const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            const bool plus = (dx != 0) ? (dx > 0) : ((dy != 0) ? (dy > 0) : (dz > 0));
            int st = dx * SX_ + dy * SY_ + dz * SZ_;
            st = plus ? st : -st;
            const double v = ppm_end(q, pc, st, plus);
            T[row * 26 + (o < 13 ? o : o - 1)] = (float)((v - qc) * rs);
        }
    }
}

hipError_t hydro_launch_pairs(const double *U, const int32_t *gm, const int32_t *prolong, int n_prolong,
                              int n, float *X, float *T, uint8_t *valid, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pairs_kernel, dim3(n), dim3(NT), 0, s, U, gm, prolong, n_prolong, X, T, valid);
    return hipGetLastError();
}

// dt = cfl * min over blocks of dx / a_max (blocks b of leaf b >> ts), by
// one workgroup of 1024 threads (the minimum is exact in any order).
constexpr int NTDT = 1024;
__global__ void __launch_bounds__(NTDT) dt_kernel(const double *dx, const double *amax, int n, int ts,
                                                  double cfl, double *dt_out) {
    __shared__ double red[NTDT / 64];
    double m = INFINITY;
    const int nb = n << ts;
    for (int b = threadIdx.x; b < nb; b += NTDT) {
        const double v = dx[b >> ts] / amax[b];
        m = v < m ? v : m;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(m, o, 64);
        m = u < m ? u : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int w = 1; w < NTDT / 64; ++w) r = red[w] < r ? red[w] : r;
        *dt_out = cfl * r;
    }
}

hipError_t hydro_launch_reflux(const RefluxArgs &r, int n_entries, hipStream_t s) {
    if (n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(reflux_kernel, dim3(n_entries), dim3(NTR), 0, s, r);
    return hipGetLastError();
}

hipError_t hydro_launch_dt(const double *dx, const double *amax, int n, int ts, double cfl,
                           double *dt_out, hipStream_t s) {
    hipLaunchKernelGGL(dt_kernel, dim3(1), dim3(NTDT), 0, s, dx, amax, n, ts, cfl, dt_out);
    return hipGetLastError();
}

// Per-leaf maximum of the signal speeds of its 2^ts blocks.
__global__ void __launch_bounds__(256) amax_leaves_kernel(const double *blk, int ts, int n, double *out) {
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= n) return;
    double m = blk[(size_t)l << ts];
    for (int t = 1; t < (1 << ts); ++t) {
        const double v = blk[((size_t)l << ts) + t];
        m = v > m ? v : m;
    }
    out[l] = m;
}

hipError_t hydro_launch_amax_leaves(const double *blk, int ts, int n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(amax_leaves_kernel, dim3((n + 255) / 256), dim3(256), 0, s, blk, ts, n, out);
    return hipGetLastError();
}

hipError_t hydro_launch_reconstruct(const double *U, const int32_t *gmap, const int32_t *prolong,
                                    int n_prolong, int n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reconstruct_kernel, dim3(n), dim3(NT), 0, s, U, gmap, prolong, n_prolong, out);
    return hipGetLastError();
}
