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

#include <math.h>

using namespace hydro;

namespace {

constexpr int NT = FACES_PER_AXIS;  // 576 threads: one face per axis each
constexpr int SX_ = 1, SY_ = PB, SZ_ = PB * PB;

__constant__ uint16_t c_ghost_pad[NG];  // padded index of each ghost slot

__device__ __forceinline__ int pidx(int i, int j, int k) {
    return ((k + GW) * PB + (j + GW)) * PB + (i + GW);
}

// Monotonised-central slope of the middle value (zero at an extremum).
__device__ __forceinline__ double mc_slope(double qm, double q0, double qp) {
    const double dl = q0 - qm;
    const double dr = qp - q0;
    const double d = 0.5 * (qp - qm);
    double m = fabs(d);
    const double a = 2.0 * fabs(dl);
    const double b = 2.0 * fabs(dr);
    m = (a < m) ? a : m;
    m = (b < m) ? b : m;
    return (dl * dr > 0.0) ? copysign(m, d) : 0.0;
}

// PPM on the five values q(c + m*st), m = -2..2, with the CW84 limiter.
// Returns the value at the +st end when `plus`, else at the -st end.
__device__ __forceinline__ double ppm_end(const double *q, int c, int st, bool plus) {
    const double q0 = q[c - 2 * st];
    const double q1 = q[c - st];
    const double q2 = q[c];
    const double q3 = q[c + st];
    const double q4 = q[c + 2 * st];
    const double sixth = 1.0 / 6.0;
    const double sm = mc_slope(q0, q1, q2);
    const double s0 = mc_slope(q1, q2, q3);
    const double sp = mc_slope(q2, q3, q4);
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
    for (int f = 0; f < NF; ++f) U[f] = ppm_end(P + f * NP, c, st, plus);
}

// Euler flux along axis N of one reconstructed state; returns |u_N| + c.
template <int N>
__device__ __forceinline__ double side_flux(const double U[NF], double xq, double yq,
                                            const Phys &ph, double F[NF]) {
    const double rho = U[RHO], E = U[EGAS], tau = U[TAU];
    const double rinv = 1.0 / rho;
    const double v0 = U[SX] * rinv, v1 = U[SY] * rinv, v2 = U[SZ] * rinv;
    const double vn = (N == 0) ? v0 : ((N == 1) ? v1 : v2);
    // velocity relative to the grid rotating about z: u = v - omega x r
    const double un = (N == 0) ? (v0 + ph.omega * yq) : ((N == 1) ? (v1 - ph.omega * xq) : v2);
    const double ek = 0.5 * (U[SX] * U[SX] + U[SY] * U[SY] + U[SZ] * U[SZ]) * rinv;
    double eint = E - ek;
    if (eint < ph.eta1 * E) eint = pow(tau, ph.gamma);
    const double p = (ph.gamma - 1.0) * eint;
    const double cs = sqrt(ph.gamma * p * rinv);
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
                                          const Phys &ph, double acc[NF], double &smax) {
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
    for (int a = -1; a <= 1; ++a) {
#pragma unroll 1
        for (int b = -1; b <= 1; ++b) {
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
            const double s = sl > sr ? sl : sr;
            smax = s > smax ? s : smax;
            const double w = (a == 0) ? wc[b + 1] : wts[b + 1];
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

// Ghost-padded block of one leaf into LDS.
__device__ __forceinline__ void gather_block(double *P, const double *U, const int32_t *gm,
                                             int leaf, int tid) {
    const double *Ul = U + (size_t)leaf * LEAF_STRIDE;
    for (int e = tid; e < LEAF_STRIDE; e += NT) {
        const int f = e >> 9, c = e & (NC - 1);
        P[f * NP + pidx(c & 7, (c >> 3) & 7, c >> 6)] = Ul[e];
    }
    const int32_t *g = gm + (size_t)leaf * NG;
    for (int s = tid; s < NG; s += NT) {
        const int src = g[s];
        const int p = c_ghost_pad[s];
        if (src >= 0) {
            const double *q = U + (size_t)(src >> 9) * LEAF_STRIDE + (src & (NC - 1));
#pragma unroll
            for (int f = 0; f < NF; ++f) P[f * NP + p] = q[f * NC];
        } else {
            const int b = -src - 1;
            const double *q = U + (size_t)(b >> 9) * LEAF_STRIDE + (b & (NC - 1));
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const double *qf = q + f * NC;
                double acc = 0.0;
                acc = acc + qf[0];
                acc = acc + qf[1];
                acc = acc + qf[8];
                acc = acc + qf[9];
                acc = acc + qf[64];
                acc = acc + qf[65];
                acc = acc + qf[72];
                acc = acc + qf[73];
                P[f * NP + p] = acc * 0.125;
            }
        }
    }
}

__global__ void __launch_bounds__(NT) stage_kernel(StageArgs a) {
    __shared__ double P[NF * NP];
    const int leaf = a.leaf0 + blockIdx.x;
    const int tid = threadIdx.x;

    gather_block(P, a.Uin, a.gmap, leaf, tid);
    __syncthreads();

    const double dx = a.dx[leaf];
    const double org[3] = {a.origin[3 * leaf], a.origin[3 * leaf + 1], a.origin[3 * leaf + 2]};
    double F0[NF], F1[NF], F2[NF];
    double smax = 0.0;
    face_flux<0>(P, tid, dx, org, a.ph, F0, smax);
    face_flux<1>(P, tid, dx, org, a.ph, F1, smax);
    face_flux<2>(P, tid, dx, org, a.ph, F2, smax);
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
        const double idx = 1.0 / dx;
        const size_t base = (size_t)leaf * LEAF_STRIDE + c;
        double u[NF], L[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double *Ff = Fl + f * 3 * NT;
            const double d = (Ff[rx1] - Ff[rx0]) + (Ff[NT + ry1] - Ff[NT + ry0]) +
                             (Ff[2 * NT + rz1] - Ff[2 * NT + rz0]);
            L[f] = -d * idx;
            u[f] = a.Uin[base + (size_t)f * NC];
        }
        // rotating-frame source -Omega x s
        L[SX] = L[SX] + a.ph.omega * u[SY];
        L[SY] = L[SY] - a.ph.omega * u[SX];
        double o[NF];
        if (a.stage == 1) {
#pragma unroll
            for (int f = 0; f < NF; ++f) o[f] = u[f] + a.dt * L[f];
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) o[f] = 0.5 * (a.Un[base + (size_t)f * NC] + (u[f] + a.dt * L[f]));
            // dual-energy resync of the tracer after the full step
            const double rinv = 1.0 / o[RHO];
            const double ek = 0.5 * (o[SX] * o[SX] + o[SY] * o[SY] + o[SZ] * o[SZ]) * rinv;
            const double eint = o[EGAS] - ek;
            if (eint > a.ph.eta2 * o[EGAS]) o[TAU] = pow(eint, 1.0 / a.ph.gamma);
        }
        bool bad = !(o[RHO] > 0.0);
        int badf = bad ? RHO : -1;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            a.Uout[base + (size_t)f * NC] = o[f];
            if (!isfinite(o[f]) && !bad) {
                bad = true;
                badf = f;
            }
        }
        if (bad && atomicCAS(&a.status->flag, 0, 1) == 0) {
            a.status->leaf = leaf;
            a.status->cell = c;
            a.status->field = badf;
        }
    }
    if (tid == 0 && a.amax) {
        double m = red[0];
        for (int w = 1; w < NT / 64; ++w) m = red[w] > m ? red[w] : m;
        if (a.amax_accumulate) {
            const double old = a.amax[leaf];
            m = old > m ? old : m;
        }
        a.amax[leaf] = m;
    }
}

// Reconstructed values at the 26 points of every interior cell.
__global__ void __launch_bounds__(NT) reconstruct_kernel(const double *U, const int32_t *gm,
                                                         double *out) {
    __shared__ double P[NF * NP];
    const int leaf = blockIdx.x;
    gather_block(P, U, gm, leaf, threadIdx.x);
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
    hipLaunchKernelGGL(stage_kernel, dim3(a.nleaf), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t hydro_launch_reconstruct(const double *U, const int32_t *gmap, int n, double *out,
                                    hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reconstruct_kernel, dim3(n), dim3(NT), 0, s, U, gmap, out);
    return hipGetLastError();
}
