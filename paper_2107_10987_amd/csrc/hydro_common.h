// Shared definitions of the gfx950 hydro library (device and host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hydro {

constexpr int NX = 8;                      // cells per leaf edge
constexpr int GW = 3;                      // ghost layers
constexpr int PB = NX + 2 * GW;            // padded edge: 14
constexpr int NF = 7;                      // rho, sx, sy, sz, E, tau, X
constexpr int NC = NX * NX * NX;           // 512 interior cells
constexpr int NP = PB * PB * PB;           // 2744 padded cells
constexpr int NG = NP - NC;                // 2232 ghost cells
constexpr int FACES_PER_AXIS = (NX + 1) * NX * NX;  // 576
constexpr int NFACE = 3 * FACES_PER_AXIS;           // 1728
constexpr int LEAF_STRIDE = NF * NC;                // doubles per leaf in U

enum Field { RHO = 0, SX = 1, SY = 2, SZ = 3, EGAS = 4, TAU = 5, SPC = 6 };

struct Phys {
    double gamma;
    double omega;
    double eta1;
    double eta2;
};

// Non-physical result report written by the stage kernels.
struct Status {
    int flag;       // 0 ok, 1 non-physical value produced
    int leaf;
    int cell;
    int field;
};

struct StageArgs {
    const double *Uin;        // [n][7][512] stage input (ghost source)
    const double *Un;         // [n][7][512] step start (stage 2)
    double *Uout;             // [n][7][512]
    const double *dx;         // [n]
    const double *origin;     // [n][3]
    const int32_t *gmap;      // [n][2232]
    double *amax;             // [n] or null
    Status *status;
    Phys ph;
    double dt;
    int leaf0;                // first leaf of this launch
    int nleaf;                // leaves in this launch
    int stage;                // 1, 2, 3; 0 = signal speed only
    int last;                 // last stage of the step: tracer resync
    double ca, cb;            // stage > 1: Uout = ca Un + cb (Uin + dt L)
    int centre_only;          // old scheme: one flux point per face, weight 1
    int amax_accumulate;      // stage 2 of a step: amax = max(amax, this stage)
    int kernel;               // KERNEL_* below
    double *dscr;             // column walk: [n][3][7][512] per-axis flux differences
    const double *dt_dev;     // if set, dt is read from device memory
    // persistent column walk
    int tiles;                // 1: whole leaves; 3: one axis per item
    int grid_limit;           // workgroups of a persistent launch
    int *queue;               // [QUEUE_INTS]: next item of each XCD's range, workgroups
                              // finished (zero between launches)
    int *leaf_done;           // [n] axis tiles finished per leaf (zero between launches)
    double *tile_amax;        // [n][3]
    // learned reconstruction (null: plain PPM)
    const float *mlp_off;     // [n][7][13][896][2] learned point values as binary32 offsets
                              // from the cell value (field, line, slot, +d / -d end)
    const uint8_t *mlp_ok;    // [n][896]
    const int32_t *mlp_alias; // [n][384] shared rows of ghost-slab cells (block * 896 + slot), or null
    // flux correction at coarse/fine faces (null: none)
    const int32_t *face_flags;  // [n]: bits 0-5 corrected faces, 8-13 faces kept for a coarser leaf
    double *bflux;              // [n][6][7][64] Simpson flux of flagged boundary faces
    // leaf edge E = 1 << lg cells (8 or 16); kernels work on 8^3 blocks, 1 << ts per leaf
    int ts, lg;
    // linear-prolongation rows named by ghost-map entries below -PROLONG_BASE
    const int32_t *prolong;   // [n_prolong][PROLONG_ROW] or null
    int n_prolong;
};

// Leaves of E = 2^lg cells per edge (8 or 16) are processed as (E/8)^3 tiles
// of 8^3 cells ("blocks"): block b is tile t = b mod 2^ts of leaf b >> ts, at
// cell offset 8 (t & 1, (t >> 1) & 1, t >> 2) inside the leaf.  Everything a
// kernel keeps per unit of work (ghost map, workspace, signal speed, learned
// values) is per block; U, dx and origin are per leaf.  For 8^3 leaves
// (ts = 0, lg = 3) a block is a leaf.
__device__ __forceinline__ size_t block_base(int b, int ts, int lg) {
    const int leaf = b >> ts, t = b & ((1 << ts) - 1);
    const size_t E = (size_t)1 << lg;
    return ((size_t)leaf * NF << (3 * lg)) +
           ((size_t)(8 * (t >> 2)) * E + (size_t)(8 * ((t >> 1) & 1))) * E + (size_t)(8 * (t & 1));
}
// Offset from the block's base of its cell c = (k * 8 + j) * 8 + i.
__device__ __forceinline__ int block_cell(int c, int lg) {
    return ((c >> 6) << (2 * lg)) + (((c >> 3) & 7) << lg) + (c & 7);
}
// U offset (field 0) of the cell a ghost-map entry names, s = leaf E^3 + cell.
__device__ __forceinline__ size_t src_offset(int s, int lg) {
    const int sh = 3 * lg;
    return ((size_t)(s >> sh) * NF << sh) + (size_t)(s & ((1 << sh) - 1));
}

// Ghost-map entries: s >= 0 copies cell s; -PROLONG_BASE <= s < 0 is the mean
// of the 2x2x2 cells whose lowest is -s-1; s < -PROLONG_BASE names row
// -s-PROLONG_BASE-1 of the prolongation table: {C, C-x, C+x, C-y, C+y, C-z,
// C+z (each a copy or mean entry), side bits}, the coarse cell containing the
// ghost cell, its neighbours at C's level, and bit a set when the ghost cell
// is the upper half of C along axis a.
constexpr int PROLONG_BASE = 1 << 30;
constexpr int PROLONG_ROW = 8;

// Field f (fields fs = E^3 apart) of a copy or mean entry.
__device__ __forceinline__ double src_value(const double *U, int s, int f, int lg) {
    const size_t fs = (size_t)1 << (3 * lg);
    if (s >= 0) return U[src_offset(s, lg) + f * fs];
    const double *qf = U + src_offset(-s - 1, lg) + f * fs;
    const int E = 1 << lg, E2 = E * E;
    double acc = 0.0;
    acc = acc + qf[0];
    acc = acc + qf[1];
    acc = acc + qf[E];
    acc = acc + qf[E + 1];
    acc = acc + qf[E2];
    acc = acc + qf[E2 + 1];
    acc = acc + qf[E2 + E];
    acc = acc + qf[E2 + E + 1];
    return acc * 0.125;
}

__device__ __forceinline__ double minmod2(double a, double b) {
    if (!(a * b > 0.0)) return 0.0;
    return fabs(a) <= fabs(b) ? a : b;
}

// Linear-limited prolongation of field f from a table row: U_C plus, axis by
// axis in x, y, z order, (+-1/4) minmod(U_{C+e} - U_C, U_C - U_{C-e}).
__device__ __forceinline__ double prolong_value(const double *U, const int32_t *row, int f, int lg) {
    const double uc = src_value(U, row[0], f, lg);
    double v = uc;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double um = src_value(U, row[1 + 2 * a], f, lg);
        const double up = src_value(U, row[2 + 2 * a], f, lg);
        const double frac = ((row[7] >> a) & 1) ? 0.25 : -0.25;
        v = v + frac * minmod2(up - uc, uc - um);
    }
    return v;
}

// Field f of whatever a ghost-map entry names; an out-of-range prolongation
// row (a map used with the wrong table) gives NaN, which the stage reports.
__device__ __forceinline__ double ghost_value(const double *U, int s, int f, int lg, const int32_t *prolong,
                                              int n_prolong) {
    if (s >= -PROLONG_BASE) return src_value(U, s, f, lg);
    const int r = -s - PROLONG_BASE - 1;
    if (!prolong || r >= n_prolong) return __builtin_nan("");
    return prolong_value(U, prolong + (size_t)r * PROLONG_ROW, f, lg);
}

// Boundary faces of a leaf: f = 2 axis + side (side 1 = +axis); the 64 face
// cells of a face by (t1, t2) = the two other axes in increasing order,
// index t1 + 8 t2.
constexpr int NBFACE = 6;
constexpr int BFLUX_STRIDE = NBFACE * NF * NX * NX;   // doubles per leaf
constexpr int REFLUX_ENTRY = 26;                      // {leaf, mask, child[6][4]}

struct RefluxArgs {
    double *U;                // [n][7][E^3] stage output, corrected in place
    const double *bflux;      // [blocks][6][7][64]
    const int32_t *entries;   // [m][26], leaf and children are blocks
    const double *dx;         // [n] per leaf
    double dt;
    const double *dt_dev;     // if set, dt is read from device memory
    double cb;                // weight of dt L in the stage combine
    int last;                 // last stage: tracer resync of the corrected cells
    Phys ph;
    Status *status;
    int ts, lg;               // blocks per leaf (log2), leaf edge (log2)
};

enum Kernel { KERNEL_FACE = 0, KERNEL_COLUMN = 1, KERNEL_PERSISTENT = 2 };

// XCDs of the chip (workgroups are dispatched round-robin over them) and the
// persistent queue's counters: one per XCD's item range, then the count of
// finished workgroups.
constexpr int NXCD = 8;
constexpr int QUEUE_INTS = 16;

// Leaf (within a launch of n leaves, one workgroup each) of workgroup b.
// Workgroups are dispatched round-robin over the chip's 8 XCDs (b runs on
// XCD b % 8), each with its own L2; XCD x gets a contiguous range of the
// launch's leaves, which are in Morton order, so the ghost cells a workgroup
// reads mostly belong to leaves its own L2 has just seen.  A bijection on
// [0, n); every leaf's result is independent of which workgroup computes it.
__device__ __forceinline__ int xcd_leaf(int b, int n) {
    const int q = n / NXCD, r = n % NXCD;
    const int x = b % NXCD, k = b / NXCD;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace hydro

// Launchers implemented in the kernel translation unit.
hipError_t hydro_upload_ghost_table(const uint16_t *table);
// Host helpers of the API translation unit: one-time upload of the ghost-slot
// tables to a device, and the thread's handle-less error text.
hipError_t hydro_internal_ghost_table(int dev);
void hydro_internal_set_error(const char *msg);
hipError_t hydro_launch_stage(const hydro::StageArgs &a, hipStream_t s);
hipError_t hydro_launch_reflux(const hydro::RefluxArgs &r, int n_entries, hipStream_t s);
hipError_t hydro_launch_dt(const double *dx, const double *amax, int n, int ts, double cfl,
                           double *dt_out, hipStream_t s);
hipError_t hydro_launch_amax_leaves(const double *blk, int ts, int n, double *out, hipStream_t s);
hipError_t hydro_launch_pairs(const double *U, const int32_t *gm, const int32_t *prolong, int n_prolong,
                              int n, float *X, float *T, uint8_t *valid, hipStream_t s);
hipError_t hydro_launch_reconstruct(const double *U, const int32_t *gmap, const int32_t *prolong,
                                    int n_prolong, int n, double *out, hipStream_t s);
