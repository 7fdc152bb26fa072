// Shared definitions of the learned-reconstruction kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hydro {
namespace mlp {

constexpr int IN = 34, HID = 64, OUT = 26, NPAR = 8090;
// offsets in the float32 parameter vector
constexpr int P_W1 = 0, P_B1 = 2176, P_W2 = 2240, P_B2 = 6336, P_W3 = 6400, P_B3 = 8064;
// offsets in the bf16 MFMA copies: W1p[64][64], W2[64][64], W3p[32][64]
constexpr int WB_W1 = 0, WB_W2 = 4096, WB_W3 = 8192, WB_SIZE = 10240;
// transposed copies for the backward pass: W2T[64][64], W3T[64][64]
constexpr int WB_W2T = 0, WB_W3T = 4096, WBT_SIZE = 8192;
// inference image (bf16): W1i[64][32] (the 27 neighbourhood inputs, zero
// padded), W2i[64][64] and W3i[32][64] with permuted columns and rows, as 16
// MFMA operand fragments of 512 values; its float32 biases: b1 per field (the
// one-hot input's weight folded in), b2, b3
constexpr int NNB = 27;
// weight-gradient reduction: 36 MFMA tiles (W3 2 x 4, W2 4 x 4, W1 4 x 3) per
// batch slice
constexpr int WG_TILES = 36, WG_SLICES = 16;
constexpr int WBI_SIZE = 8192;
constexpr int BI_B1 = 0, BI_B2 = 448, BI_B3 = 512, BI_SIZE = 544;
// cells whose reconstruction a leaf's fluxes need: 512 interior + 6 x 64
// ghost cells sharing a face with the leaf
constexpr int NSLOT = 896;

// Slot of a needed cell (i, j, k in -1..8, at most one coordinate outside
// 0..7): interior cells by linear index; face-adjacent ghost cells after them,
// slab x-, x+, y-, y+, z-, z+, each by its two in-leaf coordinates in axis order.
__host__ __device__ inline int slot_of(int i, int j, int k) {
    if (i >= 0 && i < 8 && j >= 0 && j < 8 && k >= 0 && k < 8) return (k * 8 + j) * 8 + i;
    if (i < 0 || i > 7) return 512 + 64 * (i < 0 ? 0 : 1) + j + 8 * k;
    if (j < 0 || j > 7) return 512 + 64 * (j < 0 ? 2 : 3) + i + 8 * k;
    return 512 + 64 * (k < 0 ? 4 : 5) + i + 8 * j;
}

// The 13 lines of the learned reconstruction in the network's output order,
// by the 3x3x3 index 9 (dz+1) + 3 (dy+1) + (dx+1) of their +d direction:
// (1,0,0), (0,1,0), (0,0,1), (1,1,0), (1,-1,0), (1,0,1), (1,0,-1), (0,1,1),
// (0,1,-1), (1,1,1), (1,1,-1), (1,-1,1), (1,-1,-1).
constexpr int LINE_DIR[13] = {14, 16, 22, 17, 11, 23, 5, 25, 7, 26, 8, 20, 2};

// Line of each 3x3x3 direction index: l, or l + 16 where the index is the
// line's -d end (-1 for the centre).
struct LineOfDir {
    int v[27];
};
constexpr LineOfDir make_line_of_dir() {
    LineOfDir t{};
    for (int k = 0; k < 27; ++k) t.v[k] = -1;
    for (int l = 0; l < 13; ++l) {
        t.v[LINE_DIR[l]] = l;
        t.v[26 - LINE_DIR[l]] = l + 16;
    }
    return t;
}

// Binary32 rounding toward zero of x: the nearest binary32, stepped one unit
// toward zero where it came out larger in magnitude (sign-magnitude bits:
// one less in the integer view is one unit smaller in magnitude).
__device__ __forceinline__ float rz32(double x) {
    float f = (float)x;
    if (fabs((double)f) > fabs(x)) f = __int_as_float(__float_as_int(f) - 1);
    return f;
}

// The plain limiter on a predicted pair of one line (R at +d, L at -d), the
// cell value qc and its neighbours nbR (at +d) and nbL (at -d): each value
// clamped between the cell and its neighbour in that direction, then the PPM
// monotonicity constraint on the pair (unfused FP64).  The results are kept
// as binary32 offsets from qc (the point value is qc + offset in FP64),
// rounded toward zero, i.e. toward the cell value, so a clamped end stays
// between the cell and its neighbour; an end the constraint pulls in
// (3 qc - 2 R, offset -2 (R - qc)) takes -2 times the other end's rounded
// offset (exact), so the pair stays on the constraint's boundary.  min/max
// clamps carry a NaN prediction to a bound; the pre-pass's check fails it.
__device__ __forceinline__ void learned_limit(double qc, double nbR, double nbL, double R, double L, float &oR,
                                              float &oL) {
    const double loR = fmin(qc, nbR), hiR = fmax(qc, nbR);
    const double loL = fmin(qc, nbL), hiL = fmax(qc, nbL);
    const double r = fmin(fmax(R, loR), hiR), l = fmin(fmax(L, loL), hiL);
    const bool ext = (r - qc) * (qc - l) <= 0.0;
    const double D = r - l, M6 = 6.0 * (qc - 0.5 * (l + r));
    const double DM = D * M6, DD = D * D;
    const bool lowL = DM > DD, lowR = !lowL & (DM < -DD);
    const float fr = rz32(r - qc), fl = rz32(l - qc);
    oR = ext ? 0.0f : (lowR ? -2.0f * fl : fr);
    oL = ext ? 0.0f : (lowL ? -2.0f * fr : fl);
}

struct MlpTrain {
    float *par, *m, *v, *grad;          // [NPAR]
    uint16_t *wb, *wbT;                 // bf16 MFMA copies
    uint16_t *wbi;                      // [WBI_SIZE] inference image
    float *bi;                          // [BI_SIZE] inference biases
    uint16_t *xb, *a1, *a2, *dz1, *dz2; // [B][64] bf16
    float *z1, *z2, *dz1f, *dz2f;       // [B][64]
    float *y, *dy;                      // [B][32]
    float *loss_rows;                   // [B]
    float *gpart;                       // [WG_SLICES][NPAR] per-slice gradients
};

struct MlpInfer {
    const double *U;            // [n][7][E^3]
    const int32_t *gmap;        // [blocks][2232]
    const uint16_t *wbi;        // bf16 inference image
    const float *bi;            // its float32 biases
    float *off;                 // [blocks][7][13][896][2] point values as offsets from the cell
                                // value (field, line, slot, +d / -d end), or null
    double *val;                // the same as FP64 point values, or null
    uint8_t *cell_ok;           // [blocks][896]
    unsigned long long *fb_count;  // cells that fell back to plain PPM
    int leaf0;                  // first block of the launch
    int ts, lg;                 // blocks per leaf (log2), leaf edge (log2)
    const int32_t *prolong;     // linear-prolongation rows (or null)
    int n_prolong;
    float *yraw;                // null, or [blocks][7][896][26]: the network's outputs per row
    const int32_t *alias;       // null, or [blocks][384]: ghost-slab rows shared with another
                                // block (block * 896 + slot); all-shared slabs of the launch are skipped
};

}  // namespace mlp
}  // namespace hydro

hipError_t hydro_mlp_upload_pad_ghost(const int16_t *pad_ghost);
hipError_t hydro_mlp_launch_infer(const hydro::mlp::MlpInfer &m, int nleaf, hipStream_t s);
hipError_t hydro_mlp_launch_pack(const hydro::mlp::MlpTrain &t, hipStream_t s);
hipError_t hydro_mlp_launch_forward(const hydro::mlp::MlpTrain &t, const float *X, int B, hipStream_t s);
hipError_t hydro_mlp_launch_grad(const hydro::mlp::MlpTrain &t, const float *T, int B, float *loss,
                                 hipStream_t s);
hipError_t hydro_mlp_launch_adam(const hydro::mlp::MlpTrain &t, float lr, float b1, float b2, float eps,
                                 float c1, float c2, hipStream_t s);
