// Learned reconstruction on gfx950: a 34-64-64-26 tanh-GELU network on
// normalised 3x3x3 neighbourhoods, bfloat16 operands and FP32 accumulation on
// MFMA (training: v_mfma_f32_16x16x16_bf16; inference:
// v_mfma_f32_16x16x32_bf16), with every value that reaches the FP64 scheme
// checked in FP64 (neighbour bounds, per-line PPM monotonicity, positivity).
//
// Parameter vector (float32 masters, 8090 values): W1[64][34], b1[64],
// W2[64][64], b2[64], W3[26][64], b3[26].  The MFMA copies are bfloat16,
// zero-padded to W1p[64][64] and W3p[32][64].
//
// MFMA operand layout of the 16x16x16 bf16 instruction (lane l, q = l / 16):
//   A[m][k]: lane holds m = l % 16, k = 4q .. 4q+3
//   B[k][n]: lane holds n = l % 16, k = 4q .. 4q+3
//   D[m][n]: lane holds n = l % 16, m = 4q .. 4q+3

#include "hydro_common.h"
#include "mlp_common.h"

#include <math.h>

using namespace hydro;
using namespace hydro::mlp;

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Training kernels: LDS staging of a wave's 64 rows, bf16 rows of 64 padded to a 68-element
// (136 B) stride, FP32 output rows of 32 padded to 34 (136 B).  Rows written
// one per lane then fall in different banks, and the 8-byte MFMA operand
// loads stay aligned.
constexpr int LDA = 68;
constexpr int LDY = 34;
constexpr int STAGE_ELEMS = 64 * LDA;   // bf16 elements per wave

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// binary32 -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr float GELU_C = 0.7978845608028654f;
constexpr float GELU_A = 0.044715f;

__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + tanhf(GELU_C * (z + GELU_A * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
    const float t = tanhf(GELU_C * (z + GELU_A * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * GELU_C * (1.0f + 3.0f * GELU_A * z * z);
}

// One layer for a wave's 64 rows: Z[r][n] = sum_k A[r][k] W[n][k] + b[n],
// A in LDS (bf16, row stride 64), W bf16 [NT*16][64] in global memory.
// Results in D layout: z[mt][nt] holds rows 16 mt + 4q + i, column 16 nt + l%16.
template <int NTILE>
__device__ __forceinline__ void layer(const uint16_t *A, const uint16_t *W, int lane, v4f z[4][NTILE]) {
    const int r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTILE; ++nt) z[mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        v4s b[NTILE];
#pragma unroll
        for (int nt = 0; nt < NTILE; ++nt)
            b[nt] = *(const v4s *)(W + (16 * nt + r) * 64 + 16 * kb + 4 * q);   // global, stride 64
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const v4s a = *(const v4s *)(A + (16 * mt + r) * LDA + 16 * kb + 4 * q);
#pragma unroll
            for (int nt = 0; nt < NTILE; ++nt) z[mt][nt] = mfma(a, b[nt], z[mt][nt]);
        }
    }
}

// Bias, GELU and bfloat16 rounding of a hidden layer back into the staging
// buffer S (rows x 64); optionally keeps z (FP32) and a (bf16) per row in
// global memory for the backward pass.
__device__ __forceinline__ void hidden_out(v4f z[4][4], const float *bias, uint16_t *S, int lane,
                                           float *zsave, uint16_t *asave, int row0, int nrows) {
    const int c = lane & 15, q = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * mt + 4 * q + i, col = 16 * nt + c;
                const float zz = z[mt][nt][i] + bias[col];
                const uint16_t a = bf16_bits(gelu(zz));
                S[row * LDA + col] = a;
                if (zsave && row < nrows) {
                    zsave[(size_t)(row0 + row) * 64 + col] = zz;
                    asave[(size_t)(row0 + row) * 64 + col] = a;
                }
            }
}

// Forward pass of the 64 rows staged (as bf16 inputs) in S; the 26 outputs of
// row r land in Y[r][0..25] (FP32, row stride LDY, aliasing S).
__device__ __forceinline__ void forward64(uint16_t *S, const uint16_t *Wb, const float *par, int lane,
                                          float *z1s, uint16_t *a1s, float *z2s, uint16_t *a2s, int row0,
                                          int nrows) {
    v4f z[4][4];
    layer<4>(S, Wb + WB_W1, lane, z);
    hidden_out(z, par + P_B1, S, lane, z1s, a1s, row0, nrows);
    layer<4>(S, Wb + WB_W2, lane, z);
    hidden_out(z, par + P_B2, S, lane, z2s, a2s, row0, nrows);
    v4f y[4][2];
    layer<2>(S, Wb + WB_W3, lane, y);
    float *Y = (float *)S;
    const int c = lane & 15, q = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * mt + 4 * q + i, col = 16 * nt + c;
                if (col < OUT) Y[row * LDY + col] = y[mt][nt][i] + par[P_B3 + col];
            }
}

// GELU for inference: 0.5 z (1 + tanh u) = z / (1 + exp(-2u)),
// u = C (z + A z^3) = z (C + C A z^2), with the hardware exp2 and reciprocal
// (relative error ~1e-7, far below the bfloat16 rounding that follows).
__device__ __forceinline__ float gelu_fast(float z) {
    constexpr float K = -2.0f * 1.4426950408889634f;   // exp(-2u) = exp2(K u)
    const float e = __builtin_amdgcn_exp2f(z * __builtin_fmaf(z * z, K * GELU_C * GELU_A, K * GELU_C));
    return z * __builtin_amdgcn_rcpf(1.0f + e);
}

}  // namespace

// ---------------------------------------------------------------------------
// Training
// ---------------------------------------------------------------------------

// Forward of B rows of X [B][34] (float32); keeps what the backward needs.
__global__ void __launch_bounds__(256) mlp_train_forward(MlpTrain t, const float *X, int B) {
    __shared__ uint16_t S[4][STAGE_ELEMS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row0 = (blockIdx.x * 4 + w) * 64;
    if (row0 >= B) return;                        // wave-uniform
    const int nrows = B - row0 < 64 ? B - row0 : 64;
    uint16_t *s = S[w];
    // row `lane`: inputs rounded to bf16, zero padding beyond 34 and beyond B
    for (int k = 0; k < 64; ++k) {
        const float v = (lane < nrows && k < IN) ? X[(size_t)(row0 + lane) * IN + k] : 0.f;
        const uint16_t b = bf16_bits(v);
        s[lane * LDA + k] = b;
        if (lane < nrows) t.xb[(size_t)(row0 + lane) * 64 + k] = b;
    }
    forward64(s, t.wb, t.par, lane, t.z1, t.a1, t.z2, t.a2, row0, nrows);
    const float *Y = (const float *)s;
    if (lane < nrows)
        for (int o = 0; o < OUT; ++o) t.y[(size_t)(row0 + lane) * 32 + o] = Y[lane * LDY + o];
}

// dY = 2 (y - T) / (B * 26); dZ2 = (dY W3) * gelu'(z2); dZ1 = (dZ2 W2) * gelu'(z1).
// One wave per 64 rows; per-row loss partials.
__global__ void __launch_bounds__(256) mlp_train_backward_rows(MlpTrain t, const float *T, int B) {
    __shared__ uint16_t S[4][STAGE_ELEMS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row0 = (blockIdx.x * 4 + w) * 64;
    if (row0 >= B) return;
    const int nrows = B - row0 < 64 ? B - row0 : 64;
    uint16_t *s = S[w];
    const float scale = 2.0f / ((float)B * OUT);
    float loss = 0.f;
    for (int o = 0; o < 64; ++o) {
        float d = 0.f;
        if (lane < nrows && o < OUT) {
            const float r = t.y[(size_t)(row0 + lane) * 32 + o] - T[(size_t)(row0 + lane) * OUT + o];
            loss += r * r;
            d = scale * r;
            t.dy[(size_t)(row0 + lane) * 32 + o] = d;
        }
        s[lane * LDA + o] = bf16_bits(d);   // dY as the A operand (k = output index)
    }
    if (lane < nrows) t.loss_rows[row0 + lane] = loss;
    // dA2[r][h] = sum_o dY[r][o] W3[o][h]: B operand[k = o][n = h] = W3[o][h] -> W3T copy
    v4f z[4][4];
    layer<4>(s, t.wbT + WB_W3T, lane, z);
    const int c = lane & 15, q = lane >> 4;
    // dZ2 = dA2 * gelu'(z2) -> bf16 into s (A operand of the next product) and global
    for (int mt = 0; mt < 4; ++mt)
        for (int nt = 0; nt < 4; ++nt)
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * mt + 4 * q + i, col = 16 * nt + c;
                float d = 0.f;
                if (row < nrows) d = z[mt][nt][i] * gelu_grad(t.z2[(size_t)(row0 + row) * 64 + col]);
                if (row < nrows) t.dz2f[(size_t)(row0 + row) * 64 + col] = d;
                const uint16_t b = bf16_bits(d);
                s[row * LDA + col] = b;
                if (row < nrows) t.dz2[(size_t)(row0 + row) * 64 + col] = b;
            }
    layer<4>(s, t.wbT + WB_W2T, lane, z);
    for (int mt = 0; mt < 4; ++mt)
        for (int nt = 0; nt < 4; ++nt)
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * mt + 4 * q + i, col = 16 * nt + c;
                if (row < nrows) {
                    const float d = z[mt][nt][i] * gelu_grad(t.z1[(size_t)(row0 + row) * 64 + col]);
                    t.dz1f[(size_t)(row0 + row) * 64 + col] = d;
                    t.dz1[(size_t)(row0 + row) * 64 + col] = bf16_bits(d);
                }
            }
}

// Weight and bias gradients, summed over the batch in a fixed order: the
// batch is cut into WG_SLICES slices of whole 16-row blocks; workgroup
// (slice, tile) reduces its slice for one 16 x 16 tile of one weight matrix on
// MFMA (and, for the first tile of a row block, the bias sums) into the
// slice's partial vector; mlp_grad_reduce then adds the slices in order.
__global__ void __launch_bounds__(64) mlp_train_wgrad(MlpTrain t, int B) {
    const int lane = threadIdx.x;
    const int tile = blockIdx.x % WG_TILES, slice = blockIdx.x / WG_TILES;
    const int per = (B + 16 * WG_SLICES - 1) / (16 * WG_SLICES) * 16;
    const int r0 = slice * per, r1 = min(B, r0 + per);
    float *gp = t.gpart + (size_t)slice * NPAR;
    const uint16_t *dZ, *A;
    int mt, nt, ldz, gofs, mrows, ncols;
    if (tile < 8) {            // W3: dZ = dY (bf16 copy), A = a2
        dZ = nullptr; A = t.a2; mt = tile / 4; nt = tile % 4; ldz = 32; gofs = P_W3; mrows = OUT; ncols = HID;
    } else if (tile < 24) {    // W2: dZ = dZ2, A = a1
        dZ = t.dz2; A = t.a1; mt = (tile - 8) / 4; nt = (tile - 8) % 4; ldz = 64; gofs = P_W2; mrows = HID; ncols = HID;
    } else {                   // W1: dZ = dZ1, A = x
        dZ = t.dz1; A = t.xb; mt = (tile - 24) / 3; nt = (tile - 24) % 3; ldz = 64; gofs = P_W1; mrows = HID; ncols = IN;
    }
    const int r = lane & 15, q = lane >> 4;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int b0 = r0; b0 < r1; b0 += 16) {
        // A operand [m][k = batch]: dZ[b0 + 4q + i][16 mt + r]
        v4s a, bb;
        for (int i = 0; i < 4; ++i) {
            const int row = b0 + 4 * q + i;
            uint16_t va = 0, vb = 0;
            if (row < r1) {
                const int m = 16 * mt + r, n = 16 * nt + r;
                if (m < mrows) va = dZ ? dZ[(size_t)row * ldz + m] : bf16_bits(t.dy[(size_t)row * 32 + m]);
                vb = A[(size_t)row * 64 + n];
            }
            a[i] = (short)va;
            bb[i] = (short)vb;
        }
        acc = mfma(a, bb, acc);
    }
    for (int i = 0; i < 4; ++i) {
        const int m = 16 * mt + 4 * q + i, n = 16 * nt + r;
        if (m < mrows && n < ncols) gp[gofs + m * ncols + n] = acc[i];
    }
    // bias gradients: the first tile of each matrix's row block sums columns
    if (nt == 0 && lane < 16) {
        const int m = 16 * mt + lane;
        if (m < mrows) {
            float s = 0.f;
            for (int b = r0; b < r1; ++b)
                s += (tile < 8) ? t.dy[(size_t)b * 32 + m]
                                : (tile < 24 ? t.dz2f[(size_t)b * 64 + m] : t.dz1f[(size_t)b * 64 + m]);
            const int bofs = tile < 8 ? P_B3 : (tile < 24 ? P_B2 : P_B1);
            gp[bofs + m] = s;
        }
    }
}

// grad = the slices' partial gradients added in slice order.
__global__ void __launch_bounds__(256) mlp_grad_reduce(MlpTrain t) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= NPAR) return;
    float s = 0.f;
    for (int sl = 0; sl < WG_SLICES; ++sl) s += t.gpart[(size_t)sl * NPAR + i];
    t.grad[i] = s;
}

// Loss = sum of per-row partials / (B * 26), summed in row order.
__global__ void __launch_bounds__(64) mlp_loss_reduce(MlpTrain t, int B, float *loss_out) {
    __shared__ float red[64];
    float s = 0.f;
    for (int b = threadIdx.x; b < B; b += 64) s += t.loss_rows[b];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.f;
        for (int i = 0; i < 64; ++i) tot += red[i];
        *loss_out = tot / ((float)B * OUT);
    }
}

// Adam on the float32 masters, then the bf16 MFMA copies (plain and
// transposed, zero padded).
__global__ void __launch_bounds__(256) mlp_adam(MlpTrain t, float lr, float b1, float b2, float eps,
                                                float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= NPAR) return;
    const float g = t.grad[i];
    const float m = b1 * t.m[i] + (1.f - b1) * g;
    const float v = b2 * t.v[i] + (1.f - b2) * g * g;
    t.m[i] = m;
    t.v[i] = v;
    t.par[i] = t.par[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ---------------------------------------------------------------------------
// Inference weight image
// ---------------------------------------------------------------------------
//
// Inference runs the network transposed, Z^T = W X^T: the weights are the A
// operand of v_mfma_f32_16x16x32_bf16 (lane l holds unit 16 mt + l % 16 and
// eight consecutive k), the 16 rows of a tile the B operand (lane l holds row
// l % 16 and the same eight k), so a layer's result lands with lane l holding
// row l % 16, units 16 mt + 4 (l / 16) + i.  Those sixteen values are exactly
// the B operand of the next layer if its k order lists, per 32-unit block kb
// and lane group q, units 32 kb + 4q + 0..3 and then 32 kb + 16 + 4q + 0..3:
// the image stores the next layer's weight columns in that order, and no
// activation ever goes through LDS.  The output layer's rows are ordered so
// that output position 16 e + 4q + t is end e (0: +d, 1: -d) of line 4q + t:
// the lanes of a row's group q hold both ends of up to four lines.

namespace {

// the +d direction (index into the 3x3x3 neighbourhood, 13 = centre) of the
// 13 lines in the network's output order
__constant__ int c_lines[13] = {LINE_DIR[0], LINE_DIR[1], LINE_DIR[2],  LINE_DIR[3],  LINE_DIR[4],
                                LINE_DIR[5], LINE_DIR[6], LINE_DIR[7],  LINE_DIR[8],  LINE_DIR[9],
                                LINE_DIR[10], LINE_DIR[11], LINE_DIR[12]};

// hidden unit at k position kap of a 64-wide layer input
__device__ __forceinline__ int hidden_of(int kap) {
    const int kb = kap >> 5, q = (kap >> 3) & 3, j = kap & 7;
    return 32 * kb + (j < 4 ? 4 * q + j : 16 + 4 * q + j - 4);
}

// network output (0..25) at output position o of the image, -1 for padding
__device__ __forceinline__ int output_of(int o) {
    const int e = o >> 4, lam = o & 15;
    if (lam >= 13) return -1;
    const int d = e == 0 ? c_lines[lam] : 26 - c_lines[lam];
    return d < 13 ? d : d - 1;
}

}  // namespace

// bf16 copies of the weights: W1p[64][64], W2[64][64], W3p[32][64] and the
// transposes used by the backward pass, W2T[64][64], W3T[64][64] (k = output);
// the inference image (W1i, W2i, W3i as MFMA A-operand fragments) and its
// biases (the first layer's per field: the one-hot input's weight folded in).
__global__ void __launch_bounds__(256) mlp_pack(MlpTrain t) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 64 * 64) return;
    const int n = i / 64, k = i % 64;
    t.wb[WB_W1 + i] = bf16_bits(k < IN ? t.par[P_W1 + n * IN + k] : 0.f);
    t.wb[WB_W2 + i] = bf16_bits(t.par[P_W2 + n * HID + k]);
    if (n < 32) t.wb[WB_W3 + i] = bf16_bits(n < OUT ? t.par[P_W3 + n * HID + k] : 0.f);
    // transposes: W2T[h][k2] = W2[k2][h]; W3T[h][o] = W3[o][h] (o < 26, else 0)
    t.wbT[WB_W2T + i] = bf16_bits(t.par[P_W2 + k * HID + n]);
    t.wbT[WB_W3T + i] = bf16_bits(k < OUT ? t.par[P_W3 + k * HID + n] : 0.f);
    // inference image, fragment by fragment (see infer_frag)
    for (int e = i; e < WBI_SIZE; e += 64 * 64) {
        const int F = e >> 9, lane = (e >> 3) & 63, j = e & 7, r = lane & 15, kq = 8 * (lane >> 4) + j;
        float w = 0.f;
        if (F < 4) {                       // W1i, m-tile F
            if (kq < NNB) w = t.par[P_W1 + (16 * F + r) * IN + kq];
        } else if (F < 12) {               // W2i, m-tile (F - 4) / 2, k block (F - 4) % 2
            const int mt = (F - 4) >> 1, kb = (F - 4) & 1;
            w = t.par[P_W2 + (16 * mt + r) * HID + hidden_of(32 * kb + kq)];
        } else {                           // W3i, end (F - 12) / 2, k block (F - 12) % 2
            const int en = (F - 12) >> 1, kb = (F - 12) & 1, o = output_of(16 * en + r);
            if (o >= 0) w = t.par[P_W3 + o * HID + hidden_of(32 * kb + kq)];
        }
        t.wbi[e] = bf16_bits(w);
    }
    if (i < NF * HID) {
        const int f = i / HID, u = i % HID;
        t.bi[BI_B1 + i] = t.par[P_B1 + u] + bf16_float(bf16_bits(t.par[P_W1 + u * IN + NNB + f]));
    }
    if (i < HID) t.bi[BI_B2 + i] = t.par[P_B2 + i];
    if (i < 32) {
        const int o = output_of(i);
        t.bi[BI_B3 + i] = o >= 0 ? t.par[P_B3 + o] : 0.f;
    }
}

// ---------------------------------------------------------------------------
// Inference pre-pass of a stage: every needed cell of every block
// ---------------------------------------------------------------------------

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int ICHUNK = NSLOT / 64;    // 14 workgroups per block, 64 needed cells each
constexpr int BOX = 300;              // 3 x 10 x 10 cells: the neighbourhoods of a chunk

__constant__ int16_t c_pad_ghost[NP];   // padded index -> ghost slot (-1 for interior cells)

__device__ __forceinline__ v4f mfma32(v8bf a, v8bf b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// A-operand fragment F of the inference image for this lane: fragments are
// stored lane by lane (64 x 8 bf16, 1 KB), so a wave reads 1 KB of
// consecutive LDS without bank conflicts.  F 0..3: W1i m-tile F; 4..11: W2i
// m-tile (F-4)/2, k block (F-4)%2; 12..15: W3i end (F-12)/2, k block (F-12)%2.
__device__ __forceinline__ v8bf infer_frag(const uint16_t *W, int F, int lane) {
    return *(const v8bf *)(W + 512 * F + 8 * lane);
}

// The plain limiter and the FP64 check on one line of a row, on its two
// predicted values R (at +d) and L (at -d): each value clamped between the
// cell and its neighbour in that direction, the pair put through the PPM
// monotonicity constraint and kept as binary32 offsets oR, oL from qc (see
// learned_limit), then the point values qc + offset are checked in FP64
// (bounds, positivity of rho, E, tau, non-negative X, the monotonicity
// conditions with a rounding slack of 1e-13 |D| (|L| + |q| + |R|)).  Limiter
// and check only ever couple the two ends of one line, so a row is processed
// line by line.  nbR / nbL are the neighbours in those directions.  Returns
// whether the line passes.  Written without branches: min/max clamps (a NaN
// prediction, which they would turn into a bound, fails explicitly) and
// selects for the constraint's cases.
__device__ __forceinline__ bool limit_check_line(double qc, double nbR, double nbL, int f, double R, double L,
                                                 float &oR, float &oL) {
    bool ok = (R == R) & (L == L);
    const double loR = fmin(qc, nbR), hiR = fmax(qc, nbR);
    const double loL = fmin(qc, nbL), hiL = fmax(qc, nbL);
    learned_limit(qc, nbR, nbL, R, L, oR, oL);
    const double r = qc + (double)oR, l = qc + (double)oL;
    ok = ok & (r >= loR) & (r <= hiR) & (l >= loL) & (l <= hiL);
    if (f == RHO || f == EGAS || f == TAU) ok = ok & (r > 0.0) & (l > 0.0);
    if (f == SPC) ok = ok & (r >= 0.0) & (l >= 0.0);
    {
        const double D = r - l, M6 = 6.0 * (qc - 0.5 * (l + r)), DM = D * M6;
        const double lim = D * D + 1e-13 * fabs(D) * (fabs(l) + fabs(qc) + fabs(r));
        const bool mono = ((r - qc) * (qc - l) > 0.0) & !(DM > lim) & !(DM < -lim);
        ok = ok & (((l == qc) & (r == qc)) | mono);
    }
    return ok;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
    return __shfl_xor(v, m, 64);
}

}  // namespace

// Workgroup (block, chunk): the chunk's 64 needed cells are one 8 x 8 layer of
// cells, normal to axis A at layer Lc (interior layers 0..7 along z, then the
// face-adjacent ghost slabs x-, x+, y-, y+, z-, z+); their 3x3x3
// neighbourhoods fill a 3 x 10 x 10 box, staged in LDS for all seven fields
// (one thread per box cell) next to the inference weight image.  Wave f then
// takes field f: four tiles of 16 cells, each lane group q of a tile computing
// features 8q .. 8q+7 of its cell (sigma and the density contrast combined
// over the group by lane exchange), the three layers on MFMA, and the limiter
// and FP64 check for its lines.  Point values go out as val[block][field]
// [dir][slot]; a cell passes when all seven of its rows pass.
// VAL64: the point values go out in FP64 to m.val (inspection), else as the
// binary32 offsets the stage reads to m.off.
template <bool VAL64>
__global__ void __launch_bounds__(64 * NF) __attribute__((amdgpu_waves_per_eu(7))) mlp_infer_kernel(MlpInfer m) {
    __shared__ double box[NF][BOX];                               // 16,800 B
    __shared__ __attribute__((aligned(16))) uint16_t W[WBI_SIZE];  // 16,384 B
    __shared__ __attribute__((aligned(16))) float bias[BI_SIZE];   //  2,176 B
    __shared__ unsigned long long fails[NF];
    __shared__ int4 otab[4][4];
    __shared__ int shared_s;
    const int item = xcd_leaf(blockIdx.x, gridDim.x);
    const int blk = m.leaf0 + item / ICHUNK, chunk = item % ICHUNK;
    const int tid = threadIdx.x, lane = tid & 63, f = tid >> 6;
    if (!VAL64 && m.alias && chunk >= NX) {
        // a ghost slab whose every cell shares its row with a block of this
        // launch (whose pre-pass computes it as an interior cell) is skipped:
        // the stage reads those rows there
        if (tid < 64) {
            const int al = m.alias[(size_t)blk * (NSLOT - NC) + 64 * (chunk - NX) + tid];
            const int tb = al / NSLOT;
            const bool in = al >= 0 && tb >= m.leaf0 && tb < m.leaf0 + (int)(gridDim.x / ICHUNK);
            const bool all = __all(in);
            if (tid == 0) shared_s = all;
        }
        __syncthreads();
        if (shared_s) return;
    }
    for (int i = tid; i < WBI_SIZE / 8; i += 64 * NF) ((uint4 *)W)[i] = ((const uint4 *)m.wbi)[i];
    for (int i = tid; i < BI_SIZE; i += 64 * NF) bias[i] = m.bi[i];
    // chunk geometry: box origin (o0, o1, o2), extents (d0, d1, 3 or 10)
    const int A = chunk < NX ? 2 : (chunk - NX) >> 1;
    const int Lc = chunk < NX ? chunk : (((chunk - NX) & 1) ? NX : -1);
    const int d0 = A == 0 ? 3 : 10, d1 = A == 1 ? 3 : 10;
    const int o0 = A == 0 ? Lc - 1 : -1, o1 = A == 1 ? Lc - 1 : -1, o2 = A == 2 ? Lc - 1 : -1;
    const int s1 = d0, s2 = d0 * d1;
    {
        const double *Ub = m.U + block_base(blk, m.ts, m.lg);
        const size_t fs = (size_t)1 << (3 * m.lg);
        const int32_t *gm = m.gmap + (size_t)blk * NG;
        for (int c = tid; c < BOX; c += 64 * NF) {
            const int x = o0 + c % d0, y = o1 + (c / d0) % d1, z = o2 + c / s2;
            if (x >= 0 && x < NX && y >= 0 && y < NX && z >= 0 && z < NX) {
                const double *p = Ub + block_cell((z * NX + y) * NX + x, m.lg);
#pragma unroll
                for (int ff = 0; ff < NF; ++ff) box[ff][c] = p[ff * fs];
            } else {
                const int src = gm[c_pad_ghost[((z + GW) * PB + (y + GW)) * PB + (x + GW)]];
#pragma unroll 1
                for (int ff = 0; ff < NF; ++ff)
                    box[ff][c] = ghost_value(m.U, src, ff, m.lg, m.prolong, m.n_prolong);
            }
        }
    }
    __syncthreads();
    const int r = lane & 15, q = lane >> 4;
    // per lane group q: neighbour offsets in the box of features 8q .. 8q+7
    // (k < 27), +d offsets of lines 4q .. 4q+3 and the output rows of their
    // two ends; read in each tile (kept live, they would cost 16 registers)
    if (tid < 4) {
        const int qq = tid;
        int ko[8], lo4[4], lr4[4];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * qq + j < NNB ? 8 * qq + j : 13;
            ko[j] = (k % 3 - 1) + s1 * ((k / 3) % 3 - 1) + s2 * (k / 9 - 1);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int lam = 4 * qq + t < 13 ? 4 * qq + t : 0;
            const int op = c_lines[lam], om = 26 - op;
            lo4[t] = (op % 3 - 1) + s1 * ((op / 3) % 3 - 1) + s2 * (op / 9 - 1);
            lr4[t] = (op < 13 ? op : op - 1) | ((om < 13 ? om : om - 1) << 8);
        }
        otab[qq][0] = int4{ko[0], ko[1], ko[2], ko[3]};
        otab[qq][1] = int4{ko[4], ko[5], ko[6], ko[7]};
        otab[qq][2] = int4{lo4[0], lo4[1], lo4[2], lo4[3]};
        otab[qq][3] = int4{lr4[0], lr4[1], lr4[2], lr4[3]};
    }
    __syncthreads();
    const double *bx = box[f];
    float2 *oout = VAL64 ? nullptr : (float2 *)m.off + ((size_t)blk * NF + f) * 13 * NSLOT;
    double *vout = VAL64 ? m.val + ((size_t)blk * NF + f) * 26 * NSLOT : nullptr;
    unsigned long long wfail = 0;
#pragma unroll 1
    for (int tt = 0; tt < 4; ++tt) {
        const int s = 16 * tt + r, slot = 64 * chunk + s;
        const int u = s & 7, v = s >> 3;
        const int cx = A == 0 ? Lc : u, cy = A == 1 ? Lc : (A == 0 ? u : v), cz = A == 2 ? Lc : v;
        const int cb = (cx - o0) + s1 * (cy - o1) + s2 * (cz - o2);
        const double qc = bx[cb];
        int oz = 0;
        asm volatile("" : "+s"(oz));
        const int4 ka = otab[q + oz][0], kb4 = otab[q + oz][1];
        const int koff[8] = {ka.x, ka.y, ka.z, ka.w, kb4.x, kb4.y, kb4.z, kb4.w};
        double sig = 0.0, lo = qc, hi = qc;
#pragma unroll
        for (int j = 0; j < 8; ++j) {   // (fmax and fmin pass over a NaN)
            const double nvj = bx[cb + koff[j]];
            sig = fmax(sig, fabs(nvj - qc));
            lo = fmin(lo, nvj);
            hi = fmax(hi, nvj);
        }
        // over the row's four lane groups
        sig = fmax(sig, shfl_xor_d(sig, 16));
        sig = fmax(sig, shfl_xor_d(sig, 32));
        const bool flat = !(sig > 0.0);
        if (__all(flat)) {
            // sixteen flat cells (sigma = 0 in this field): every point value
            // is the cell value, exactly, every row passes, and the network
            // is not evaluated
            const int4 lb = otab[q + oz][3];
            const int lrow[4] = {lb.x, lb.y, lb.z, lb.w};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (4 * q + t >= 13) continue;
                if (VAL64) {
                    vout[(size_t)(lrow[t] & 255) * NSLOT + slot] = qc;
                    vout[(size_t)(lrow[t] >> 8) * NSLOT + slot] = qc;
                } else {
                    oout[(size_t)(4 * q + t) * NSLOT + slot] = float2{0.0f, 0.0f};
                }
            }
            continue;
        }
        // the network's error is a few percent of sigma: where the density
        // spans more than a factor 8 over the neighbourhood, the low side's
        // point values (and s / rho from them) would be off by order one
        bool ok = true;
        if (f == RHO) {
            lo = fmin(lo, shfl_xor_d(lo, 16));
            lo = fmin(lo, shfl_xor_d(lo, 32));
            hi = fmax(hi, shfl_xor_d(hi, 16));
            hi = fmax(hi, shfl_xor_d(hi, 32));
            ok = flat || hi <= 8.0 * lo;
        }
        const double rs = flat ? 0.0 : 1.0 / sig;
        asm volatile("" ::: "memory");   // re-read the neighbours rather than keep them live
        v8bf x;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float fv = (flat || 8 * q + j >= NNB) ? 0.f : (float)((bx[cb + koff[j]] - qc) * rs);
            x[j] = (__bf16)fv;
        }
        // an opaque zero offset: the weight and bias fragments are then read
        // from LDS in every tile rather than hoisted out of the loop, where
        // they would hold 104 registers
        int wz = 0;
        asm volatile("" : "+s"(wz));
        const uint16_t *Wt = W + wz;
        const float *bt = bias + wz;
        // layer 1 (K = 32: the 27 neighbourhood features, zero padded)
        v4f z[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            z[mt] = mfma32(infer_frag(Wt, mt, lane), x,
                           *(const v4f *)(bt + BI_B1 + HID * f + 16 * mt + 4 * q));
        v8bf h[2];
#pragma unroll
        for (int j = 0; j < 16; ++j) h[j >> 3][j & 7] = (__bf16)gelu_fast(z[(j >> 3) * 2 + ((j >> 2) & 1)][j & 3]);
        // layer 2
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            v4f c = *(const v4f *)(bt + BI_B2 + 16 * mt + 4 * q);
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                c = mfma32(infer_frag(Wt, 4 + 2 * mt + kb, lane), h[kb], c);
            z[mt] = c;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) h[j >> 3][j & 7] = (__bf16)gelu_fast(z[(j >> 3) * 2 + ((j >> 2) & 1)][j & 3]);
        // output layer: y[e][t] = end e of line 4q + t
        v4f y[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            v4f c = *(const v4f *)(bt + BI_B3 + 16 * e + 4 * q);
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
                c = mfma32(infer_frag(Wt, 12 + 2 * e + kb, lane), h[kb], c);
            y[e] = c;
        }
        // this lane's lines: denormalise, limit, check, store
        const int4 la = otab[q + wz][2], lb = otab[q + wz][3];
        const int loff[4] = {la.x, la.y, la.z, la.w}, lrow[4] = {lb.x, lb.y, lb.z, lb.w};
        float *yr = m.yraw ? m.yraw + (((size_t)blk * NF + f) * NSLOT + slot) * 26 : nullptr;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (4 * q + t >= 13) continue;
            if (yr) {
                yr[lrow[t] & 255] = y[0][t];
                yr[lrow[t] >> 8] = y[1][t];
            }
            float oR = 0.0f, oL = 0.0f;
            if (!flat) {
                const double R = qc + sig * (double)y[0][t];
                const double L = qc + sig * (double)y[1][t];
                ok = limit_check_line(qc, bx[cb + loff[t]], bx[cb - loff[t]], f, R, L, oR, oL) && ok;
            }
            if (VAL64) {
                vout[(size_t)(lrow[t] & 255) * NSLOT + slot] = qc + (double)oR;
                vout[(size_t)(lrow[t] >> 8) * NSLOT + slot] = qc + (double)oL;
            } else {
                oout[(size_t)(4 * q + t) * NSLOT + slot] = float2{oR, oL};
            }
        }
        const unsigned long long bad = __ballot(!ok);
        wfail |= ((bad | (bad >> 16) | (bad >> 32) | (bad >> 48)) & 0xffffull) << (16 * tt);
    }
    if (lane == 0) fails[f] = wfail;
    __syncthreads();
    // verdicts of the chunk's cells, and the count of those that fall back
    if (tid < 64) {
        unsigned long long any = 0;
#pragma unroll
        for (int ff = 0; ff < NF; ++ff) any |= fails[ff];
        const bool bad = (any >> tid) & 1ull;
        m.cell_ok[(size_t)blk * NSLOT + 64 * chunk + tid] = bad ? 0 : 1;
        // statistics count each block's interior cells (a ghost-slab cell is
        // counted in the block it belongs to)
        if (tid == 0 && any && chunk < NX) atomicAdd(m.fb_count, (unsigned long long)__popcll(any));
    }
}

hipError_t hydro_mlp_upload_pad_ghost(const int16_t *pad_ghost) {
    return hipMemcpyToSymbol(HIP_SYMBOL(c_pad_ghost), pad_ghost, sizeof(int16_t) * NP);
}

hipError_t hydro_mlp_launch_infer(const MlpInfer &m, int nleaf, hipStream_t s) {
    if (nleaf <= 0) return hipSuccess;
    if (m.val)
        hipLaunchKernelGGL(mlp_infer_kernel<true>, dim3(nleaf * ICHUNK), dim3(64 * NF), 0, s, m);
    else
        hipLaunchKernelGGL(mlp_infer_kernel<false>, dim3(nleaf * ICHUNK), dim3(64 * NF), 0, s, m);
    return hipGetLastError();
}

hipError_t hydro_mlp_launch_pack(const MlpTrain &t, hipStream_t s) {
    hipLaunchKernelGGL(mlp_pack, dim3(16), dim3(256), 0, s, t);
    return hipGetLastError();
}

hipError_t hydro_mlp_launch_forward(const MlpTrain &t, const float *X, int B, hipStream_t s) {
    const int waves = (B + 63) / 64;
    hipLaunchKernelGGL(mlp_train_forward, dim3((waves + 3) / 4), dim3(256), 0, s, t, X, B);
    return hipGetLastError();
}

hipError_t hydro_mlp_launch_grad(const MlpTrain &t, const float *T, int B, float *loss, hipStream_t s) {
    const int waves = (B + 63) / 64;
    hipLaunchKernelGGL(mlp_train_backward_rows, dim3((waves + 3) / 4), dim3(256), 0, s, t, T, B);
    hipLaunchKernelGGL(mlp_train_wgrad, dim3(WG_TILES * WG_SLICES), dim3(64), 0, s, t, B);
    hipLaunchKernelGGL(mlp_grad_reduce, dim3((NPAR + 255) / 256), dim3(256), 0, s, t);
    if (loss) hipLaunchKernelGGL(mlp_loss_reduce, dim3(1), dim3(64), 0, s, t, B, loss);
    return hipGetLastError();
}

hipError_t hydro_mlp_launch_adam(const MlpTrain &t, float lr, float b1, float b2, float eps, float c1,
                                 float c2, hipStream_t s) {
    hipLaunchKernelGGL(mlp_adam, dim3((NPAR + 255) / 256), dim3(256), 0, s, t, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}
