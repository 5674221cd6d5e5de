// Neural-field device routines (gfx950): a Fourier-feature MLP evaluated by
// whole waves with bf16 MFMA (v_mfma_f32_32x32x16_bf16, FP32 accumulation).
//
// Network: xhat = frac((x - origin) / (n * spacing)); features
// [cos 2pi F xhat, sin 2pi F xhat] (F: 64 integer vectors); four 128-wide ReLU
// layers; a linear 3-output layer; B = b_scale * out.
//
// Wave layout.  A wave evaluates 64 points (its 64 lanes' points) as two
// 32-column blocks.  Layer activations are the MFMA B operand: for column
// block cb, lane l (group g = l / 32) holds, for point 32 cb + l % 32, the
// features 16 m + 8 g + j (k-block m = 0..7, j = 0..7) as eight bf16x8.
// Weight rows inside each 32-row tile are stored permuted (lambda below), so
// that the accumulator registers of one layer are exactly the next layer's
// B operand: no data movement between layers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int NF_WIDTH = 128;
constexpr int NF_FEAT = 64;
constexpr int NF_LAYER_PARAMS = NF_WIDTH * NF_WIDTH + NF_WIDTH;  // 16512
constexpr int NF_W5 = 4 * NF_LAYER_PARAMS;                        // 66048
constexpr int NF_B5 = NF_W5 + 3 * NF_WIDTH;                       // 66432
constexpr int NF_NPARAM = NF_B5 + 3;                              // 66435

// LDS image of the network (bf16 weights, FP32 biases, FP32 frequencies).
constexpr int NF_IMG_LAYER = NF_WIDTH * NF_WIDTH;     // bf16 elements per layer
constexpr size_t NF_LDS_BYTES = 4 * NF_IMG_LAYER * 2   // W1..W4 images
                                + 3 * NF_WIDTH * 2      // W5 (bf16)
                                + (4 * NF_WIDTH + 4) * 4  // biases (+pad)
                                + NF_FEAT * 3 * 4;        // frequencies

// Physical MFMA row rho of a 32-row tile holds logical row lambda(rho):
// rho = 8 (i / 4) + 4 g + (i % 4)  <->  lambda = 16 (i / 8) + 8 g + (i % 8).
__host__ __device__ inline int nf_lambda(int rho)
{
    const int g = (rho >> 2) & 1;
    const int i = ((rho >> 3) << 2) | (rho & 3);
    return 16 * (i >> 3) + 8 * g + (i & 7);
}

// Element offset of (row, col) in a 128x128 image: 16-byte chunks XOR-swizzled
// by the row so that the 32 rows read by one MFMA operand load fall on
// different LDS banks.
__host__ __device__ inline int nf_img_off(int row, int col)
{
    const int chunk = (col >> 3) ^ (row & 15);
    return row * NF_WIDTH + chunk * 8 + (col & 7);
}

struct NFView {
    const __bf16* w[4];     // LDS images of layers 1..4
    const __bf16* w5;       // LDS [3][128]
    const float* bias;      // LDS [4][128] then b5[3]
    const float* freq;      // LDS [64][3]
    double origin[3];
    double inv_box[3];      // 1 / (n_a * spacing)
    float b_scale;
};

// Carves the LDS image (layout of NF_LDS_BYTES) starting at `base`.
__device__ __attribute__((always_inline)) inline NFView nf_view_lds(char* base, const double origin[3], const double inv_box[3],
                                     float b_scale)
{
    NFView v;
    __bf16* w = (__bf16*)base;
    for (int k = 0; k < 4; ++k)
        v.w[k] = w + k * NF_IMG_LAYER;
    v.w5 = w + 4 * NF_IMG_LAYER;
    float* f = (float*)(base + 4 * NF_IMG_LAYER * 2 + 3 * NF_WIDTH * 2);
    v.bias = f;
    v.freq = f + 4 * NF_WIDTH + 4;
    for (int a = 0; a < 3; ++a) {
        v.origin[a] = origin[a];
        v.inv_box[a] = inv_box[a];
    }
    v.b_scale = b_scale;
    return v;
}

// Cooperative copy of the global network image (same layout) into LDS, eight
// 16-byte loads of a thread in flight before their LDS writes (one at a time,
// each write would wait for its load: ~33 memory latencies per block).
__device__ __attribute__((always_inline)) inline void nf_stage_lds(char* dst, const char* src)
{
    constexpr int U = 8;   // loads in flight per thread
    const int4* s = (const int4*)src;
    int4* d = (int4*)dst;
    const int n16 = (int)(NF_LDS_BYTES / 16);
    const int nt = (int)blockDim.x;
    int i = (int)threadIdx.x;
    for (; i + (U - 1) * nt < n16; i += U * nt) {
        // eight named registers (an array here was kept in scratch memory)
        const int4 v0 = s[i], v1 = s[i + nt], v2 = s[i + 2 * nt], v3 = s[i + 3 * nt];
        const int4 v4 = s[i + 4 * nt], v5 = s[i + 5 * nt], v6 = s[i + 6 * nt],
                   v7 = s[i + 7 * nt];
        d[i] = v0;
        d[i + nt] = v1;
        d[i + 2 * nt] = v2;
        d[i + 3 * nt] = v3;
        d[i + 4 * nt] = v4;
        d[i + 5 * nt] = v5;
        d[i + 6 * nt] = v6;
        d[i + 7 * nt] = v7;
    }
    for (; i < n16; i += nt)
        d[i] = s[i];
}

// ReLU as a 32-bit integer maximum with 0: a float is negative exactly when
// its sign bit is set, i.e. when it is negative as an int32 (-0 included), and
// non-negative floats order alike, so this is max(v, 0) in one instruction
// (a floating-point maximum would be preceded by a canonicalisation).
__device__ __attribute__((always_inline)) inline float nf_relu(float v)
{
    return __int_as_float(max(__float_as_int(v), 0));
}

// Hides an LDS pointer's value from the optimiser: inside persistent loops
// the weight loads must stay next to their MFMAs instead of being hoisted out
// of the loop (which would need hundreds of registers).
// The pointer is hidden as its 32-bit LDS address and turned back into a
// pointer from the LDS address space, so that the loads through it remain LDS
// loads (a laundered generic pointer would turn them into flat loads, each
// waited for on its own).
template <class T>
__device__ __attribute__((always_inline)) inline const T* nf_launder(const T* p)
{
    typedef const __attribute__((address_space(3))) T* lds_ptr;
    uint32_t a = (uint32_t)(uintptr_t)(lds_ptr)p;
    asm volatile("" : "+s"(a));
    return (const T*)(lds_ptr)(uintptr_t)a;
}

// Fourier features of one point (this lane's half: group g) as B operand.
__device__ __attribute__((always_inline)) inline void nf_embed(const float* freq, float x0, float x1, float x2, int g,
                                bf16x8 act[8])
{
    freq = nf_launder(freq);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int jj = 16 * m + 8 * g + j;
            // fused: the phases only feed bf16 features
            const float ang = __builtin_fmaf(
                freq[3 * jj + 2], x2, __builtin_fmaf(freq[3 * jj + 1], x1, freq[3 * jj] * x0));
            act[m][j] = (__bf16)__builtin_amdgcn_cosf(ang);       // cos 2 pi ang
            act[m + 4][j] = (__bf16)__builtin_amdgcn_sinf(ang);   // sin 2 pi ang
        }
    }
}

// Fourier features for training, in FP64: the phase F . xhat (integer F, FP32
// xhat: each product exact in FP64) reduced to its fraction in [0, 1) (exact),
// cos and sin of 2 pi times it by the FP64 library (sincospi), then rounded to
// bf16.  The features are then within an FP64 rounding of their exact values,
// so their bf16 roundings are those of the exact features (the stepper's
// FP32 phase and hardware sin / cos above move a feature by up to ~1e-5).
__device__ __attribute__((always_inline)) inline void nf_embed_fp64(const float* freq, float x0,
                                                                     float x1, float x2, int g,
                                                                     bf16x8 act[8])
{
    freq = nf_launder(freq);
    const double d0 = x0, d1 = x1, d2 = x2;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int jj = 16 * m + 8 * g + j;
            double ph = ((double)freq[3 * jj] * d0 + (double)freq[3 * jj + 1] * d1) +
                        (double)freq[3 * jj + 2] * d2;
            ph = ph - floor(ph);
            double sv, cv;
            sincospi(2.0 * ph, &sv, &cv);
            act[m][j] = (__bf16)cv;
            act[m + 4][j] = (__bf16)sv;
        }
    }
}

// One hidden layer for the two column blocks: out = relu(W in + b) as bf16.
// If store_pre is given, it receives the activation (bf16) for later use.
__device__ __attribute__((always_inline)) inline void nf_layer(const __bf16* wimg, const float* bias, const bf16x8 in[2][8],
                                bf16x8 out[2][8])
{
    wimg = nf_launder(wimg);
    bias = nf_launder(bias);
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int rr = lane & 31;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        // the accumulators start from the biases: the epilogue is ReLU and
        // the bf16 conversion only
        floatx16 acc0, acc1;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float b = bias[32 * r + 16 * (i >> 3) + 8 * g + (i & 7)];
            acc0[i] = b;
            acc1[i] = b;
        }
        const int row = 32 * r + rr;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const bf16x8 a = *(const bf16x8*)(wimg + nf_img_off(row, 16 * m + 8 * g));
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, in[0][m], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, in[1][m], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            out[0][2 * r + (i >> 3)][i & 7] = (__bf16)nf_relu(acc0[i]);
            out[1][2 * r + (i >> 3)][i & 7] = (__bf16)nf_relu(acc1[i]);
        }
    }
}

// Output layer on the matrix cores: W5 (3 x 128) is the A operand of a
// 32-row tile whose rows 3..31 are zero, so rows 0..2 of the result (the three
// outputs) land in registers 0..2 of lanes 0..31 for the 32 points of each
// column block.  Every lane returns the outputs of its own point (lanes 0..31:
// column block 0, 32..63: block 1, moved across by a lane swap).
__device__ __attribute__((always_inline)) inline void nf_output(const __bf16* w5, const float* b5, const bf16x8 h[2][8],
                                 float out[3])
{
    w5 = nf_launder(w5);
    b5 = nf_launder(b5);
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int row = lane & 31;
    const bool live = row < 3;
    const __bf16* wrow = w5 + (live ? row : 0) * NF_WIDTH + 8 * g;
    floatx16 acc0 = {}, acc1 = {};
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        bf16x8 a = *(const bf16x8*)(wrow + 16 * m);
        if (!live)
            a = bf16x8{};
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, h[0][m], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, h[1][m], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float other = __shfl_xor(acc1[c], 32);
        out[c] = (g == 0 ? acc0[c] : other) + b5[c];
    }
}

// One hidden layer for one column block: out = relu(W in + b) as bf16.
__device__ __forceinline__ void nf_layer1(const __bf16* wimg, const float* bias,
                                          const bf16x8 in[8], bf16x8 out[8])
{
    wimg = nf_launder(wimg);
    bias = nf_launder(bias);
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int rr = lane & 31;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        floatx16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            acc[i] = bias[32 * r + 16 * (i >> 3) + 8 * g + (i & 7)];
        const int row = 32 * r + rr;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const bf16x8 a = *(const bf16x8*)(wimg + nf_img_off(row, 16 * m + 8 * g));
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, in[m], acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            out[2 * r + (i >> 3)][i & 7] = (__bf16)nf_relu(acc[i]);
    }
}

// Output layer for one column block: lanes 0..31 receive the three outputs of
// their point (rows 0..2 of the result, registers 0..2 of group 0).
__device__ __forceinline__ void nf_output1(const __bf16* w5, const float* b5, const bf16x8 h[8],
                                           float out[3])
{
    w5 = nf_launder(w5);
    b5 = nf_launder(b5);
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int row = lane & 31;
    const bool live = row < 3;
    const __bf16* wrow = w5 + (live ? row : 0) * NF_WIDTH + 8 * g;
    floatx16 acc = {};
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        bf16x8 a = *(const bf16x8*)(wrow + 16 * m);
        if (!live)
            a = bf16x8{};
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, h[m], acc, 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        out[c] = acc[c] + b5[c];
}

// Normalised position of a point in [0, 1)^3 (FP64, then FP32).
__device__ __attribute__((always_inline)) inline void nf_xhat(const NFView& v, const double x[3], float xh[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double f = (x[a] - v.origin[a]) * v.inv_box[a];
        xh[a] = (float)(f - floor(f));
    }
}

// Whole-wave evaluation: every lane passes its own point and receives its
// own network output (all 64 lanes must call together).
__device__ __attribute__((always_inline)) inline void nf_eval_wave(const NFView& v, const float xh[3], float out[3])
{
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    bf16x8 a[2][8], b[2][8];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int src = 32 * cb + (lane & 31);
        const float x0 = __shfl(xh[0], src), x1 = __shfl(xh[1], src), x2 = __shfl(xh[2], src);
        nf_embed(v.freq, x0, x1, x2, g, a[cb]);
    }
    nf_layer(v.w[0], v.bias, a, b);
    nf_layer(v.w[1], v.bias + NF_WIDTH, b, a);
    nf_layer(v.w[2], v.bias + 2 * NF_WIDTH, a, b);
    nf_layer(v.w[3], v.bias + 3 * NF_WIDTH, b, a);
    nf_output(v.w5, v.bias + 4 * NF_WIDTH, a, out);
}

// Field source for the stepper: the trained network (precision form only;
// the whole wave takes part in every evaluation).
struct NeuralFieldSrc {
    NFView v;
    // the whole wave evaluates the network together, so `need` saves nothing
    __device__ inline void fp32(const double p[3], float B[3], bool need = true) const
    {
        (void)need;
        float xh[3], o[3];
        nf_xhat(v, p, xh);
        nf_eval_wave(v, xh, o);
        B[0] = v.b_scale * o[0];
        B[1] = v.b_scale * o[1];
        B[2] = v.b_scale * o[2];
    }
    __device__ inline void fp64(const double p[3], double B[3], bool need = true) const
    {
        float b[3];
        fp32(p, b, need);
        B[0] = b[0];
        B[1] = b[1];
        B[2] = b[2];
    }
};

}  // namespace crp
