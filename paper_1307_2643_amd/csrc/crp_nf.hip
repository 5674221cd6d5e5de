// Neural-field kernels and host side of libcrp: packing of the bf16 weight
// images, whole-wave MFMA evaluation, training (sampling, forward with stored
// activations, backward, weight and bias gradients, Adam).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "crp_nf.hpp"
#include "crp_nf_device.hpp"

namespace crp {

// -------------------------------------------------------------------------
// Device kernels.
// -------------------------------------------------------------------------

// Logical row of physical row R of a 128-row weight image.
__device__ inline int nf_logical_row(int R) { return 32 * (R >> 5) + nf_lambda(R & 31); }

// Builds the forward image (W_k rows permuted) and the backward image (W_k^T
// rows permuted) plus W5, biases and frequencies from the FP32 masters.
__global__ void k_nf_pack(const float* master, const int32_t* freq, char* fwd, char* bwd)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    __bf16* wf = (__bf16*)fwd;
    __bf16* wb = (__bf16*)bwd;
    if (i < 4 * NF_IMG_LAYER) {
        const int k = i / NF_IMG_LAYER, e = i % NF_IMG_LAYER;
        const int R = e / NF_WIDTH, c = e % NF_WIDTH;
        const float* W = master + k * NF_LAYER_PARAMS;
        const int lr = nf_logical_row(R);
        wf[k * NF_IMG_LAYER + nf_img_off(R, c)] = (__bf16)W[lr * NF_WIDTH + c];
        wb[k * NF_IMG_LAYER + nf_img_off(R, c)] = (__bf16)W[c * NF_WIDTH + lr];
        return;
    }
    int j = i - 4 * NF_IMG_LAYER;
    if (j < 3 * NF_WIDTH) {
        const __bf16 v = (__bf16)master[NF_W5 + j];
        wf[4 * NF_IMG_LAYER + j] = v;
        wb[4 * NF_IMG_LAYER + j] = v;
        return;
    }
    j -= 3 * NF_WIDTH;
    float* bf = (float*)(fwd + 4 * NF_IMG_LAYER * 2 + 3 * NF_WIDTH * 2);
    float* bb = (float*)(bwd + 4 * NF_IMG_LAYER * 2 + 3 * NF_WIDTH * 2);
    if (j < 4 * NF_WIDTH + 4) {
        float v = 0.0f;
        if (j < 4 * NF_WIDTH)
            v = master[(j / NF_WIDTH) * NF_LAYER_PARAMS + NF_WIDTH * NF_WIDTH + (j % NF_WIDTH)];
        else if (j < 4 * NF_WIDTH + 3)
            v = master[NF_B5 + (j - 4 * NF_WIDTH)];
        bf[j] = v;
        bb[j] = v;
        return;
    }
    j -= 4 * NF_WIDTH + 4;
    if (j < 3 * NF_FEAT) {
        bf[4 * NF_WIDTH + 4 + j] = (float)freq[j];
        bb[4 * NF_WIDTH + 4 + j] = (float)freq[j];
    }
}

struct NFGeom {
    double origin[3];
    double inv_box[3];
    double box[3];
    float b_scale;
};

__device__ inline NFView nf_view(char* lds, const NFGeom& G)
{
    return nf_view_lds(lds, G.origin, G.inv_box, G.b_scale);
}

// Field of the network at n positions (whole waves; lanes past n evaluate a
// copy of the last point and write nothing).
__global__ void __launch_bounds__(256) k_nf_eval(const char* img, NFGeom G, int64_t n,
                                                 const double* pos, double* B)
{
    extern __shared__ __attribute__((aligned(16))) char nf_lds[];
    nf_stage_lds(nf_lds, img);
    __syncthreads();
    const NFView v = nf_view(nf_lds, G);
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        const int64_t i = base + lane < n ? base + lane : n - 1;
        const double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        float xh[3], o[3];
        nf_xhat(v, p, xh);
        nf_eval_wave(v, xh, o);
        if (base + lane < n) {
            B[3 * i] = (double)(v.b_scale * o[0]);
            B[3 * i + 1] = (double)(v.b_scale * o[1]);
            B[3 * i + 2] = (double)(v.b_scale * o[2]);
        }
    }
}

// Normalised positions of caller-given points.
__global__ void k_nf_xhat(NFGeom G, int64_t n, const double* pos, float* xh)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    for (int a = 0; a < 3; ++a) {
        const double f = (pos[3 * i + a] - G.origin[a]) * G.inv_box[a];
        xh[3 * i + a] = (float)(f - floor(f));
    }
}

// Training samples: uniform points in one period of the grid (Philox draws
// keyed by the run seed and the sample's index) as xhat (FP32) and position,
// then the grid's trilinear field there (FP32 weights and sums) in units of
// b_scale.
__device__ __forceinline__ void nf_sample_xhat(const NFGeom& G, uint64_t seed, uint64_t idx,
                                               float xh[3], double p[3])
{
    const U64x4 w = philox4x64_10(idx, 0, 0, 0, seed, 0x4e46u);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = (double)(w.w[a] >> 11) * 0x1p-53;
        xh[a] = (float)u;
        p[a] = G.origin[a] + u * G.box[a];
    }
}

__device__ __forceinline__ void nf_sample_target(const GridView& g, const NFGeom& G,
                                                 const double p[3], float tgt[3])
{
    const GridField<float, 0> F{g};
    float B[3];
    F.fp32(p, B);
    const float inv = 1.0f / G.b_scale;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        tgt[c] = B[c] * inv;
}

// -------------------------------------------------------------------------
// Training buffers in tile order.
//
// The weight gradients contract over the points, so they read each feature's
// values of consecutive points side by side, while a layer holds one point's
// features per lane.  The training kernels therefore keep activations and
// gradients by 32-point tiles: in a buffer layer [tile][128 features][32],
// feature f of tile T holds its 32 points as consecutive values, point p of
// the tile at position nf_tile_pos(p) = 16 g + i for p = 8 (i / 4) + 4 g +
// i % 4 -- the row order of an MFMA 32x32 result, so that a lane writes its
// 16 values of a transposed tile as 32 consecutive bytes.  The tiles are
// transposed on the matrix cores: an MFMA whose B operand is an identity
// moves activations from the operand layout (lane = point) to the result
// layout (lane = feature) exactly (products with 1, sums with 0).
// -------------------------------------------------------------------------
__device__ __forceinline__ int nf_tile_pos(int p)
{
    return 16 * ((p >> 2) & 1) + ((p >> 3) << 2) + (p & 3);
}

// Identity B operands of the transposes: lane (column c, group g) holds
// K = 8 g + j; `lo` selects K = c (columns 0..15), `hi` K = c - 16 (16..31).
__device__ __forceinline__ void nf_ident(bf16x8& lo, bf16x8& hi)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int c = lane & 31, k0 = 8 * (lane >> 5);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        lo[j] = (__bf16)(k0 + j == c ? 1.0f : 0.0f);
        hi[j] = (__bf16)(k0 + j == c - 16 ? 1.0f : 0.0f);
    }
}

// Transpose of k-blocks 2q and 2q + 1 of one column block: lane (c, g)
// receives feature 32 q + c of the tile positions 16 g + i, i = 0..15.
__device__ __forceinline__ floatx16 nf_transpose(const bf16x8& x0, const bf16x8& x1,
                                                 const bf16x8& lo, const bf16x8& hi)
{
    floatx16 t = {};
    t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, lo, t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, hi, t, 0, 0, 0);
    return t;
}

// Writes a transposed tile of bf16 values (exact in FP32) as 32 bytes.
__device__ __forceinline__ void nf_store_tile(__bf16* dst, const floatx16& t)
{
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)t[i];
        b[i] = (__bf16)t[8 + i];
    }
    *(bf16x8*)dst = a;
    *(bf16x8*)(dst + 8) = b;
}

// Positive-activation bits of eight non-negative bf16 values (bit j: value
// j > 0).  A 15-bit half is non-zero exactly when adding 0x7fff sets its top
// bit, and no carry crosses into the next half.
__device__ __forceinline__ uint32_t nf_nz8(const bf16x8& v)
{
    uint32_t w[4];
    __builtin_memcpy(w, &v, 16);
    uint32_t b = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        b |= ((w[t] + 0x7fff7fffu) & 0x80008000u) >> (15 - 2 * t);
    return (b | (b >> 15)) & 0xffu;
}

// ReLU pattern of a lane's 64 activations of one column block: bit 8 m + j
// of word m / 4 (m mod 4 in place of m) for feature 16 m + 8 g + j.
__device__ __forceinline__ uint2 nf_relu_bits(const bf16x8 h[8])
{
    uint2 r;
    r.x = nf_nz8(h[0]) | nf_nz8(h[1]) << 8 | nf_nz8(h[2]) << 16 | nf_nz8(h[3]) << 24;
    r.y = nf_nz8(h[4]) | nf_nz8(h[5]) << 8 | nf_nz8(h[6]) << 16 | nf_nz8(h[7]) << 24;
    return r;
}

__device__ __forceinline__ bool nf_on(const uint2 mk, int m, int j)
{
    return (((m < 4 ? mk.x : mk.y) >> (8 * (m & 3) + j)) & 1u) != 0;
}

constexpr int NF_DBP = 4 * NF_WIDTH + 4;     // per-tile bias sums: dZ_1..dZ_4, dOut, pad

// The training forward gives each wave one 32-point tile (a column block of
// the MFMA layout) and runs 512-thread blocks: one block per CU (the network
// image fills the LDS) but two waves per SIMD, whose latencies then hide
// behind each other's work.  (The backward, whose MFMA chains are denser,
// measured faster with two column blocks per wave sharing each weight load,
// as in the stepper's whole-wave evaluation.)
constexpr int NF_TRAIN_BLOCK = 512;

// Training forward, one 32-point tile per wave (points past n repeat point
// n - 1): the outputs, the input of every layer in tile order (acts: five
// layers of [tile][128][32] bf16) and the ReLU pattern of the four hidden
// outputs (relu: [4][tile][64 lanes]) for the backward.  The points are the
// caller's (xh) or, with `sample`, drawn here (indices offset.. of the Philox
// stream seed) with their targets (tgt) from the grid, read after the network
// so that the gathers' latency is hidden behind it.
__global__ void __launch_bounds__(NF_TRAIN_BLOCK) k_nf_fwd(const char* img, NFGeom G, int64_t n,
                                                           int64_t ld, const float* xh,
                                                           bool sample, GridView grid,
                                                           uint64_t seed, uint64_t offset,
                                                           float* tgt, __bf16* acts, uint2* relu,
                                                           float* out)
{
    extern __shared__ __attribute__((aligned(16))) char nf_lds[];
    nf_stage_lds(nf_lds, img);
    __syncthreads();
    const NFView v = nf_view(nf_lds, G);
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int rr = lane & 31;
    const int64_t ntile = ld >> 5;
    bf16x8 Ilo, Ihi;
    nf_ident(Ilo, Ihi);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t T = wave; T * 32 < n; T += nwaves) {
        const int64_t p = T * 32 + rr;              // this lane's point (both groups)
        const int64_t q = p < n ? p : n - 1;
        float x0, x1, x2;
        double sp[3] = {0.0, 0.0, 0.0};
        if (sample) {
            float sx[3];
            nf_sample_xhat(G, seed, offset + (uint64_t)q, sx, sp);
            x0 = sx[0];
            x1 = sx[1];
            x2 = sx[2];
        } else {
            x0 = xh[3 * q];
            x1 = xh[3 * q + 1];
            x2 = xh[3 * q + 2];
        }
        bf16x8 a[8], b[8];
        nf_embed_fp64(v.freq, x0, x1, x2, g, a);
        auto keep = [&](int L, const bf16x8 h[8]) {
            __bf16* dst = acts + (int64_t)L * NF_WIDTH * ld;
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const floatx16 t = nf_transpose(h[2 * qq], h[2 * qq + 1], Ilo, Ihi);
                nf_store_tile(dst + (T * NF_WIDTH + 32 * qq + rr) * 32 + 16 * g, t);
            }
            if (L > 0)
                relu[((int64_t)(L - 1) * ntile + T) * 64 + lane] = nf_relu_bits(h);
        };
        keep(0, a);
        nf_layer1(v.w[0], v.bias, a, b);
        keep(1, b);
        nf_layer1(v.w[1], v.bias + NF_WIDTH, b, a);
        keep(2, a);
        nf_layer1(v.w[2], v.bias + 2 * NF_WIDTH, a, b);
        keep(3, b);
        nf_layer1(v.w[3], v.bias + 3 * NF_WIDTH, b, a);
        keep(4, a);
        float o[3];
        nf_output1(v.w5, v.bias + 4 * NF_WIDTH, a, o);
        if (g == 0 && p < n) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                out[3 * p + c] = o[c];
            if (sample) {
                float t[3];
                nf_sample_target(grid, G, sp, t);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    tgt[3 * p + c] = t[c];
            }
        }
    }
}

// Training backward: dOut = 2 (out - target) / n (FP32; zero past n); dH4 =
// W5^T bf16(dOut) on the vector ALU; dZ_k = dH_k where h_k > 0; dH_{k-1} =
// W_k^T bf16(dZ_k) by MFMA with the transposed images.  For the weight
// gradients it stores bf16(dZ_k) in tile order (dz: four layers of
// [tile][128][32]) and dOut in tile order (dout: [tile][3][32], FP32); for the
// bias gradients, each tile's sums over its 32 points (dbp: [tile][NF_DBP],
// dZ_1..dZ_4 by 128 features, then the three outputs).  Two tiles per wave:
// its 64 lanes hold one point each for dOut, and two column blocks in the
// layers, so that each weight load from LDS feeds two MFMAs.  The sums take dZ as
// bf16(dZ) + bf16(dZ - bf16(dZ)), within 2^-17 of the FP32 value, both parts
// transposed exactly on the matrix cores.  Adds the loss mean_p |out - tgt|^2
// (FP64; one atomic per wave) to *loss.
__global__ void __launch_bounds__(256) k_nf_bwd(const char* img_t, NFGeom G, int64_t n,
                                                int64_t ld, const float* out, const float* tgt,
                                                const uint2* relu, __bf16* dz, float* dout,
                                                float* dbp, double* loss, float inv_n)
{
    extern __shared__ __attribute__((aligned(16))) char nf_lds[];
    nf_stage_lds(nf_lds, img_t);
    __syncthreads();
    const NFView v = nf_view(nf_lds, G);
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int rr = lane & 31;
    const int64_t ntile = ld >> 5;
    bf16x8 Ilo, Ihi;
    nf_ident(Ilo, Ihi);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        const int64_t T0 = base >> 5;
        // dOut of this lane's own point, in tile order, and its wave sums
        float d[3] = {0.f, 0.f, 0.f}, dr[3] = {0.f, 0.f, 0.f};
        double sq = 0.0;
        const int64_t me = base + lane;
        if (me < n) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float oc = out[3 * me + c], tc = tgt[3 * me + c];
                d[c] = 2.0f * (oc - tc) * inv_n;
                dr[c] = (float)(__bf16)d[c];
                const double e = (double)oc - (double)tc;
                sq += e * e;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            sq += __shfl_xor(sq, o);
        if (lane == 0)
            atomicAdd(loss, sq / (double)n);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dout[((T0 + g) * 3 + c) * 32 + nf_tile_pos(rr)] = d[c];
            float s = d[c];
#pragma unroll
            for (int o = 16; o >= 1; o >>= 1)
                s += __shfl_xor(s, o);
            if (rr == 0)
                dbp[(T0 + g) * NF_DBP + 4 * NF_WIDTH + c] = s;    // tile T0 + g
        }
        // one hidden layer's gradient tile (k-blocks 2q, 2q + 1 of column
        // block cb, FP32 values s[16] in result order) kept for the weight and
        // bias gradients
        auto keep = [&](int k, int cb, int q, const bf16x8& h0, const bf16x8& h1,
                        const bf16x8& l0, const bf16x8& l1) {
            const floatx16 th = nf_transpose(h0, h1, Ilo, Ihi);
            const floatx16 tl = nf_transpose(l0, l1, Ilo, Ihi);
            nf_store_tile(dz + (int64_t)k * NF_WIDTH * ld +
                              ((T0 + cb) * NF_WIDTH + 32 * q + rr) * 32 + 16 * g,
                          th);
            float s = 0.0f;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                s += th[i] + tl[i];
            s += __shfl_xor(s, 32);
            if (g == 0)
                dbp[(T0 + cb) * NF_DBP + k * NF_WIDTH + 32 * q + rr] = s;
        };
        bf16x8 dzb[2][8];
        // layer 4: dH4 = W5^T dOut on the vector ALU, then the ReLU mask
        {
            const __bf16* w5 = nf_launder(v.w5);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const int src = 32 * cb + rr;
                const float d0 = __shfl(dr[0], src), d1 = __shfl(dr[1], src),
                            d2 = __shfl(dr[2], src);
                const uint2 mk = relu[((int64_t)3 * ntile + T0 + cb) * 64 + lane];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bf16x8 lo[2];
#pragma unroll
                    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int m = 2 * q + mm;
                            const int f = 16 * m + 8 * g + j;
                            float s = ((float)w5[f] * d0 + (float)w5[NF_WIDTH + f] * d1) +
                                      (float)w5[2 * NF_WIDTH + f] * d2;
                            s = nf_on(mk, m, j) ? s : 0.0f;
                            const __bf16 h = (__bf16)s;
                            dzb[cb][m][j] = h;
                            lo[mm][j] = (__bf16)(s - (float)h);
                        }
                    keep(3, cb, q, dzb[cb][2 * q], dzb[cb][2 * q + 1], lo[0], lo[1]);
                }
            }
        }
        // layers 4 -> 1: dH_{k-1} = W_k^T dZ_k, mask with h_{k-1} > 0
#pragma unroll 1
        for (int k = 3; k >= 1; --k) {
            const __bf16* wimg = nf_launder(v.w[0] + k * NF_IMG_LAYER);
            const uint2 mk0 = relu[((int64_t)(k - 1) * ntile + T0) * 64 + lane];
            const uint2 mk1 = relu[((int64_t)(k - 1) * ntile + T0 + 1) * 64 + lane];
            bf16x8 nxt[2][8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                floatx16 acc0 = {}, acc1 = {};
                const int row = 32 * r + rr;
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const bf16x8 a = *(const bf16x8*)(wimg + nf_img_off(row, 16 * m + 8 * g));
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, dzb[0][m], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, dzb[1][m], acc1, 0, 0, 0);
                }
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    bf16x8 lo[2];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int m = 2 * r + (i >> 3), j = i & 7;
                        float s = cb == 0 ? acc0[i] : acc1[i];
                        s = nf_on(cb == 0 ? mk0 : mk1, m, j) ? s : 0.0f;
                        const __bf16 h = (__bf16)s;
                        nxt[cb][m][j] = h;
                        lo[i >> 3][j] = (__bf16)(s - (float)h);
                    }
                    keep(k - 1, cb, r, nxt[cb][2 * r], nxt[cb][2 * r + 1], lo[0], lo[1]);
                }
            }
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int m = 0; m < 8; ++m)
                    dzb[cb][m] = nxt[cb][m];
        }
    }
}

// Sum of n values p[0], p[stride], ... in index order, eight loads in flight.
__device__ __forceinline__ float nf_sum_strided(const float* p, int64_t stride, int n)
{
    float s = 0.0f;
    int c = 0;
    for (; c + 8 <= n; c += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = p[(int64_t)(c + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            s += v[u];
    }
    for (; c < n; ++c)
        s += p[(int64_t)c * stride];
    return s;
}

// Weight and bias gradients of all five layers in one launch, split over the
// points: block (chunk c, layer L) forms the partial sums over the tiles
// [t0, t1) of its chunk
//   dW_L[o][i] = sum_p bf16(g_L[o][p]) a_L[i][p],   db_L[o] = sum_p g_L[o][p]
// with g_L the gradient at layer L's output (g_4: dOut, 3 rows) and a_L its
// bf16 input, both in tile order, and writes them to part[c][L]
// (NF_PART_LAYER floats per layer: dW row-major, then db; db from the
// backward's per-tile sums).  MFMA 32x32x16 bf16: a tile is two K-steps, K
// index 8 g + j of step h being tile position 16 g + 8 h + j in both operands
// (any common order of the points gives the same sums up to rounding).
// Eight waves: wave w forms row tile w % 4 of a hidden layer's 128 x 128
// result (column tile w % 4 of the output layer's 3 x 128, rows 3..31 of its
// tile zero) over the even (w < 4) or odd (w >= 4) tiles of the chunk, with
// the next tile's operands loaded while the current one's products run; the
// odd half is added to the even half through LDS.
constexpr int NF_PART_LAYER = NF_WIDTH * NF_WIDTH + NF_WIDTH;
constexpr int NF_GRAD_CHUNKS = 64;      // point chunks of one gradient launch (at most)

struct NFGradIn {
    const __bf16* dz[4];     // bf16 gradients of layers 1-4, tile order
    const float* dout;       // FP32 output gradient [tile][3][32]
    const __bf16* a[5];      // bf16 layer inputs, tile order
    const float* dbp;        // per-tile bias sums [tile][NF_DBP]
};

__device__ __forceinline__ bf16x8 nf_cvt8(const float4 lo, const float4 hi)
{
    bf16x8 r;
    r[0] = (__bf16)lo.x;
    r[1] = (__bf16)lo.y;
    r[2] = (__bf16)lo.z;
    r[3] = (__bf16)lo.w;
    r[4] = (__bf16)hi.x;
    r[5] = (__bf16)hi.y;
    r[6] = (__bf16)hi.z;
    r[7] = (__bf16)hi.w;
    return r;
}

// Operands of one tile for one wave: A (two K-steps) and B (two K-steps of
// NCT column tiles).
template <int NCT>
struct NFTileOps {
    bf16x8 A[2];
    bf16x8 B[NCT][2];
};

template <int NCT>
__device__ __forceinline__ void nf_wgrad_load(const NFGradIn& in, int L, int64_t T, int wt,
                                              NFTileOps<NCT>& o)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int rr = lane & 31;
    const int64_t pos = 16 * g;
    if (NCT == 1) {
        // output layer: A rows are the three outputs (rows 3..31 zero)
        if (rr < 3) {
            const float* src = in.dout + (T * 3 + rr) * 32 + pos;
#pragma unroll
            for (int h = 0; h < 2; ++h)
                o.A[h] = nf_cvt8(*(const float4*)(src + 8 * h), *(const float4*)(src + 8 * h + 4));
        } else {
            o.A[0] = bf16x8{};
            o.A[1] = bf16x8{};
        }
        const __bf16* b = in.a[L] + (T * NF_WIDTH + 32 * wt + rr) * 32 + pos;
        o.B[0][0] = *(const bf16x8*)b;
        o.B[0][1] = *(const bf16x8*)(b + 8);
    } else {
        const __bf16* a = in.dz[L] + (T * NF_WIDTH + 32 * wt + rr) * 32 + pos;
        o.A[0] = *(const bf16x8*)a;
        o.A[1] = *(const bf16x8*)(a + 8);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const __bf16* b = in.a[L] + (T * NF_WIDTH + 32 * ct + rr) * 32 + pos;
            o.B[ct][0] = *(const bf16x8*)b;
            o.B[ct][1] = *(const bf16x8*)(b + 8);
        }
    }
}

template <int NCT>
__device__ inline void nf_wgrad_block(const NFGradIn& in, int L, int64_t t0, int64_t t1,
                                      float* red, float* out)
{
    constexpr bool out_layer = NCT == 1;
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int rr = lane & 31;
    const int w = (int)(threadIdx.x >> 6);
    const int wt = w & 3, kg = w >> 2;
    floatx16 acc[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
        acc[ct] = floatx16{};
    int64_t T = t0 + kg;
    NFTileOps<NCT> cur, nxt;
    if (T < t1)
        nf_wgrad_load<NCT>(in, L, T, wt, cur);
    for (; T < t1; T += 2) {
        if (T + 2 < t1)
            nf_wgrad_load<NCT>(in, L, T + 2, wt, nxt);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cur.A[h], cur.B[ct][h], acc[ct],
                                                                  0, 0, 0);
        cur = nxt;
    }
    // the odd tiles' sums to LDS, added by the wave of the same tile
    if (kg == 1)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                red[((wt * NCT + ct) * 16 + i) * 64 + lane] = acc[ct][i];
    __syncthreads();
    if (kg == 0) {
        // result element i of a lane: row 8 (i / 4) + 4 g + i % 4 of the
        // tile, column rr
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float s = acc[ct][i] + red[((wt * NCT + ct) * 16 + i) * 64 + lane];
                const int r = 8 * (i >> 2) + 4 * g + (i & 3);
                if (out_layer) {
                    if (r < 3)
                        out[r * NF_WIDTH + 32 * wt + rr] = s;
                } else {
                    out[(32 * wt + r) * NF_WIDTH + 32 * ct + rr] = s;
                }
            }
    }
    // bias partials: the chunk's per-wave sums in order
    const int nb = out_layer ? 3 : NF_WIDTH;
    const int off = out_layer ? 4 * NF_WIDTH : L * NF_WIDTH;
    for (int f = (int)threadIdx.x; f < nb; f += (int)blockDim.x)
        out[(out_layer ? 3 : NF_WIDTH) * NF_WIDTH + f] =
            nf_sum_strided(in.dbp + t0 * NF_DBP + off + f, NF_DBP, (int)(t1 - t0));
}

__global__ void __launch_bounds__(512) k_nf_wgrad(NFGradIn in, int64_t ntl, int64_t chunk,
                                                  float* part)
{
    __shared__ float red[4 * 4 * 16 * 64];
    const int L = (int)blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x * chunk;
    const int64_t t1 = t0 + chunk < ntl ? t0 + chunk : ntl;
    float* out = part + ((int64_t)blockIdx.x * 5 + L) * NF_PART_LAYER;
    if (L == 4)
        nf_wgrad_block<1>(in, L, t0, t1, red, out);
    else
        nf_wgrad_block<4>(in, L, t0, t1, red, out);
}

// Sum of the chunk partials into the flat gradient (W1, b1, ..., W4, b4, W5,
// b5): one thread per parameter, chunks summed in order.
__global__ void k_nf_wgrad_reduce(const float* part, int nchunks, float* grad)
{
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= NF_NPARAM)
        return;
    // hidden layers: W [128][128] then b [128], as in the partials; output
    // layer: W5 [3][128] then b5 [3], also as in its partial
    const int L = e < NF_W5 ? e / NF_LAYER_PARAMS : 4;
    const int k = e < NF_W5 ? e % NF_LAYER_PARAMS : e - NF_W5;
    grad[e] = nf_sum_strided(part + (int64_t)L * NF_PART_LAYER + k, (int64_t)5 * NF_PART_LAYER,
                             nchunks);
}

// Physical row of logical row l in a 128-row weight image (inverse of
// nf_logical_row).
__device__ __forceinline__ int nf_phys_row(int l)
{
    const int t = l & 31;
    const int i = 8 * (t >> 4) + (t & 7), g = (t >> 3) & 1;
    return 32 * (l >> 5) + 8 * (i >> 2) + 4 * g + (i & 3);
}

// One Adam step (Kingma & Ba: beta1 0.9, beta2 0.999, eps 1e-8, bias
// corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t) of every FP32 master with
// its gradient summed over the nchunks partials (chunks in order; the flat
// gradient itself is a one-chunk partial), then the parameter's bf16 copies in
// the forward and backward images, placed as k_nf_pack places them: the
// gradient reduction, the update and the repacking in one pass.
__global__ void k_nf_update(const float* part, int nchunks, float* p, float* m, float* v,
                            float lr, float c1, float c2, char* fwd, char* bwd)
{
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= NF_NPARAM)
        return;
    const int L = e < NF_W5 ? e / NF_LAYER_PARAMS : 4;
    const int k = e < NF_W5 ? e % NF_LAYER_PARAMS : e - NF_W5;
    const float gs = nf_sum_strided(part + (int64_t)L * NF_PART_LAYER + k,
                                    (int64_t)5 * NF_PART_LAYER, nchunks);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mi = b1 * m[e] + (1.0f - b1) * gs;
    const float vi = b2 * v[e] + (1.0f - b2) * gs * gs;
    m[e] = mi;
    v[e] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float pn = p[e] - lr * mh / (sqrtf(vh) + eps);
    p[e] = pn;
    __bf16* wf = (__bf16*)fwd;
    __bf16* wb = (__bf16*)bwd;
    float* bf = (float*)(fwd + 4 * NF_IMG_LAYER * 2 + 3 * NF_WIDTH * 2);
    float* bb = (float*)(bwd + 4 * NF_IMG_LAYER * 2 + 3 * NF_WIDTH * 2);
    if (L < 4) {
        if (k < NF_IMG_LAYER) {
            const int o = k / NF_WIDTH, i = k % NF_WIDTH;    // W_L[o][i]
            wf[L * NF_IMG_LAYER + nf_img_off(nf_phys_row(o), i)] = (__bf16)pn;
            wb[L * NF_IMG_LAYER + nf_img_off(nf_phys_row(i), o)] = (__bf16)pn;
        } else {
            bf[L * NF_WIDTH + (k - NF_IMG_LAYER)] = pn;
            bb[L * NF_WIDTH + (k - NF_IMG_LAYER)] = pn;
        }
    } else if (k < 3 * NF_WIDTH) {
        wf[4 * NF_IMG_LAYER + k] = (__bf16)pn;
        wb[4 * NF_IMG_LAYER + k] = (__bf16)pn;
    } else {
        bf[4 * NF_WIDTH + (k - 3 * NF_WIDTH)] = pn;
        bb[4 * NF_WIDTH + (k - 3 * NF_WIDTH)] = pn;
    }
}

// -------------------------------------------------------------------------
// Host side.
// -------------------------------------------------------------------------
struct NeuralField {
    hipStream_t stream = nullptr;
    float* master = nullptr;    // FP32 parameters
    float* grad = nullptr;
    float* am = nullptr;        // Adam moments
    float* av = nullptr;
    int32_t* freq = nullptr;
    char* img_fwd = nullptr;    // NF_LDS_BYTES each
    char* img_bwd = nullptr;
    double b_scale = 1.0;
    int64_t t = 0;              // Adam step
    // training buffers
    int64_t cap = 0;
    float *xh = nullptr, *tgt = nullptr, *out = nullptr, *dout = nullptr;
    __bf16* acts = nullptr;     // five layer inputs, tile order
    __bf16* dz = nullptr;       // four hidden gradients, tile order
    uint2* relu = nullptr;      // ReLU patterns of the hidden outputs
    float* dbp = nullptr;       // per-wave bias sums
    float* part = nullptr;      // split-K partial gradients [NF_GRAD_CHUNKS][5][NF_PART_LAYER]
    double* loss = nullptr;
    int num_cus = 256;
    bool loaded = false;
    bool lds_attr_set = false;
};

static void nf_free_train(NeuralField* nf)
{
    for (void* p : {(void*)nf->xh, (void*)nf->tgt, (void*)nf->out, (void*)nf->dout,
                    (void*)nf->acts, (void*)nf->dz, (void*)nf->relu, (void*)nf->dbp,
                    (void*)nf->part})
        if (p)
            (void)hipFree(p);
    nf->xh = nf->tgt = nf->out = nf->dout = nf->dbp = nf->part = nullptr;
    nf->acts = nf->dz = nullptr;
    nf->relu = nullptr;
    nf->cap = 0;
}

NeuralField* nf_create(hipStream_t s)
{
    NeuralField* nf = new (std::nothrow) NeuralField();
    if (!nf)
        return nullptr;
    nf->stream = s;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        nf->num_cus = prop.multiProcessorCount;
    bool ok = hipMalloc((void**)&nf->master, NF_NPARAM * 4) == hipSuccess &&
              hipMalloc((void**)&nf->grad, NF_NPARAM * 4) == hipSuccess &&
              hipMalloc((void**)&nf->am, NF_NPARAM * 4) == hipSuccess &&
              hipMalloc((void**)&nf->av, NF_NPARAM * 4) == hipSuccess &&
              hipMalloc((void**)&nf->freq, NF_FEAT * 3 * 4) == hipSuccess &&
              hipMalloc((void**)&nf->img_fwd, NF_LDS_BYTES) == hipSuccess &&
              hipMalloc((void**)&nf->img_bwd, NF_LDS_BYTES) == hipSuccess &&
              hipMalloc((void**)&nf->loss, 8) == hipSuccess;
    if (!ok) {
        nf_destroy(nf);
        return nullptr;
    }
    return nf;
}

void nf_destroy(NeuralField* nf)
{
    if (!nf)
        return;
    nf_free_train(nf);
    for (void* p : {(void*)nf->master, (void*)nf->grad, (void*)nf->am, (void*)nf->av,
                    (void*)nf->freq, (void*)nf->img_fwd, (void*)nf->img_bwd, (void*)nf->loss})
        if (p)
            (void)hipFree(p);
    delete nf;
}

static hipError_t nf_pack(NeuralField* nf)
{
    const int total = 4 * NF_IMG_LAYER + 3 * NF_WIDTH + 4 * NF_WIDTH + 4 + 3 * NF_FEAT;
    k_nf_pack<<<(total + 255) / 256, 256, 0, nf->stream>>>(nf->master, nf->freq, nf->img_fwd,
                                                            nf->img_bwd);
    return hipGetLastError();
}

static NFGeom nf_geom(const NeuralField* nf, const GridView& g)
{
    NFGeom G;
    for (int a = 0; a < 3; ++a) {
        G.origin[a] = g.origin[a];
        G.box[a] = (double)g.n[a] / g.inv_spacing;
        G.inv_box[a] = 1.0 / G.box[a];
    }
    G.b_scale = (float)nf->b_scale;
    return G;
}

// The dynamic-LDS limit is a per-device function attribute: set once per
// network object (bound to the device current at its creation).
static hipError_t nf_set_lds_attr(NeuralField* nf)
{
    if (nf->lds_attr_set)
        return hipSuccess;
    const int bytes = (int)NF_LDS_BYTES;
    hipError_t e = hipFuncSetAttribute((const void*)k_nf_eval,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_nf_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_nf_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes);
    nf->lds_attr_set = e == hipSuccess;
    return e;
}

crp_status nf_load(NeuralField* nf, const int32_t* freq, const float* params, double b_scale,
                   std::string& err)
{
    for (int i = 0; i < NF_NPARAM; ++i)
        if (!std::isfinite(params[i])) {
            err = "nf_init: non-finite parameter";
            return CRP_EINVAL;
        }
    for (int i = 0; i < 3 * NF_FEAT; ++i)
        if (freq[i] < -256 || freq[i] > 256) {
            err = "nf_init: frequencies must lie in [-256, 256]";
            return CRP_EINVAL;
        }
    nf->b_scale = b_scale;
    hipError_t e = hipMemcpyAsync(nf->master, params, NF_NPARAM * 4, hipMemcpyHostToDevice,
                                  nf->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(nf->freq, freq, NF_FEAT * 3 * 4, hipMemcpyHostToDevice, nf->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(nf->am, 0, NF_NPARAM * 4, nf->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(nf->av, 0, NF_NPARAM * 4, nf->stream);
    if (e == hipSuccess)
        e = nf_pack(nf);
    if (e == hipSuccess)
        e = nf_set_lds_attr(nf);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nf->stream);
    if (e != hipSuccess) {
        err = std::string("nf_init: ") + hipGetErrorString(e);
        return CRP_EDEVICE;
    }
    nf->t = 0;
    nf->loaded = true;
    return CRP_OK;
}

crp_status nf_get(NeuralField* nf, float* params, std::string& err)
{
    hipError_t e = hipMemcpyAsync(params, nf->master, NF_NPARAM * 4, hipMemcpyDeviceToHost,
                                  nf->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nf->stream);
    if (e != hipSuccess) {
        err = std::string("nf_get_params: ") + hipGetErrorString(e);
        return CRP_EDEVICE;
    }
    return CRP_OK;
}

static int nf_eval_blocks(const NeuralField* nf, int64_t n)
{
    const int64_t waves = (n + 63) / 64;
    const int64_t blocks = (waves + 3) / 4;
    return (int)(blocks < (int64_t)nf->num_cus * 2 ? blocks : (int64_t)nf->num_cus * 2);
}

crp_status nf_eval(NeuralField* nf, const GridView& g, int64_t n, const double* dpos, double* dB,
                   hipStream_t s)
{
    const NFGeom G = nf_geom(nf, g);
    k_nf_eval<<<nf_eval_blocks(nf, n), 256, NF_LDS_BYTES, s>>>(nf->img_fwd, G, n, dpos, dB);
    return hipGetLastError() == hipSuccess ? CRP_OK : CRP_EDEVICE;
}

static hipError_t nf_ensure_cap(NeuralField* nf, int64_t n)
{
    if (nf->cap >= n)
        return hipSuccess;
    nf_free_train(nf);
    const int64_t ld = (n + 63) & ~int64_t(63);
    hipError_t e = hipSuccess;
    auto al = [&](void** p, size_t b) {
        if (e == hipSuccess)
            e = hipMalloc(p, b);
    };
    al((void**)&nf->xh, ld * 12);
    al((void**)&nf->tgt, ld * 12);
    al((void**)&nf->out, ld * 12);
    al((void**)&nf->dout, ld * 12);
    al((void**)&nf->acts, (size_t)5 * NF_WIDTH * ld * 2);
    al((void**)&nf->dz, (size_t)4 * NF_WIDTH * ld * 2);
    al((void**)&nf->relu, (size_t)4 * (ld / 32) * 64 * sizeof(uint2));
    al((void**)&nf->dbp, (size_t)(ld / 32) * NF_DBP * 4);
    al((void**)&nf->part, (size_t)NF_GRAD_CHUNKS * 5 * NF_PART_LAYER * 4);
    if (e == hipSuccess)
        nf->cap = ld;
    return e;
}

// Forward, backward and the split weight gradients (chunk partials in
// nf->part; their count in *nchunks).  The points are those in nf->xh /
// nf->tgt, or with `sample` drawn in the forward (indices offset.. of the
// Philox stream seed, targets from the grid g).  The loss is added to *loss.
static hipError_t nf_fwd_bwd(NeuralField* nf, const NFGeom& G, const GridView& g, int64_t n,
                             bool sample, uint64_t seed, uint64_t offset, double* loss,
                             int* nchunks)
{
    hipStream_t s = nf->stream;
    const int64_t ld = nf->cap;
    // one 32-point tile per wave, eight waves per block, at most one block per CU
    const int64_t ntl = (n + 31) / 32;
    int nb = (int)((ntl + NF_TRAIN_BLOCK / 64 - 1) / (NF_TRAIN_BLOCK / 64));
    if (nb > nf->num_cus)
        nb = nf->num_cus;
    k_nf_fwd<<<nb, NF_TRAIN_BLOCK, NF_LDS_BYTES, s>>>(nf->img_fwd, G, n, ld, nf->xh, sample, g, seed, offset,
                                           nf->tgt, nf->acts, nf->relu, nf->out);
    k_nf_bwd<<<nf_eval_blocks(nf, n), 256, NF_LDS_BYTES, s>>>(nf->img_bwd, G, n, ld, nf->out, nf->tgt, nf->relu,
                                           nf->dz, nf->dout, nf->dbp, loss,
                                           (float)(1.0 / (double)n));
    // the tiles, split over at most NF_GRAD_CHUNKS chunks of at least 8 tiles
    int64_t chunk = (ntl + NF_GRAD_CHUNKS - 1) / NF_GRAD_CHUNKS;
    if (chunk < 8)
        chunk = 8;
    *nchunks = (int)((ntl + chunk - 1) / chunk);
    NFGradIn gi;
    for (int k = 0; k < 4; ++k)
        gi.dz[k] = nf->dz + (int64_t)k * NF_WIDTH * ld;
    gi.dout = nf->dout;
    for (int k = 0; k < 5; ++k)
        gi.a[k] = nf->acts + (int64_t)k * NF_WIDTH * ld;
    gi.dbp = nf->dbp;
    k_nf_wgrad<<<dim3(*nchunks, 5), 512, 0, s>>>(gi, ntl, chunk, nf->part);
    return hipGetLastError();
}

// One Adam step of the masters with the gradient summed over nchunks
// partials (step count t + 1 for the bias corrections, formed in FP64 and
// rounded once), the bf16 images updated in the same pass.
static hipError_t nf_update_launch(NeuralField* nf, const float* part, int nchunks, double lr)
{
    nf->t += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)nf->t));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)nf->t));
    k_nf_update<<<(NF_NPARAM + 255) / 256, 256, 0, nf->stream>>>(
        part, nchunks, nf->master, nf->am, nf->av, (float)lr, c1, c2, nf->img_fwd, nf->img_bwd);
    return hipGetLastError();
}

crp_status nf_adam_step(NeuralField* nf, const float* grad, double lr, std::string& err)
{
    hipError_t e = hipMemcpyAsync(nf->grad, grad, NF_NPARAM * 4, hipMemcpyHostToDevice,
                                  nf->stream);
    if (e == hipSuccess)
        e = nf_update_launch(nf, nf->grad, 1, lr);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nf->stream);
    if (e != hipSuccess) {
        err = std::string("nf_adam_step: ") + hipGetErrorString(e);
        return CRP_EDEVICE;
    }
    return CRP_OK;
}

crp_status nf_loss_grad(NeuralField* nf, const GridView& g, int64_t n, const double* pos,
                        const float* target, float* out, float* grad, double* loss,
                        std::string& err)
{
    hipStream_t s = nf->stream;
    hipError_t e = nf_ensure_cap(nf, n);
    const NFGeom G = nf_geom(nf, g);
    double* dpos = nullptr;
    if (e == hipSuccess)
        e = hipMalloc((void**)&dpos, n * 24);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dpos, pos, n * 24, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(nf->tgt, target, n * 12, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        k_nf_xhat<<<(int)((n + 255) / 256), 256, 0, s>>>(G, n, dpos, nf->xh);
        e = hipGetLastError();
    }
    int nchunks = 0;
    if (e == hipSuccess)
        e = hipMemsetAsync(nf->loss, 0, 8, s);
    if (e == hipSuccess)
        e = nf_fwd_bwd(nf, G, g, n, false, 0, 0, nf->loss, &nchunks);
    if (e == hipSuccess) {
        k_nf_wgrad_reduce<<<(NF_NPARAM + 255) / 256, 256, 0, s>>>(nf->part, nchunks, nf->grad);
        e = hipGetLastError();
    }
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(out, nf->out, n * 12, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && grad)
        e = hipMemcpyAsync(grad, nf->grad, NF_NPARAM * 4, hipMemcpyDeviceToHost, s);
    double l = 0.0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&l, nf->loss, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (dpos)
        (void)hipFree(dpos);
    if (e != hipSuccess) {
        err = std::string("nf_loss_grad: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? CRP_ENOMEM : CRP_EDEVICE;
    }
    if (loss)
        *loss = l;
    return CRP_OK;
}

crp_status nf_train(NeuralField* nf, const GridView& g, int64_t steps, int64_t batch, double lr0,
                    double lr1, uint64_t seed, float* loss_out, std::string& err)
{
    if (g.dtype != 0) {
        err = "nf_train: needs an FP32 grid";
        return CRP_EINVAL;
    }
    hipStream_t s = nf->stream;
    hipError_t e = nf_ensure_cap(nf, batch);
    const NFGeom G = nf_geom(nf, g);
    // the losses of all steps stay on the device until the end
    double* dloss = nullptr;
    const size_t lbytes = (size_t)(steps > 0 ? steps : 1) * 8;
    if (e == hipSuccess)
        e = hipMalloc((void**)&dloss, lbytes);
    if (e == hipSuccess)
        e = hipMemsetAsync(dloss, 0, lbytes, s);
    for (int64_t it = 0; it < steps && e == hipSuccess; ++it) {
        int nchunks = 0;
        e = nf_fwd_bwd(nf, G, g, batch, true, seed, (uint64_t)(it * batch), dloss + it, &nchunks);
        if (e == hipSuccess) {
            const double frac = steps > 1 ? (double)it / (double)(steps - 1) : 1.0;
            e = nf_update_launch(nf, nf->part, nchunks,
                                 lr1 + 0.5 * (lr0 - lr1) * (1.0 + std::cos(M_PI * frac)));
        }
    }
    std::vector<double> losses((size_t)(steps > 0 ? steps : 1));
    if (e == hipSuccess && loss_out && steps > 0)
        e = hipMemcpyAsync(losses.data(), dloss, (size_t)steps * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (dloss)
        (void)hipFree(dloss);
    if (e != hipSuccess) {
        err = std::string("nf_train: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? CRP_ENOMEM : CRP_EDEVICE;
    }
    if (loss_out)
        for (int64_t it = 0; it < steps; ++it)
            loss_out[it] = (float)losses[(size_t)it];
    return CRP_OK;
}

// Parameters of the neural field for the propagation kernel.
void nf_prop_params(const NeuralField* nf, const GridView& g, NFProp* p)
{
    const NFGeom G = nf_geom(nf, g);
    p->img = nf->img_fwd;
    for (int a = 0; a < 3; ++a) {
        p->origin[a] = G.origin[a];
        p->inv_box[a] = G.inv_box[a];
    }
    p->b_scale = G.b_scale;
}

}  // namespace crp
