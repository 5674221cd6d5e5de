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
// keyed by the run seed and the sample's index) and the grid's trilinear
// field there (FP32 weights and sums), in units of b_scale.
__global__ void k_nf_sample(GridView g, NFGeom G, int64_t n, uint64_t seed, uint64_t offset,
                            float* xh, float* tgt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const U64x4 w = philox4x64_10(offset + (uint64_t)i, 0, 0, 0, seed, 0x4e46u);
    double p[3];
    for (int a = 0; a < 3; ++a) {
        const double u = (double)(w.w[a] >> 11) * 0x1p-53;
        xh[3 * i + a] = (float)u;
        p[a] = G.origin[a] + u * G.box[a];
    }
    const GridField<float, 0> F{g};
    float B[3];
    F.fp32(p, B);
    const float inv = 1.0f / G.b_scale;
    tgt[3 * i] = B[0] * inv;
    tgt[3 * i + 1] = B[1] * inv;
    tgt[3 * i + 2] = B[2] * inv;
}

// Training forward: activations of every layer input stored feature-major
// (acts[L][f][p], bf16, leading dimension ld) and the outputs.
__global__ void __launch_bounds__(256) k_nf_fwd(const char* img, NFGeom G, int64_t n, int64_t ld,
                                                const float* xh, __bf16* acts, float* out)
{
    extern __shared__ __attribute__((aligned(16))) char nf_lds[];
    nf_stage_lds(nf_lds, img);
    __syncthreads();
    const NFView v = nf_view(nf_lds, G);
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        bf16x8 a[2][8], b[2][8];
        int64_t pt[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            int64_t p = base + 32 * cb + (lane & 31);
            pt[cb] = p;
            const int64_t q = p < n ? p : n - 1;
            nf_embed_fp64(v.freq, xh[3 * q], xh[3 * q + 1], xh[3 * q + 2], g, a[cb]);
        }
        auto store = [&](int L, const bf16x8 h[2][8]) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                if (pt[cb] >= n)
                    continue;
#pragma unroll
                for (int m = 0; m < 8; ++m)
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        acts[((int64_t)L * NF_WIDTH + 16 * m + 8 * g + j) * ld + pt[cb]] = h[cb][m][j];
            }
        };
        store(0, a);
        nf_layer(v.w[0], v.bias, a, b);
        store(1, b);
        nf_layer(v.w[1], v.bias + NF_WIDTH, b, a);
        store(2, a);
        nf_layer(v.w[2], v.bias + 2 * NF_WIDTH, a, b);
        store(3, b);
        nf_layer(v.w[3], v.bias + 3 * NF_WIDTH, b, a);
        store(4, a);
        float o[3];
        nf_output(v.w5, v.bias + 4 * NF_WIDTH, a, o);
        const int64_t me = base + lane;
        if (me < n)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                out[3 * me + c] = o[c];
    }
}

// Training backward for activations: dOut = 2 (out - target) / n; dH4 = W5^T
// dOut(bf16); dZ_k = dH_k * (h_k > 0); dH_{k-1} = W_k^T dZ_k(bf16) by MFMA with
// the transposed images.  Stores dZ_k and dOut in FP32, feature-major
// ([128][ld] and [3][ld]), for the weight and bias gradients.
__global__ void __launch_bounds__(256) k_nf_bwd(const char* img_t, NFGeom G, int64_t n,
                                                int64_t ld, const float* out, const float* tgt,
                                                const __bf16* acts, float* dzf, float* dout,
                                                float inv_n)
{
    extern __shared__ __attribute__((aligned(16))) char nf_lds[];
    nf_stage_lds(nf_lds, img_t);
    __syncthreads();
    const NFView v = nf_view(nf_lds, G);
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        // dOut of this lane's own point, then shared with the column-block lanes
        float d[3] = {0.f, 0.f, 0.f}, dr[3] = {0.f, 0.f, 0.f};
        const int64_t me = base + lane;
        if (me < n) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                d[c] = 2.0f * (out[3 * me + c] - tgt[3 * me + c]) * inv_n;
                dr[c] = (float)(__bf16)d[c];
                dout[(int64_t)c * ld + me] = d[c];
            }
        }
        bf16x8 dzb[2][8];
        int64_t pt[2];
        // layer 4: dH4 = W5^T dOut on the vector ALU, then the ReLU mask
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const __bf16* w5 = nf_launder(v.w5);
            const int src = 32 * cb + (lane & 31);
            pt[cb] = base + src;
            const float d0 = __shfl(dr[0], src), d1 = __shfl(dr[1], src), d2 = __shfl(dr[2], src);
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int f = 16 * m + 8 * g + j;
                    float s = ((float)w5[f] * d0 + (float)w5[NF_WIDTH + f] * d1) +
                              (float)w5[2 * NF_WIDTH + f] * d2;
                    const bool on = pt[cb] < n &&
                                    (float)acts[((int64_t)4 * NF_WIDTH + f) * ld + pt[cb]] > 0.0f;
                    s = on ? s : 0.0f;
                    dzb[cb][m][j] = (__bf16)s;
                    if (pt[cb] < n)
                        dzf[((int64_t)3 * NF_WIDTH + f) * ld + pt[cb]] = s;
                }
        }
        // layers 4 -> 1: dH_{k-1} = W_k^T dZ_k, mask with h_{k-1} > 0
#pragma unroll 1
        for (int k = 3; k >= 1; --k) {
            const __bf16* wimg = nf_launder(v.w[0] + k * NF_IMG_LAYER);
            bf16x8 nxt[2][8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                floatx16 acc0 = {}, acc1 = {};
                const int row = 32 * r + (lane & 31);
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const bf16x8 a = *(const bf16x8*)(wimg + nf_img_off(row, 16 * m + 8 * g));
                    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, dzb[0][m], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, dzb[1][m], acc1, 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int f = 32 * r + 16 * (i >> 3) + 8 * g + (i & 7);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        float s = cb == 0 ? acc0[i] : acc1[i];
                        const bool on =
                            pt[cb] < n &&
                            (float)acts[((int64_t)k * NF_WIDTH + f) * ld + pt[cb]] > 0.0f;
                        s = on ? s : 0.0f;
                        nxt[cb][2 * r + (i >> 3)][i & 7] = (__bf16)s;
                        if (pt[cb] < n)
                            dzf[((int64_t)(k - 1) * NF_WIDTH + f) * ld + pt[cb]] = s;
                    }
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

// Weight and bias gradients of all five layers in one launch, split over the
// points: block (chunk c, layer L) forms the partial sums over its chunk
//   dW_L[o][i] = sum_p bf16(g_L[o][p]) a_L[i][p],   db_L[o] = sum_p g_L[o][p]
// with g_L the FP32 gradient at layer L's output (g_4: the output gradient,
// 3 rows) and a_L its bf16 input activations, both feature-major with leading
// dimension ld, and writes them to part[c][L] (NF_PART_LAYER floats per layer:
// dW row-major, then db).  Matrix products on MFMA 32x32x16 bf16: the A
// operand is eight consecutive points of a gradient row (converted to bf16
// with round to nearest even, as the backward's own products use it), the B
// operand eight consecutive points of an activation row, both straight from
// memory as 16-byte loads.  Hidden layers: wave w forms rows 32 w.. of the
// 128 x 128 result; output layer: wave w forms columns 32 w.. of the 3 x 128
// result (rows 3..31 of its tile are zero).
constexpr int NF_PART_LAYER = NF_WIDTH * NF_WIDTH + NF_WIDTH;
constexpr int NF_GRAD_CHUNKS = 64;      // point chunks of one gradient launch (at most)

struct NFGradIn {
    const float* g[5];       // FP32 gradients: [128][ld] (layers 1-4), [3][ld] (output)
    const __bf16* a[5];      // bf16 activations [128][ld] (layer inputs)
};

__device__ inline bf16x8 nf_cvt8(const float4 lo, const float4 hi)
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

// One block's partial sums for layer L; NCT column tiles per wave (4 for a
// hidden layer, 1 for the output layer).
template <int NCT>
__device__ inline void nf_wgrad_block(const NFGradIn& in, int L, int64_t p0, int64_t p1,
                                      int64_t ld, float* out)
{
    constexpr bool out_layer = NCT == 1;
    const int lane = (int)(threadIdx.x & 63u);
    const int g = lane >> 5;
    const int w = (int)(threadIdx.x >> 6);
    // this lane's gradient row (A operand) and activation rows (B operands)
    const int arow = out_layer ? (lane & 31) : 32 * w + (lane & 31);
    const bool alive = !out_layer || arow < 3;
    const float* grow = in.g[L] + (int64_t)(alive ? arow : 0) * ld;
    const __bf16* abase = in.a[L];
    floatx16 acc[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
        acc[ct] = floatx16{};
    float bsum = 0.0f;
    for (int64_t p = p0; p < p1; p += 16) {
        const int64_t q = p + 8 * g;          // this lane's eight points
        float4 lo = {0.f, 0.f, 0.f, 0.f}, hi = {0.f, 0.f, 0.f, 0.f};
        const bool full = q + 8 <= p1;
        if (alive && full) {
            lo = *(const float4*)(grow + q);
            hi = *(const float4*)(grow + q + 4);
        } else if (alive) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = q + j < p1 ? grow[q + j] : 0.0f;
            lo = make_float4(v[0], v[1], v[2], v[3]);
            hi = make_float4(v[4], v[5], v[6], v[7]);
        }
        bsum += ((lo.x + lo.y) + (lo.z + lo.w)) + ((hi.x + hi.y) + (hi.z + hi.w));
        const bf16x8 A = nf_cvt8(lo, hi);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int col = out_layer ? 32 * w + (lane & 31) : 32 * ct + (lane & 31);
            const __bf16* brow = abase + (int64_t)col * ld;
            bf16x8 B;
            if (full) {
                B = *(const bf16x8*)(brow + q);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    B[j] = q + j < p1 ? brow[q + j] : (__bf16)0.0f;
            }
            acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[ct], 0, 0, 0);
        }
    }
    // result element i of a lane: row 8 (i / 4) + 4 g + i % 4 of the tile, its column
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = 8 * (i >> 2) + 4 * g + (i & 3);
            if (out_layer) {
                if (r < 3)
                    out[r * NF_WIDTH + 32 * w + (lane & 31)] = acc[ct][i];
            } else {
                out[(32 * w + r) * NF_WIDTH + 32 * ct + (lane & 31)] = acc[ct][i];
            }
        }
    // bias partials: the two lanes of a row hold its two halves of each step
    bsum += __shfl_xor(bsum, 32);
    if (g == 0 && alive && (!out_layer || w == 0))
        out[(out_layer ? 3 : NF_WIDTH) * NF_WIDTH + arow] = bsum;
}

__global__ void __launch_bounds__(256) k_nf_wgrad(NFGradIn in, int64_t n, int64_t ld,
                                                  int64_t chunk, float* part)
{
    const int L = (int)blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * chunk;
    const int64_t p1 = p0 + chunk < n ? p0 + chunk : n;
    float* out = part + ((int64_t)blockIdx.x * 5 + L) * NF_PART_LAYER;
    if (L == 4)
        nf_wgrad_block<1>(in, L, p0, p1, ld, out);
    else
        nf_wgrad_block<4>(in, L, p0, p1, ld, out);
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
    float s = 0.0f;
    for (int c = 0; c < nchunks; ++c)
        s += part[((int64_t)c * 5 + L) * NF_PART_LAYER + k];
    grad[e] = s;
}

// Mean squared error sum_c (out - tgt)^2 averaged over points.
__global__ void k_nf_loss(const float* out, const float* tgt, int64_t n, double* loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)out[i] - (double)tgt[i];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicAdd(loss, red[0] / (double)n);
}

// Adam (Kingma & Ba) with bias correction on the FP32 masters.
__global__ void k_nf_adam(float* p, const float* gr, float* m, float* v, int n, float lr,
                          float c1, float c2)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n)
        return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
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
    __bf16* acts = nullptr;
    float* dzf = nullptr;
    float* part = nullptr;      // split-K partial gradients [NF_GRAD_CHUNKS][5][NF_PART_LAYER]
    double* loss = nullptr;
    int num_cus = 256;
    bool loaded = false;
    bool lds_attr_set = false;
};

static void nf_free_train(NeuralField* nf)
{
    for (void* p : {(void*)nf->xh, (void*)nf->tgt, (void*)nf->out, (void*)nf->dout,
                    (void*)nf->acts, (void*)nf->dzf, (void*)nf->part})
        if (p)
            (void)hipFree(p);
    nf->xh = nf->tgt = nf->out = nf->dout = nf->dzf = nf->part = nullptr;
    nf->acts = nullptr;
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
    al((void**)&nf->dzf, (size_t)4 * NF_WIDTH * ld * 4);
    al((void**)&nf->part, (size_t)NF_GRAD_CHUNKS * 5 * NF_PART_LAYER * 4);
    if (e == hipSuccess)
        nf->cap = ld;
    return e;
}

// Forward + backward + gradients for the points already in nf->xh / nf->tgt.
static hipError_t nf_fwd_bwd(NeuralField* nf, const NFGeom& G, int64_t n)
{
    hipStream_t s = nf->stream;
    const int64_t ld = nf->cap;
    const int nb = nf_eval_blocks(nf, n);
    // (the gradient is written whole by the reduction)
    hipError_t e = hipMemsetAsync(nf->loss, 0, 8, s);
    if (e != hipSuccess)
        return e;
    k_nf_fwd<<<nb, 256, NF_LDS_BYTES, s>>>(nf->img_fwd, G, n, ld, nf->xh, nf->acts, nf->out);
    k_nf_loss<<<256, 256, 0, s>>>(nf->out, nf->tgt, n, nf->loss);
    k_nf_bwd<<<nb, 256, NF_LDS_BYTES, s>>>(nf->img_bwd, G, n, ld, nf->out, nf->tgt, nf->acts,
                                           nf->dzf, nf->dout, (float)(1.0 / (double)n));
    // split over at most NF_GRAD_CHUNKS chunks of a multiple of 16 points
    int64_t chunk = (n + NF_GRAD_CHUNKS - 1) / NF_GRAD_CHUNKS;
    chunk = (chunk + 15) & ~int64_t(15);
    if (chunk < 256)
        chunk = 256;
    const int nchunks = (int)((n + chunk - 1) / chunk);
    NFGradIn gi;
    for (int k = 0; k < 4; ++k)
        gi.g[k] = nf->dzf + (int64_t)k * NF_WIDTH * ld;
    gi.g[4] = nf->dout;
    for (int k = 0; k < 5; ++k)
        gi.a[k] = nf->acts + (int64_t)k * NF_WIDTH * ld;
    k_nf_wgrad<<<dim3(nchunks, 5), 256, 0, s>>>(gi, n, ld, chunk, nf->part);
    k_nf_wgrad_reduce<<<(NF_NPARAM + 255) / 256, 256, 0, s>>>(nf->part, nchunks, nf->grad);
    return hipGetLastError();
}

// One Adam step of the masters with the gradient in nf->grad (step count
// t + 1 for the bias corrections, formed in FP64 and rounded once), then the
// bf16 images are repacked.
static hipError_t nf_adam_launch(NeuralField* nf, double lr)
{
    nf->t += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)nf->t));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)nf->t));
    k_nf_adam<<<(NF_NPARAM + 255) / 256, 256, 0, nf->stream>>>(nf->master, nf->grad, nf->am,
                                                                 nf->av, NF_NPARAM, (float)lr, c1,
                                                                 c2);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = nf_pack(nf);
    return e;
}

crp_status nf_adam_step(NeuralField* nf, const float* grad, double lr, std::string& err)
{
    hipError_t e = hipMemcpyAsync(nf->grad, grad, NF_NPARAM * 4, hipMemcpyHostToDevice,
                                  nf->stream);
    if (e == hipSuccess)
        e = nf_adam_launch(nf, lr);
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
    if (e == hipSuccess)
        e = nf_fwd_bwd(nf, G, n);
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
    std::vector<double> losses((size_t)(steps > 0 ? steps : 1));
    for (int64_t it = 0; it < steps && e == hipSuccess; ++it) {
        k_nf_sample<<<(int)((batch + 255) / 256), 256, 0, s>>>(g, G, batch, seed,
                                                                (uint64_t)(it * batch), nf->xh,
                                                                nf->tgt);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = nf_fwd_bwd(nf, G, batch);
        if (e == hipSuccess) {
            const double frac = steps > 1 ? (double)it / (double)(steps - 1) : 1.0;
            e = nf_adam_launch(nf, lr1 + 0.5 * (lr0 - lr1) * (1.0 + std::cos(M_PI * frac)));
        }
        if (e == hipSuccess && loss_out)
            e = hipMemcpyAsync(&losses[(size_t)it], nf->loss, 8, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
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
