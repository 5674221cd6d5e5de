// Device-side building blocks of the propagation kernels (gfx950, wave64).
//
// Arithmetic contract (both precision forms): this file is compiled with
// -ffp-contract=off and without fast-math, so each + - * / sqrt below is one
// correctly rounded IEEE operation in the order written; sums are evaluated
// left to right in index order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crp {

constexpr double kC = 299792458.0;   // m/s

// -------------------------------------------------------------------------
// Cash-Karp embedded Runge-Kutta 4(5) tableau (Cash & Karp, ACM TOMS 16,
// 1990).  Each rational coefficient is rounded once to FP64.
// -------------------------------------------------------------------------
struct CK {
    static constexpr double a[6][5] = {
        {0.0, 0.0, 0.0, 0.0, 0.0},
        {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0},
        {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0},
        {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0},
        {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0},
        {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
    // 5th-order weights of stages 1, 3, 4, 6 (stages 2 and 5 have weight 0)
    static constexpr double b0 = 37.0 / 378.0, b2 = 250.0 / 621.0, b3 = 125.0 / 594.0,
                            b5 = 512.0 / 1771.0;
    // 5th minus embedded 4th order weights of stages 1, 3, 4, 5, 6
    static constexpr double e0 = -277.0 / 64512.0, e2 = 6925.0 / 370944.0,
                            e3 = -6925.0 / 202752.0, e4 = -277.0 / 14336.0, e5 = 277.0 / 7084.0;
};

// -------------------------------------------------------------------------
// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
// -------------------------------------------------------------------------
struct U64x4 {
    uint64_t w[4];
};

__device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                      uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return U64x4{{c0, c1, c2, c3}};
}

// Draw for event number m of candidate (id, lineage): key (seed, id<<32|lineage).
__device__ inline U64x4 event_draw(uint64_t seed, uint32_t id, uint32_t lineage, uint32_t m)
{
    return philox4x64_10((uint64_t)m, 0, 0, 0, seed, ((uint64_t)id << 32) | (uint64_t)lineage);
}

// Optical depth to the next interaction from one 64-bit word: -ln U with
// U = ((w >> 11) + 1) 2^-53 in (0, 1], rounded to a multiple of 2^-24 (so a
// last-ulp difference between log implementations almost never shows) and at
// least 2^-24.
__device__ inline double optical_depth(uint64_t w)
{
    const double U = (double)((w >> 11) + 1) * 0x1p-53;
    const double t = -log(U);
    const double q = floor(t * 16777216.0 + 0.5) * 0x1p-24;
    return q < 0x1p-24 ? 0x1p-24 : q;
}

// Uniform [0, 1) from one word: (w >> 11) 2^-53.
__device__ inline double unit_uniform(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }

// -------------------------------------------------------------------------
// Step-size factor k / 1024 with k = floor(1024 * 0.95 * r^(-1/5)) defined
// exactly as the largest integer with k^5 r <= (0.95 * 1024)^5 in FP64 (fixed
// order); pow() only supplies the first guess.  k is capped at 5121.
// -------------------------------------------------------------------------
__device__ inline bool ctrl_ok(int k, double r)
{
    const double c1 = 0.95 * 1024.0;
    const double c5 = (((c1 * c1) * c1) * c1) * c1;
    const double kd = (double)k;
    const double k5 = (((kd * kd) * kd) * kd) * kd;
    return k5 * r <= c5;
}

__device__ inline int ctrl_k(double r)
{
    const int KMAX = 5121;
    // first guess from the hardware log2/exp2 in FP32 (a few ulp off at most);
    // the exact search below decides
    int k = KMAX;
    if (r > 1e-30) {
        const float rf = r < 1e30 ? (float)r : 1e30f;
        const float g = 972.8f * __builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf(rf));
        k = g >= (float)KMAX ? KMAX : (g >= 1.0f ? (int)g : 0);
    } else if (!(r >= 0.0)) {
        k = 0;   // NaN
    }
    while (k < KMAX && ctrl_ok(k + 1, r))
        ++k;
    while (k > 0 && !ctrl_ok(k, r))
        --k;
    return k;
}

// -------------------------------------------------------------------------
// Interaction tables (per nucleon at eps = E/A), staged in LDS.
// -------------------------------------------------------------------------
struct TableView {
    const double* e;     // LDS: nodes
    const double* v[3];  // LDS: t_pi, t_n, beta_p
    int n;
    float lg0, scale;    // log2(e[0]), (n - 1) / (log2 e[n-1] - log2 e[0])
};

// Bracketing node and fraction of eps, shared by the three tables (they have
// the same nodes): e[j] <= eps < e[j+1] and t = (eps - e[j]) / (e[j+1] - e[j]);
// clamp < 0 below the first node, > 0 at or above the last.
struct TablePos {
    int j;
    int clamp;
    double t;
};

__device__ inline TablePos table_pos(const TableView& T, double eps)
{
    const double* e = T.e;
    const int n = T.n;
    TablePos p;
    p.j = 0;
    p.t = 0.0;
    p.clamp = 0;
    if (eps <= e[0]) {
        p.clamp = -1;
        return p;
    }
    if (eps >= e[n - 1]) {
        p.clamp = 1;
        return p;
    }
    // first guess from the log-spaced layout (FP32 hardware log2), then exact
    // correction against the node values
    const float gs = (__builtin_amdgcn_logf((float)eps) - T.lg0) * T.scale;
    int j = 0;
    if (gs > 0.0f)   // also false for NaN
        j = gs > (float)(n - 2) ? n - 2 : (int)gs;
    while (j < n - 2 && e[j + 1] <= eps)
        ++j;
    while (j > 0 && e[j] > eps)
        --j;
    p.j = j;
    p.t = (eps - e[j]) / (e[j + 1] - e[j]);
    return p;
}

__device__ inline double table_at(const TableView& T, int which, const TablePos& p)
{
    const double* v = T.v[which];
    if (p.clamp < 0)
        return v[0];
    if (p.clamp > 0)
        return v[T.n - 1];
    return v[p.j] + p.t * (v[p.j + 1] - v[p.j]);
}

__device__ inline double table_value(const TableView& T, int which, double eps)
{
    return table_at(T, which, table_pos(T, eps));
}

struct Rates {
    double rpi, rn, r, beta;
};

// Species scaling: rates A t(E/A) (nucleon channel only for A >= 2),
// continuous loss Z^2/A beta_p(E/A).
__device__ inline Rates species_rates(const TableView& T, int A, int Z, double E)
{
    const double eps = E / (double)A;
    const TablePos p = table_pos(T, eps);
    Rates R;
    R.rpi = (double)A * table_at(T, 0, p);
    R.rn = A >= 2 ? (double)A * table_at(T, 1, p) : 0.0;
    R.r = R.rpi + R.rn;
    const double zz = (double)(Z * Z) / (double)A;
    R.beta = zz * table_at(T, 2, p);
    return R;
}

// -------------------------------------------------------------------------
// Field grid: periodic trilinear interpolation on a vertex grid.
// -------------------------------------------------------------------------
struct GridView {
    const void* data;       // linear [nx][ny][nz][3] (float or double)
    const float* corner;    // FP32 grid: corner records [nx][ny][nz][32] (float) or null
    const double* corner64; // FP64 grid: corner records [nx][ny][nz][24] (double) or null
    int n[3];
    int mask[3];            // n-1 if n is a power of two, else -1
    int64_t stride[3];      // elements: ny*nz*3, nz*3, 3
    double inv_spacing;     // 1 / spacing, rounded once
    double origin[3];
    int dtype;              // 0 float, 1 double
};

struct Cell {
    int i0[3], i1[3];
    double t[3];
};

// Refinement patch of a multi-resolution grid: a non-periodic vertex grid of
// the base grid's element type, refine patch cells per base cell, vertex 0 on
// base vertex `off`.
constexpr int MAX_PATCHES = 4;
struct PatchView {
    const void* data;
    const float* corner;    // corner records [n0][n1][n2][32] (FP32 patches), or null
    int n[3];
    int off[3];
    int64_t stride[2];      // elements: n1*n2*3, n2*3
    double refine;
};
struct NestView {
    int np;
    PatchView p[MAX_PATCHES];
};

__device__ inline int wrap_index(int i, int n, int mask)
{
    if (mask >= 0)
        return i & mask;
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Cell of a position some 2^31 or more cells out on some axis (as a forced
// step with a huge error estimate can produce), or not finite: floor(f) mod n
// by fmod, exact for every finite value, so the periodic cell is the same as
// for any nearer image; a non-finite offset takes cell 0 (its t is NaN, and so
// is the field).  Out of line, arguments and result in registers: no lane of
// a normal run takes it.
struct CellIdx {
    int i[3];
};

__device__ __attribute__((noinline)) CellIdx far_cells(int n0, int n1, int n2, double f0,
                                                       double f1, double f2)
{
    const int n[3] = {n0, n1, n2};
    const double fl[3] = {f0, f1, f2};
    CellIdx r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double m = fmod(fl[a], (double)n[a]);
        if (m < 0.0)
            m += (double)n[a];
        r.i[a] = m == m ? (int)m : 0;
    }
    return r;
}

__device__ inline Cell locate(const GridView& g, const double p[3])
{
    Cell c;
    double fl[3];
    bool near = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double f = (p[a] - g.origin[a]) * g.inv_spacing;
        fl[a] = floor(f);
        near = near & (fabs(fl[a]) < 0x1p31);   // false for a non-finite offset
        // the conversion is only used for offsets within 32 bits; the clamp
        // keeps it defined for the others, which far_cells then replaces
        const double fc = fmin(fmax(fl[a], -0x1p31), 0x1p31 - 1.0);
        c.i0[a] = wrap_index((int)fc, g.n[a], g.mask[a]);
        c.t[a] = f - fl[a];
    }
    if (__builtin_expect(!near, 0)) {
        const CellIdx r = far_cells(g.n[0], g.n[1], g.n[2], fl[0], fl[1], fl[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            c.i0[a] = r.i[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
        c.i1[a] = (c.i0[a] + 1 == g.n[a]) ? 0 : c.i0[a] + 1;
    return c;
}

// The 8 corner vectors of a cell in the order c = dx + 2 dy + 4 dz.
template <class GT>
__device__ inline void gather_linear(const GridView& g, const Cell& c, GT v[8][3])
{
    const GT* G = (const GT*)g.data;
    const int64_t ox[2] = {(int64_t)c.i0[0] * g.stride[0], (int64_t)c.i1[0] * g.stride[0]};
    const int64_t oy[2] = {(int64_t)c.i0[1] * g.stride[1], (int64_t)c.i1[1] * g.stride[1]};
    const int64_t oz[2] = {(int64_t)c.i0[2] * 3, (int64_t)c.i1[2] * 3};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const GT* p = G + ox[k & 1] + oy[(k >> 1) & 1] + oz[(k >> 2) & 1];
        v[k][0] = p[0];
        v[k][1] = p[1];
        v[k][2] = p[2];
    }
}

// Corner-replicated layout: one 128-byte record per cell holds the 8 corner
// vectors (24 floats) followed by 8 pad floats.
__device__ inline void gather_corner(const GridView& g, const Cell& c, float v[8][3])
{
    const int64_t cell = ((int64_t)c.i0[0] * g.n[1] + c.i0[1]) * g.n[2] + c.i0[2];
    const float4* rec = (const float4*)(g.corner + cell * 32);
    float f[24];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const float4 w = rec[q];
        f[4 * q + 0] = w.x;
        f[4 * q + 1] = w.y;
        f[4 * q + 2] = w.z;
        f[4 * q + 3] = w.w;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k][0] = f[3 * k + 0];
        v[k][1] = f[3 * k + 1];
        v[k][2] = f[3 * k + 2];
    }
}

// Wave-cooperative gather of the 64 lanes' corner records (all 64 lanes of
// the wave must call it together).  The 64 records x 6 sixteen-byte chunks
// are spread over the lanes in two halves of 32 records, so one load
// instruction touches about 11 records (cache lines and address translations)
// instead of 64 and each line is read by 6 neighbouring lanes.  The six loads
// of a lane go straight from memory into `stage` (a 64 x 24-float LDS area
// private to the wave; 16-byte global-to-LDS loads, which place lane l's chunk
// at byte 16 l of the instruction's destination), all in flight together and
// holding no registers; then every lane reads its own record back.
constexpr int COOP_STAGE_FLOAT4 = 384;   // float4 slots of one wave's staging area

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// Issue half: the loads of the records of lanes with `need` into the staging
// area (records no lane needs are not fetched).
__device__ inline void coop_issue(const float* corner, uint32_t cell, float* stage, bool need)
{
    const int lane = (int)(threadIdx.x & 63u);
    float4* st = (float4*)stage;
    const uint64_t needm = __ballot(need);
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int idx = 64 * j + lane;            // 0..191
            const int r = idx / 6, c = idx - 6 * r;   // record within the half, chunk
            const int owner = 32 * half + r;
            const uint32_t rc = (uint32_t)__shfl((int)cell, owner);
            const float4* src = (const float4*)(corner + (uint64_t)rc * 32u) + c;
            if ((needm >> owner) & 1ull)
                __builtin_amdgcn_global_load_lds((const void*)src,
                                                 (lds_void_ptr)(st + 192 * half + 64 * j), 16, 0,
                                                 0);
        }
}

// Consume half: waits for the loads, then every lane reads its own record
// (lanes whose record was not fetched get whatever the area holds).
__device__ inline void coop_consume(const float* stage, float v[8][3])
{
    const int lane = (int)(threadIdx.x & 63u);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float f[24];
    const float4* my = (const float4*)stage + 192 * (lane >> 5) + 6 * (lane & 31);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const float4 x = my[q];
        f[4 * q + 0] = x.x;
        f[4 * q + 1] = x.y;
        f[4 * q + 2] = x.z;
        f[4 * q + 3] = x.w;
    }
    // the staging area is rewritten by the wave's next gather
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k][0] = f[3 * k + 0];
        v[k][1] = f[3 * k + 1];
        v[k][2] = f[3 * k + 2];
    }
}

// As coop_issue, for records given by a per-lane address (records of several
// arrays, e.g. the levels of a multi-resolution grid).
__device__ inline void coop_issue_rec(const float* rec, float* stage, bool need)
{
    const int lane = (int)(threadIdx.x & 63u);
    float4* st = (float4*)stage;
    const uint64_t needm = __ballot(need);
    const uint64_t a = (uint64_t)(uintptr_t)rec;
    const int lo = (int)(uint32_t)a, hi = (int)(uint32_t)(a >> 32);
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int idx = 64 * j + lane;            // 0..191
            const int r = idx / 6, c = idx - 6 * r;   // record within the half, chunk
            const int owner = 32 * half + r;
            const uint64_t ra = ((uint64_t)(uint32_t)__shfl(hi, owner) << 32) |
                                (uint64_t)(uint32_t)__shfl(lo, owner);
            const float4* src = (const float4*)(uintptr_t)ra + c;
            if ((needm >> owner) & 1ull)
                __builtin_amdgcn_global_load_lds((const void*)src,
                                                 (lds_void_ptr)(st + 192 * half + 64 * j), 16, 0,
                                                 0);
        }
}

__device__ inline void gather_corner_coop(const float* corner, uint32_t cell, float* stage,
                                          float v[8][3], bool need)
{
    coop_issue(corner, cell, stage, need);
    coop_consume(stage, v);
}

// FP64 corner records: the 8 corner vectors as 24 doubles, 192 bytes with no
// pad, so that every record spans exactly two 128-byte lines.  The wave's 64
// records x 12 sixteen-byte chunks take twelve loads, chunk c of record r
// landing in float4 slot 12 r + c of the staging area (12 KiB per wave).
constexpr int COOP_STAGE64_FLOAT4 = 768;

template <class GT>
constexpr int coop_stage_float4 = sizeof(GT) == 8 ? COOP_STAGE64_FLOAT4 : COOP_STAGE_FLOAT4;

__device__ inline void coop_issue(const double* corner, uint32_t cell, float* stage, bool need)
{
    const int lane = (int)(threadIdx.x & 63u);
    float4* st = (float4*)stage;
    const uint64_t needm = __ballot(need);
    // partly rolled: the fully unrolled form keeps all twelve addresses live
    // and made the FP64 method spill (30% slower on the 256^3 workload)
#pragma unroll 4
    for (int j = 0; j < 12; ++j) {
        const int idx = 64 * j + lane;            // 0..767
        const int r = idx / 12, c = idx - 12 * r;  // record (= owning lane), chunk
        const uint32_t rc = (uint32_t)__shfl((int)cell, r);
        const float4* src = (const float4*)(corner + (uint64_t)rc * 24u) + c;
        if ((needm >> r) & 1ull)
            __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_ptr)(st + 64 * j), 16,
                                             0, 0);
    }
}

__device__ inline void coop_consume(const float* stage, double v[8][3])
{
    const int lane = (int)(threadIdx.x & 63u);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double f[24];
    const double2* my = (const double2*)stage + 12 * lane;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const double2 x = my[q];
        f[2 * q + 0] = x.x;
        f[2 * q + 1] = x.y;
    }
    // the staging area is rewritten by the wave's next gather
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k][0] = f[3 * k + 0];
        v[k][1] = f[3 * k + 1];
        v[k][2] = f[3 * k + 2];
    }
}

__device__ inline void gather_corner_coop(const double* corner, uint32_t cell, float* stage,
                                          double v[8][3], bool need)
{
    coop_issue(corner, cell, stage, need);
    coop_consume(stage, v);
}

// The corner records of a grid's element type.
template <class GT>
__device__ inline const GT* corner_records(const GridView& g)
{
    if constexpr (sizeof(GT) == 8)
        return g.corner64;
    else
        return g.corner;
}

__device__ inline int64_t cell_index(const GridView& g, const Cell& c)
{
    return ((int64_t)c.i0[0] * g.n[1] + c.i0[1]) * g.n[2] + c.i0[2];
}

// FP64 weights and sums: w0 = 1 - t, w1 = t; weight (wx * wy) * wz.
template <class GT>
__device__ inline void interp_fp64(const double t[3], const GT v[8][3], double B[3])
{
    const double wx[2] = {1.0 - t[0], t[0]};
    const double wy[2] = {1.0 - t[1], t[1]};
    const double wz[2] = {1.0 - t[2], t[2]};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double w = (wx[k & 1] * wy[(k >> 1) & 1]) * wz[(k >> 2) & 1];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double term = w * (double)v[k][q];
            B[q] = k == 0 ? term : B[q] + term;
        }
    }
}

// FP32 weights and sums (precision form); t is rounded to FP32 first.
template <class GT>
__device__ inline void interp_fp32(const double t[3], const GT v[8][3], float B[3])
{
    const float tx = (float)t[0], ty = (float)t[1], tz = (float)t[2];
    const float wx[2] = {1.0f - tx, tx};
    const float wy[2] = {1.0f - ty, ty};
    const float wz[2] = {1.0f - tz, tz};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float w = (wx[k & 1] * wy[(k >> 1) & 1]) * wz[(k >> 2) & 1];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float term = w * (float)v[k][q];
            B[q] = k == 0 ? term : B[q] + term;
        }
    }
}

// Field sources used by the stepper.  LAYOUT: 0 linear, 1 corner records
// (per lane, FP32 grids), 2 corner records gathered cooperatively by the whole
// wave (FP32 or FP64 records of the grid's element type).
template <class GT, int LAYOUT>
struct GridField {
    GridView g;
    float* stage = nullptr;   // LAYOUT 2: the wave's LDS staging area
    // need = false: this lane's value will not be used (the cooperative
    // gather then skips its record; the per-lane gathers skip the loads)
    __device__ inline void corners(const Cell& c, GT v[8][3], bool need) const
    {
        if constexpr (LAYOUT == 2) {
            gather_corner_coop(corner_records<GT>(g), (uint32_t)cell_index(g, c), stage, v, need);
        } else if (need) {
            if constexpr (LAYOUT == 1)
                gather_corner(g, c, v);
            else
                gather_linear<GT>(g, c, v);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                v[k][0] = v[k][1] = v[k][2] = (GT)0;
        }
    }
    __device__ inline void fp64(const double p[3], double B[3], bool need = true) const
    {
        const Cell c = locate(g, p);
        GT v[8][3];
        corners(c, v, need);
        interp_fp64(c.t, v, B);
    }
    __device__ inline void fp32(const double p[3], float B[3], bool need = true) const
    {
        const Cell c = locate(g, p);
        GT v[8][3];
        corners(c, v, need);
        float vf[8][3];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                vf[k][q] = (float)v[k][q];
        interp_fp32(c.t, vf, B);
    }

    // Split evaluation (cooperative layout only): prefetch() issues the loads
    // of B(p) for the lanes with `need`; a later *_prefetched(p) with the same
    // p completes it.  Nothing else may use the staging area in between.
    __device__ inline void prefetch(const double p[3], bool need) const
    {
        static_assert(LAYOUT == 2, "split evaluation needs the cooperative layout");
        const Cell c = locate(g, p);
        coop_issue(corner_records<GT>(g), (uint32_t)cell_index(g, c), stage, need);
    }
    __device__ inline void fp32_prefetched(const double p[3], float B[3]) const
    {
        const Cell c = locate(g, p);
        GT v[8][3];
        coop_consume(stage, v);
        interp_fp32(c.t, v, B);
    }
    __device__ inline void fp64_prefetched(const double p[3], double B[3]) const
    {
        const Cell c = locate(g, p);
        GT v[8][3];
        coop_consume(stage, v);
        interp_fp64(c.t, v, B);
    }
};

// Analytic galactic field (section 4: analytic field models for galactic
// propagation; a synthetic disk / halo / X-field model, see crp.h), FP64 in
// the order written: the toroidal factor g with B_t = g (-y, x, 0), then the
// X-field B_x = x q, B_y = y q, B_z = b_x / D - b_x r^2 / (r_x^2 D^2) with
// q = b_x z / (h_x^2 D^2).  The precision form rounds the result to FP32.
// Analytic galactic field: the model parameters and the derived constants
// (1/r_disk^2, 1/h_disk^2, 1/r_halo^2, 1/h_halo^2, 1/h_halo, 1/r_x^2, 1/h_x^2),
// each formed on the host as one FP64 operation on the squared value.
struct AnalyticParams {
    double center[3];
    double b_disk, r_disk, b_halo, r_halo, b_x;
    double kd, ld, kh, lh, ih, kx, lx;
};

// Multi-resolution grid: the base grid plus up to MAX_PATCHES refinement
// patches (P: the patch table, staged in LDS).  A position is located in the
// base grid first; the last patch whose cells hold it, in the patch's own
// cell units r = ((i0 - off) + t) * refine, supplies the cell instead.  Each
// lane gathers its 8 corners from whichever level it selected.
template <class GT, bool COOP = false>
struct NestedField {
    GridView g;
    const PatchView* P = nullptr;
    int np = 0;
    float* stage = nullptr;   // COOP: the wave's LDS staging area
    // the first patch's parameters, kept in (scalar) registers for the common
    // single-patch case, so that its test reads no LDS
    const float* c0 = nullptr;
    int n0[3] = {0, 0, 0}, off0[3] = {0, 0, 0};
    double ref0 = 1.0;
    __device__ inline void set_first(const PatchView& q)
    {
        c0 = q.corner;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            n0[a] = q.n[a];
            off0[a] = q.off[a];
        }
        ref0 = q.refine;
    }
    // COOP: the corner record of the cell that holds p on its level, and the
    // offsets t within that cell
    __device__ inline const float* record(const double p[3], double t[3]) const
    {
        const Cell c = locate(g, p);
        const float* rec = g.corner + cell_index(g, c) * 32;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            t[a] = c.t[a];
        if (np == 1) {
            double r[3];
            bool in = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                r[a] = ((double)(c.i0[a] - off0[a]) + c.t[a]) * ref0;
                in = in && r[a] >= 0.0 && r[a] < (double)(n0[a] - 1);
            }
            if (in) {
                int i[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double fl = floor(r[a]);
                    i[a] = (int)fl;
                    t[a] = r[a] - fl;
                }
                rec = c0 + (((int64_t)i[0] * n0[1] + i[1]) * n0[2] + i[2]) * 32;
            }
            return rec;
        }
        for (int k = np - 1; k >= 0; --k) {
            const PatchView& q = P[k];
            double r[3];
            bool in = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                r[a] = ((double)(c.i0[a] - q.off[a]) + c.t[a]) * q.refine;
                in = in && r[a] >= 0.0 && r[a] < (double)(q.n[a] - 1);
            }
            if (in) {
                int i[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double fl = floor(r[a]);
                    i[a] = (int)fl;
                    t[a] = r[a] - fl;
                }
                rec = q.corner + (((int64_t)i[0] * q.n[1] + i[1]) * q.n[2] + i[2]) * 32;
                break;
            }
        }
        return rec;
    }
    __device__ inline void corners(const double p[3], GT v[8][3], double t[3], bool need) const
    {
        const Cell c = locate(g, p);
        const GT* src = (const GT*)g.data;
        int64_t ox[2] = {(int64_t)c.i0[0] * g.stride[0], (int64_t)c.i1[0] * g.stride[0]};
        int64_t oy[2] = {(int64_t)c.i0[1] * g.stride[1], (int64_t)c.i1[1] * g.stride[1]};
        int64_t oz[2] = {(int64_t)c.i0[2] * 3, (int64_t)c.i1[2] * 3};
#pragma unroll
        for (int a = 0; a < 3; ++a)
            t[a] = c.t[a];
        for (int k = np - 1; k >= 0; --k) {
            const PatchView& q = P[k];
            double r[3];
            bool in = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                r[a] = ((double)(c.i0[a] - q.off[a]) + c.t[a]) * q.refine;
                in = in && r[a] >= 0.0 && r[a] < (double)(q.n[a] - 1);
            }
            if (in) {
                int i[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double fl = floor(r[a]);
                    i[a] = (int)fl;
                    t[a] = r[a] - fl;
                }
                src = (const GT*)q.data;
                ox[0] = (int64_t)i[0] * q.stride[0];
                ox[1] = ox[0] + q.stride[0];
                oy[0] = (int64_t)i[1] * q.stride[1];
                oy[1] = oy[0] + q.stride[1];
                oz[0] = (int64_t)i[2] * 3;
                oz[1] = oz[0] + 3;
                break;
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (need) {
                const GT* e = src + ox[k & 1] + oy[(k >> 1) & 1] + oz[(k >> 2) & 1];
                v[k][0] = e[0];
                v[k][1] = e[1];
                v[k][2] = e[2];
            } else {
                v[k][0] = v[k][1] = v[k][2] = (GT)0;
            }
        }
    }
    __device__ inline void fp64(const double p[3], double B[3], bool need = true) const
    {
        double t[3];
        if constexpr (COOP) {
            float v[8][3];
            coop_issue_rec(record(p, t), stage, need);
            coop_consume(stage, v);
            interp_fp64(t, v, B);
        } else {
            GT v[8][3];
            corners(p, v, t, need);
            interp_fp64(t, v, B);
        }
    }
    __device__ inline void fp32(const double p[3], float B[3], bool need = true) const
    {
        double t[3];
        if constexpr (COOP) {
            float v[8][3];
            coop_issue_rec(record(p, t), stage, need);
            coop_consume(stage, v);
            interp_fp32(t, v, B);
        } else {
            GT v[8][3];
            corners(p, v, t, need);
            float vf[8][3];
#pragma unroll
            for (int k = 0; k < 8; ++k)
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    vf[k][q] = (float)v[k][q];
            interp_fp32(t, vf, B);
        }
    }
    // Split evaluation (COOP only), as GridField's: prefetch() issues the
    // record loads of B(p); *_prefetched(p) with the same p completes it.
    __device__ inline void prefetch(const double p[3], bool need) const
    {
        static_assert(COOP, "split evaluation needs the cooperative gather");
        double t[3];
        coop_issue_rec(record(p, t), stage, need);
    }
    __device__ inline void fp32_prefetched(const double p[3], float B[3]) const
    {
        double t[3];
        (void)record(p, t);
        float v[8][3];
        coop_consume(stage, v);
        interp_fp32(t, v, B);
    }
    __device__ inline void fp64_prefetched(const double p[3], double B[3]) const
    {
        double t[3];
        (void)record(p, t);
        float v[8][3];
        coop_consume(stage, v);
        interp_fp64(t, v, B);
    }
};

struct AnalyticFieldSrc {
    AnalyticParams a;
    __device__ inline void fp64(const double p[3], double B[3], bool need = true) const
    {
        (void)need;
        const double dx = p[0] - a.center[0], dy = p[1] - a.center[1], dz = p[2] - a.center[2];
        const double r2 = dx * dx + dy * dy;
        const double z2 = dz * dz;
        // two divisions: g over the common denominator of its disk and halo
        // parts, and one reciprocal of D for the X-field
        const double X = (a.r_disk * (1.0 + r2 * a.kd)) * (1.0 + z2 * a.ld);
        const double wh = 1.0 + z2 * a.lh;
        const double Y = (a.r_halo * (1.0 + r2 * a.kh)) * (wh * wh);
        const double g = (a.b_disk * Y + (a.b_halo * (dz * a.ih)) * X) / (X * Y);
        const double D = (1.0 + r2 * a.kx) + z2 * a.lx;
        const double iD = 1.0 / D;
        const double iD2 = iD * iD;
        const double q = (a.b_x * (dz * a.lx)) * iD2;
        B[0] = (-g) * dy + dx * q;
        B[1] = g * dx + dy * q;
        B[2] = a.b_x * iD - (a.b_x * (r2 * a.kx)) * iD2;
    }
    __device__ inline void fp32(const double p[3], float B[3], bool need = true) const
    {
        double b[3];
        fp64(p, b, need);
        B[0] = (float)b[0];
        B[1] = (float)b[1];
        B[2] = (float)b[2];
    }
};

// -------------------------------------------------------------------------
// One Cash-Karp attempt.  FP64 form: state y = (x, u), derivative
// K = (u, kappa u x B(x)), kappa = Z c / E.  Returns the error estimate
// h |sum e_i K_i^u| and the 5th-order state (local extrapolation).
// -------------------------------------------------------------------------
__device__ inline void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ inline double dot3(const double a[3], const double b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

__device__ inline void cross3f(const float a[3], const float b[3], float c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ inline float dot3f(const float a[3], const float b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

__device__ inline void deriv_from_field(double kappa, const double y[6], const double B[3],
                                         double k[6])
{
    double c[3];
    cross3(y + 3, B, c);
    k[0] = y[3];
    k[1] = y[4];
    k[2] = y[5];
    k[3] = kappa * c[0];
    k[4] = kappa * c[1];
    k[5] = kappa * c[2];
}

// `need`: this lane's result is used.  `reuse`: b1 already holds B(x) of this
// very position (a retry after a rejected attempt), so the first stage does
// not gather it again; otherwise b1 receives B(x).
template <class F>
__device__ inline double ck_attempt_fp64(const F& field, double kappa, const double y[6],
                                         double h, double y5[6], bool need, bool reuse,
                                         double b1[3])
{
    double K[6][6];
    {
        double B[3];
        field.fp64(y, B, need && !reuse);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (reuse)
                B[q] = b1[q];
            b1[q] = B[q];
        }
        deriv_from_field(kappa, y, B, K[0]);
    }
#pragma unroll
    for (int i = 1; i < 6; ++i) {
        double ys[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            double s = CK::a[i][0] * K[0][q];
#pragma unroll
            for (int j = 1; j < i; ++j)
                s = s + CK::a[i][j] * K[j][q];
            ys[q] = y[q] + h * s;
        }
        double B[3];
        field.fp64(ys, B, need);
        deriv_from_field(kappa, ys, B, K[i]);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double s = CK::b0 * K[0][q];
        s = s + CK::b2 * K[2][q];
        s = s + CK::b3 * K[3][q];
        s = s + CK::b5 * K[5][q];
        y5[q] = y[q] + h * s;
    }
    double e[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double s = CK::e0 * K[0][3 + q];
        s = s + CK::e2 * K[2][3 + q];
        s = s + CK::e3 * K[3][3 + q];
        s = s + CK::e4 * K[4][3 + q];
        s = s + CK::e5 * K[5][3 + q];
        e[q] = s;
    }
    return h * sqrt(dot3(e, e));
}

// Precision form: stage increments G_i = (h u_i, (h kappa) u_i x B(x_i)) in
// FP32 with h and h*kappa formed in FP64 and rounded once; stage positions
// are the FP64 position plus the FP32 offset; the error is |sum e_i G_i^u|.
__device__ inline void incr_from_field(float hf, float hk, const float u[3], const float B[3],
                                        float G[6])
{
    float c[3];
    cross3f(u, B, c);
    G[0] = hf * u[0];
    G[1] = hf * u[1];
    G[2] = hf * u[2];
    G[3] = hk * c[0];
    G[4] = hk * c[1];
    G[5] = hk * c[2];
}

// need / reuse / b1 as for ck_attempt_fp64 (b1 in FP32).
template <class F>
__device__ inline double ck_attempt_mix_f(const F& field, double kappa, const double x[3],
                                          const float u[3], double h, double x5[3],
                                          float u5[3], bool need, bool reuse, float b1[3])
{
    const float hf = (float)h;
    const float hk = (float)(h * kappa);
    float G[6][6];
    {
        float B[3];
        field.fp32(x, B, need && !reuse);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (reuse)
                B[q] = b1[q];
            b1[q] = B[q];
        }
        incr_from_field(hf, hk, u, B, G[0]);
    }
#pragma unroll
    for (int i = 1; i < 6; ++i) {
        float s[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            float acc = (float)CK::a[i][0] * G[0][q];
#pragma unroll
            for (int j = 1; j < i; ++j)
                acc = acc + (float)CK::a[i][j] * G[j][q];
            s[q] = acc;
        }
        double xs[3];
        float us[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            xs[q] = x[q] + (double)s[q];
            us[q] = u[q] + s[3 + q];
        }
        float B[3];
        field.fp32(xs, B, need);
        incr_from_field(hf, hk, us, B, G[i]);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        float s = (float)CK::b0 * G[0][q];
        s = s + (float)CK::b2 * G[2][q];
        s = s + (float)CK::b3 * G[3][q];
        s = s + (float)CK::b5 * G[5][q];
        if (q < 3)
            x5[q] = x[q] + (double)s;
        else
            u5[q - 3] = u[q - 3] + s;
    }
    float e[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        float s = (float)CK::e0 * G[0][3 + q];
        s = s + (float)CK::e2 * G[2][3 + q];
        s = s + (float)CK::e3 * G[3][3 + q];
        s = s + (float)CK::e4 * G[4][3 + q];
        s = s + (float)CK::e5 * G[5][3 + q];
        e[q] = s;
    }
    return (double)sqrtf(dot3f(e, e));
}

// The same precision-form attempt with the six stages in a rolled loop, so
// that the field evaluation appears once in the code.  Used where that
// evaluation is large (the neural field: an inlined copy per stage would not
// fit the instruction cache).  The stage sums keep the index order of the
// unrolled form: a term j >= i is skipped, not added as zero.
template <class F>
__device__ inline double ck_attempt_mix_rolled(const F& field, double kappa, const double x[3],
                                               const float u[3], double h, double x5[3],
                                               float u5[3])
{
    static constexpr float A[6][5] = {
        {(float)CK::a[0][0], (float)CK::a[0][1], (float)CK::a[0][2], (float)CK::a[0][3], (float)CK::a[0][4]},
        {(float)CK::a[1][0], (float)CK::a[1][1], (float)CK::a[1][2], (float)CK::a[1][3], (float)CK::a[1][4]},
        {(float)CK::a[2][0], (float)CK::a[2][1], (float)CK::a[2][2], (float)CK::a[2][3], (float)CK::a[2][4]},
        {(float)CK::a[3][0], (float)CK::a[3][1], (float)CK::a[3][2], (float)CK::a[3][3], (float)CK::a[3][4]},
        {(float)CK::a[4][0], (float)CK::a[4][1], (float)CK::a[4][2], (float)CK::a[4][3], (float)CK::a[4][4]},
        {(float)CK::a[5][0], (float)CK::a[5][1], (float)CK::a[5][2], (float)CK::a[5][3], (float)CK::a[5][4]}};
    const float hf = (float)h;
    const float hk = (float)(h * kappa);
    float G[6][6];
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
        for (int q = 0; q < 6; ++q)
            G[j][q] = 0.0f;
#pragma unroll 1
    for (int i = 0; i < 6; ++i) {
        double xs[3];
        float us[3];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            float acc = A[i][0] * G[0][q];
#pragma unroll
            for (int j = 1; j < 5; ++j) {
                const float t = acc + A[i][j] * G[j][q];
                acc = j < i ? t : acc;
            }
            if (q < 3)
                xs[q] = i == 0 ? x[q] : x[q] + (double)acc;
            else
                us[q - 3] = i == 0 ? u[q - 3] : u[q - 3] + acc;
        }
        float B[3], Gi[6];
        field.fp32(xs, B, true);
        incr_from_field(hf, hk, us, B, Gi);
#pragma unroll
        for (int j = 0; j < 6; ++j)
#pragma unroll
            for (int q = 0; q < 6; ++q)
                G[j][q] = j == i ? Gi[q] : G[j][q];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        float s = (float)CK::b0 * G[0][q];
        s = s + (float)CK::b2 * G[2][q];
        s = s + (float)CK::b3 * G[3][q];
        s = s + (float)CK::b5 * G[5][q];
        if (q < 3)
            x5[q] = x[q] + (double)s;
        else
            u5[q - 3] = u[q - 3] + s;
    }
    float e[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        float s = (float)CK::e0 * G[0][3 + q];
        s = s + (float)CK::e2 * G[2][3 + q];
        s = s + (float)CK::e3 * G[3][3 + q];
        s = s + (float)CK::e4 * G[4][3 + q];
        s = s + (float)CK::e5 * G[5][3 + q];
        e[q] = s;
    }
    return (double)sqrtf(dot3f(e, e));
}

// -------------------------------------------------------------------------
// Wave64 helpers.
// -------------------------------------------------------------------------
__device__ inline uint64_t wave_ballot(bool p) { return __ballot(p); }

// number of set bits of mask in lanes below this one
__device__ inline int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline int lane_id() { return (int)(threadIdx.x & 63u); }

}  // namespace crp
