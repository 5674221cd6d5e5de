// Host runtime of libcrp: the C-ABI declared in include/crp.h.
//
// Owns every device buffer of a context (queue, parked queue, finished and
// neutral record buffers, counters, tables, optional corner-layout grid),
// launches the kernels on the context's stream and converts errors into
// crp_status codes (no exception crosses the ABI).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/crp.h"
#include "crp_internal.hpp"
#include "crp_lens.hpp"
#include "crp_nf.hpp"
#include "crp_nf_device.hpp"

namespace crp {
template <int MODE, class GT, int LAYOUT, int BS, bool TRAJ>
__global__ void k_propagate(const PropParams* PP);
template <class GT, int LAYOUT>
__global__ void k_eval_field(GridView g, int64_t n, const double* pos, double* B, int mode);
__global__ void k_validate(int64_t n, const uint32_t* id, const int32_t* A, const int32_t* Z,
                           const double* E, const double* pos, const double* dir,
                           const double* lmax, double max_extent, unsigned long long* first_bad);
__global__ void k_inject(QueueSoA q, int64_t base, int64_t n, const uint32_t* id,
                         const int32_t* A, const int32_t* Z, const double* E,
                         const double* pos, const double* dir, const double* lmax,
                         const uint32_t* perm, uint64_t seed, double hmin, int mix);
__global__ void k_inject_keys(int64_t n, const int32_t* Z, const double* E, const double* lmax,
                              unsigned long long* keys, uint32_t* idx);
template <class GT>
__global__ void k_corner_relayout(GridView g, GT* out);
__global__ void k_gather_ceiling(const float* corner, uint32_t ncell, int iters, float* sink);
__global__ void k_eval_analytic(AnalyticParams a, int64_t n, const double* pos, double* B);
__global__ void k_observe(ObsParams p);
size_t observe_lds_bytes(int ne, int ng);
template <class GT>
__global__ void k_eval_nested(GridView g, NestView nv, int64_t n, const double* pos, double* B,
                              int mode);
}  // namespace crp

using namespace crp;

struct crp_ctx {
    crp_config cfg;
    hipStream_t stream = nullptr;
    std::string err;
    int num_cus = 256;
    std::string device_name;

    // field grid
    bool has_grid = false;
    const void* grid = nullptr;
    void* grid_owned = nullptr;
    int grid_dtype = CRP_F64;
    int64_t gn[3] = {0, 0, 0};
    double spacing = 0.0;
    double origin[3] = {0, 0, 0};
    float* corner = nullptr;       // corner records of an FP32 grid (128 B per cell)
    double* corner64 = nullptr;    // corner records of an FP64 grid (192 B per cell)
    // refinement patches of the grid (multi-resolution)
    NestView nest{};
    void* patch_owned[MAX_PATCHES] = {nullptr, nullptr, nullptr, nullptr};
    float* patch_corner[MAX_PATCHES] = {nullptr, nullptr, nullptr, nullptr};

    // tables (device: e, tpi, tn, bp consecutive)
    bool has_tables = false;
    bool has_analytic = false;
    AnalyticParams ana{};
    double* tab = nullptr;
    int tab_n = 0;
    float lg0 = 0.0f, lgscale = 0.0f;

    // buffers
    void* qmem[2] = {nullptr, nullptr};
    QueueSoA q, park;
    void* fmem = nullptr;
    FinishedSoA fin;
    void* nmem = nullptr;
    NeutralSoA neu;
    void* tmem = nullptr;                    // trajectory points (traj_capacity > 0)
    TrajSoA traj{};
    DevCounters* cnt = nullptr;
    PropParams* d_params = nullptr;          // kernel parameter block (device)
    unsigned long long* scratch = nullptr;   // small device scratch (validation)
    void* xfer = nullptr;                    // read-back staging (grow-only)
    size_t xfer_bytes = 0;
    void* order_mem = nullptr;               // injection-order sort buffers (grow-only)
    size_t order_bytes = 0;

    int64_t pending = 0;
    int64_t fin_unread = 0, neu_unread = 0, traj_unread = 0;
    crp_counters totals;

    crp_launch launch;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0.0;
    int64_t last_launches = 0;

    NeuralField* nf = nullptr;
    bool nf_attr_set = false;

    // observable sums (crp_set_observables)
    bool has_obs = false;
    crp_observables obs{};
    void* obs_mem = nullptr;
    ObsParams obs_p{};
    size_t obs_sky_n = 0;                    // sky entries

    // galactic lenses (crp_lens_build)
    Lens lens;
    bool has_lens = false;
};

namespace {

crp_status fail(crp_ctx* ctx, crp_status st, const std::string& msg)
{
    if (ctx)
        ctx->err = msg;
    // a failed HIP call (an allocation that did not fit, say) stays the
    // thread's last error until read: clear it here, so that the launch check
    // of a later call reports only its own launch
    (void)hipGetLastError();
    return st;
}

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, e_ == hipErrorOutOfMemory ? CRP_ENOMEM : CRP_EDEVICE,           \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    } while (0)

// Carves a structure of arrays out of one allocation (256-byte aligned pieces).
struct Carver {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t n)
    {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

size_t queue_layout(char* base, int64_t cap, QueueSoA* q)
{
    Carver c{base};
    QueueSoA t;
    t.x = c.take<double>(3 * cap);
    t.u = c.take<double>(3 * cap);
    t.u0 = c.take<double>(3 * cap);
    t.E = c.take<double>(cap);
    t.L = c.take<double>(cap);
    t.Lmax = c.take<double>(cap);
    t.hctrl = c.take<double>(cap);
    t.tau = c.take<double>(cap);
    t.E0 = c.take<double>(cap);
    t.id = c.take<uint32_t>(cap);
    t.lineage = c.take<uint32_t>(cap);
    t.m = c.take<uint32_t>(cap);
    t.nsteps = c.take<uint32_t>(cap);
    t.nrej = c.take<uint32_t>(cap);
    t.A = c.take<int32_t>(cap);
    t.Z = c.take<int32_t>(cap);
    t.ready = c.take<uint32_t>(cap);
    t.cap = cap;
    if (q)
        *q = t;
    return c.off;
}

size_t finished_layout(char* base, int64_t cap, FinishedSoA* f)
{
    Carver c{base};
    FinishedSoA t;
    t.x = c.take<double>(3 * cap);
    t.u = c.take<double>(3 * cap);
    t.u0 = c.take<double>(3 * cap);
    t.E = c.take<double>(cap);
    t.L = c.take<double>(cap);
    t.E0 = c.take<double>(cap);
    t.id = c.take<uint32_t>(cap);
    t.lineage = c.take<uint32_t>(cap);
    t.m = c.take<uint32_t>(cap);
    t.nsteps = c.take<uint32_t>(cap);
    t.nrej = c.take<uint32_t>(cap);
    t.status = c.take<int32_t>(cap);
    t.A = c.take<int32_t>(cap);
    t.Z = c.take<int32_t>(cap);
    t.cap = cap;
    if (f)
        *f = t;
    return c.off;
}

size_t neutral_layout(char* base, int64_t cap, NeutralSoA* n)
{
    Carver c{base};
    NeutralSoA t;
    t.x = c.take<double>(3 * cap);
    t.u = c.take<double>(3 * cap);
    t.E = c.take<double>(cap);
    t.id = c.take<uint32_t>(cap);
    t.lineage = c.take<uint32_t>(cap);
    t.m = c.take<uint32_t>(cap);
    t.chan = c.take<int32_t>(cap);
    t.cap = cap;
    if (n)
        *n = t;
    return c.off;
}

size_t traj_layout(char* base, int64_t cap, TrajSoA* t)
{
    Carver c{base};
    TrajSoA r;
    r.x = c.take<double>(3 * cap);
    r.L = c.take<double>(cap);
    r.E = c.take<double>(cap);
    r.id = c.take<uint32_t>(cap);
    r.lineage = c.take<uint32_t>(cap);
    r.n = c.take<uint32_t>(cap);
    r.A = c.take<int32_t>(cap);
    r.cap = cap;
    if (t)
        *t = r;
    return c.off;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

GridView make_view(const crp_ctx* ctx)
{
    GridView g;
    g.data = ctx->grid;
    g.corner = ctx->corner;
    g.corner64 = ctx->corner64;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = (int)ctx->gn[a];
        g.mask[a] = is_pow2(ctx->gn[a]) ? (int)(ctx->gn[a] - 1) : -1;
        g.origin[a] = ctx->origin[a];
    }
    g.stride[0] = ctx->gn[1] * ctx->gn[2] * 3;
    g.stride[1] = ctx->gn[2] * 3;
    g.stride[2] = 3;
    g.inv_spacing = 1.0 / ctx->spacing;
    g.dtype = ctx->grid_dtype == CRP_F32 ? 0 : 1;
    return g;
}

int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// Dynamic LDS of the propagation kernel: the four tables (the per-lane state
// kept out of registers is static LDS of the kernel).
size_t lds_bytes(int ntab, int block)
{
    (void)block;
    return (size_t)4 * ntab * sizeof(double);
}

// Blocks of one propagation kernel that fit on a compute unit at once.
template <int MODE, class GT, int LAYOUT>
int resident_blocks(int bs, size_t lds)
{
    int nbpm = 0;
    hipError_t e;
    if (bs == 128)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nbpm, (const void*)k_propagate<MODE, GT, LAYOUT, 128, false>, 128, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nbpm, (const void*)k_propagate<MODE, GT, LAYOUT, 256, false>, 256, lds);
    return (e == hipSuccess && nbpm > 0) ? nbpm : 1;
}

// traj: the variant with the per-step output module (only when it records)
template <int MODE, class GT, int LAYOUT>
void launch_propagate(int nb, int bs, size_t lds, hipStream_t s, const PropParams* dp, bool traj)
{
    if (bs == 128 && traj)
        k_propagate<MODE, GT, LAYOUT, 128, true><<<nb, 128, lds, s>>>(dp);
    else if (bs == 128)
        k_propagate<MODE, GT, LAYOUT, 128, false><<<nb, 128, lds, s>>>(dp);
    else if (traj)
        k_propagate<MODE, GT, LAYOUT, 256, true><<<nb, 256, lds, s>>>(dp);
    else
        k_propagate<MODE, GT, LAYOUT, 256, false><<<nb, 256, lds, s>>>(dp);
}

// [start, start+k) of a planar [3][cap] array as [k][3] (a thread per row, grid
// stride: coalesced reads of each plane, 24-byte rows written side by side).
__global__ void k_interleave3(const double* __restrict__ planar, int64_t cap, int64_t start,
                              int64_t k, double* __restrict__ out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            out[3 * i + a] = planar[a * cap + start + i];
    }
}

// Copies [start, start+k) of a planar [3][cap] device array into host [k][3]:
// interleaved on the device into the context's grow-only staging buffer
// (chunks of at most 2^25 rows, 768 MiB), each chunk then copied once; the
// steps are ordered on the stream, so a chunk's copy ends before the next
// chunk overwrites the buffer.
hipError_t copy_planar(crp_ctx* ctx, double* host, const double* dev, int64_t cap, int64_t start,
                       int64_t k)
{
    if (k == 0 || host == nullptr)
        return hipSuccess;
    const int64_t chunk_max = 1ll << 25;
    const size_t need = (size_t)std::min<int64_t>(k, chunk_max) * 3 * sizeof(double);
    if (need > ctx->xfer_bytes) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess)
            return e;
        if (ctx->xfer)
            (void)hipFree(ctx->xfer);
        ctx->xfer = nullptr;
        ctx->xfer_bytes = 0;
        e = hipMalloc(&ctx->xfer, need);
        if (e != hipSuccess)
            return e;
        ctx->xfer_bytes = need;
    }
    for (int64_t c0 = 0; c0 < k; c0 += chunk_max) {
        const int64_t kc = std::min<int64_t>(chunk_max, k - c0);
        const int nb = (int)std::min<int64_t>(blocks_for(kc, 256), 65536);
        k_interleave3<<<nb, 256, 0, ctx->stream>>>(dev, cap, start + c0, kc, (double*)ctx->xfer);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(host + 3 * c0, ctx->xfer, (size_t)kc * 3 * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <class T>
hipError_t copy_d2h(T* host, const T* dev, int64_t k, hipStream_t s)
{
    if (k == 0 || host == nullptr)
        return hipSuccess;
    return hipMemcpyAsync(host, dev, k * sizeof(T), hipMemcpyDeviceToHost, s);
}

// Builds the corner records of grid g (ncell cells; 128 bytes per FP32 record,
// 192 per FP64 record) into a new allocation; *out is set only once the
// records are complete, so a failed build leaves nothing behind.
template <class GT>
crp_status build_corner_records(crp_ctx* ctx, const GridView& g, int64_t ncell, GT** out)
{
    const size_t rec = sizeof(GT) == 8 ? 192 : 128;
    GT* p = nullptr;
    HIPCHK(ctx, hipMalloc((void**)&p, (size_t)ncell * rec));
    k_corner_relayout<GT><<<ctx->num_cus * 8, 256, 0, ctx->stream>>>(g, p);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return fail(ctx, CRP_EDEVICE, std::string("corner records: ") + hipGetErrorString(e));
    }
    *out = p;
    return CRP_OK;
}

// Corner records of the base grid and of every refinement patch (built on
// first use).  A patch's record of cell (i,j,k) holds its vertices i..i+1 etc.;
// the records of its last vertex planes are built too (from wrapped indices)
// but never read, since level selection keeps r < n - 1.  An FP64 grid has
// records of its base grid only (192 bytes per cell); its patches are always
// read from their linear arrays.
crp_status ensure_corner(crp_ctx* ctx)
{
    const int64_t ncell = ctx->gn[0] * ctx->gn[1] * ctx->gn[2];
    if (ncell >= (1ll << 32))
        return fail(ctx, CRP_EINVAL, "corner layout: at most 2^32 - 1 cells");
    if (ctx->grid_dtype == CRP_F64)
        return ctx->corner64 ? CRP_OK
                             : build_corner_records<double>(ctx, make_view(ctx), ncell,
                                                            &ctx->corner64);
    if (!ctx->corner) {
        crp_status st = build_corner_records<float>(ctx, make_view(ctx), ncell, &ctx->corner);
        if (st != CRP_OK)
            return st;
    }
    for (int k = 0; k < ctx->nest.np; ++k) {
        if (ctx->patch_corner[k])
            continue;
        PatchView& q = ctx->nest.p[k];
        GridView g{};
        g.data = q.data;
        for (int a = 0; a < 3; ++a) {
            g.n[a] = q.n[a];
            g.mask[a] = is_pow2(q.n[a]) ? q.n[a] - 1 : -1;
        }
        g.stride[0] = q.stride[0];
        g.stride[1] = q.stride[1];
        g.stride[2] = 3;
        g.inv_spacing = 1.0;
        g.dtype = 0;
        crp_status st = build_corner_records<float>(ctx, g, (int64_t)q.n[0] * q.n[1] * q.n[2],
                                                    &ctx->patch_corner[k]);
        if (st != CRP_OK)
            return st;
        q.corner = ctx->patch_corner[k];
    }
    return CRP_OK;
}

void free_patches(crp_ctx* ctx)
{
    for (int k = 0; k < MAX_PATCHES; ++k) {
        if (ctx->patch_owned[k])
            (void)hipFree(ctx->patch_owned[k]);
        ctx->patch_owned[k] = nullptr;
        if (ctx->patch_corner[k])
            (void)hipFree(ctx->patch_corner[k]);
        ctx->patch_corner[k] = nullptr;
    }
    ctx->nest = NestView{};
}

void free_corner(crp_ctx* ctx)
{
    if (ctx->corner) {
        (void)hipFree(ctx->corner);
        ctx->corner = nullptr;
    }
    if (ctx->corner64) {
        (void)hipFree(ctx->corner64);
        ctx->corner64 = nullptr;
    }
}

// Launches one propagation run over the pending queue (no host bookkeeping
// of totals).  On return the device counter block is in *dc.
crp_status run_kernel(crp_ctx* ctx, int64_t max_cycles, DevCounters* dc)
{
    DevCounters init;
    std::memset(&init, 0, sizeof init);
    init.head = 0;
    init.tail = (unsigned long long)ctx->pending;
    init.head1 = (unsigned long long)ctx->pending;
    init.fin_n = (unsigned long long)ctx->fin_unread;
    init.neu_n = (unsigned long long)ctx->neu_unread;
    init.traj_n = (unsigned long long)ctx->traj_unread;
    HIPCHK(ctx, hipMemcpyAsync(ctx->cnt, &init, sizeof init, hipMemcpyHostToDevice, ctx->stream));

    PropParams P;
    P.q = ctx->q;
    P.park = ctx->park;
    P.fin = ctx->fin;
    P.neu = ctx->neu;
    P.traj = ctx->traj;
    P.cnt = ctx->cnt;
    P.grid = make_view(ctx);
    P.tab.e = ctx->tab;
    P.tab.v[0] = ctx->tab + ctx->tab_n;
    P.tab.v[1] = ctx->tab + 2 * ctx->tab_n;
    P.tab.v[2] = ctx->tab + 3 * ctx->tab_n;
    P.tab.n = ctx->tab_n;
    P.tab.lg0 = ctx->lg0;
    P.tab.scale = ctx->lgscale;
    const crp_config& c = ctx->cfg;
    P.sp.tol = c.tol;
    P.sp.hmin = c.hmin;
    P.sp.hmax = c.hmax;
    P.sp.eps_loss = c.eps_loss;
    P.sp.kappa_pi = c.kappa_pi;
    P.sp.e_floor = c.e_floor;
    for (int a = 0; a < 3; ++a)
        P.sp.obs[a] = c.obs_center[a];
    P.sp.obs_r = c.obs_radius;
    P.sp.seed = c.seed;
    P.sp.renorm = c.renormalize;
    P.sp.charge_sign = c.charge_sign == -1 ? -1 : 1;
    for (int a = 0; a < 3; ++a)
        P.sp.bnd[a] = c.boundary_center[a];
    P.sp.bnd_r = c.boundary_radius;
    P.sp.traj_every = (uint32_t)c.traj_every;
    P.sp.traj_ids = c.traj_ids;
    P.ana = ctx->ana;
    P.nest = ctx->nest;
    P.max_cycles = max_cycles;
    P.tail0 = (unsigned long long)ctx->pending;
    P.fin0 = init.fin_n;
    // the neural-field stepper costs the same per wave however many lanes are
    // busy, so it refills a lane as soon as it is idle
    P.refill = c.field_mode == CRP_FIELD_NEURAL ? 1 : ctx->launch.refill;

    const bool neural = c.field_mode == CRP_FIELD_NEURAL;
    const bool traj = c.traj_every > 0;
    if (neural)
        nf_prop_params(ctx->nf, P.grid, &P.nf);
    const bool analytic = c.field_mode == CRP_FIELD_ANALYTIC;
    // refinement patches: levels selected per lane
    const bool nested = !neural && !analytic && ctx->nest.np > 0;
    const int layout = ctx->launch.layout;
    // (the multi-resolution kernel of an FP64 grid reads linear arrays only)
    if (layout == CRP_LAYOUT_CORNER && !neural && !analytic &&
        (ctx->grid_dtype == CRP_F32 || !nested)) {
        crp_status st = ensure_corner(ctx);
        if (st != CRP_OK)
            return st;
        P.grid.corner = ctx->corner;
        P.grid.corner64 = ctx->corner64;
        P.nest = ctx->nest;        // now with the patches' corner records
    }
    const int bs = ctx->launch.block;
    const size_t lds = lds_bytes(ctx->tab_n, bs);
    const bool mix = c.precision == CRP_MIX;
    const bool f32 = ctx->grid_dtype == CRP_F32;
    int bpc = ctx->launch.blocks_per_cu;
    if (bpc == 0) {   // as many blocks as fit on a compute unit
        if (nested && f32 && layout == CRP_LAYOUT_CORNER)
            bpc = mix ? resident_blocks<MODE_MIX, float, 6>(bs, lds)
                      : resident_blocks<MODE_FP64, float, 6>(bs, lds);
        else if (nested && f32)
            bpc = mix ? resident_blocks<MODE_MIX, float, 5>(bs, lds)
                      : resident_blocks<MODE_FP64, float, 5>(bs, lds);
        else if (nested)
            bpc = mix ? resident_blocks<MODE_MIX, double, 5>(bs, lds)
                      : resident_blocks<MODE_FP64, double, 5>(bs, lds);
        else if (analytic)
            bpc = mix ? resident_blocks<MODE_MIX, double, 4>(bs, lds)
                      : resident_blocks<MODE_FP64, double, 4>(bs, lds);
        else if (!mix && !f32 && layout == CRP_LAYOUT_CORNER)
            bpc = resident_blocks<MODE_FP64, double, 2>(bs, lds);
        else if (!mix && !f32)
            bpc = resident_blocks<MODE_FP64, double, 0>(bs, lds);
        else if (!mix && layout == CRP_LAYOUT_CORNER)
            bpc = resident_blocks<MODE_FP64, float, 2>(bs, lds);
        else if (!mix)
            bpc = resident_blocks<MODE_FP64, float, 0>(bs, lds);
        else if (!f32 && layout == CRP_LAYOUT_CORNER)
            bpc = resident_blocks<MODE_MIX, double, 2>(bs, lds);
        else if (!f32)
            bpc = resident_blocks<MODE_MIX, double, 0>(bs, lds);
        else if (layout == CRP_LAYOUT_CORNER)
            bpc = resident_blocks<MODE_MIX, float, 2>(bs, lds);
        else
            bpc = resident_blocks<MODE_MIX, float, 0>(bs, lds);
    }
    const int nb = ctx->num_cus * bpc;

    HIPCHK(ctx, hipMemcpyAsync(ctx->d_params, &P, sizeof P, hipMemcpyHostToDevice, ctx->stream));
    const PropParams* dp = ctx->d_params;
    hipStream_t s = ctx->stream;
    if (neural) {
        const size_t nl = lds + NF_LDS_BYTES;
        // the network, the tables and the per-lane state share the CU's LDS
        if (nl + (size_t)256 * (7 * 8 + 7 * 4) + 256 > (size_t)160 * 1024)
            return fail(ctx, CRP_EINVAL, "neural propagation: tables too large for LDS (n <= 200)");
        // the dynamic-LDS limit is a per-device function attribute: set it
        // once per context (each context is bound to one device)
        if (!ctx->nf_attr_set) {
            HIPCHK(ctx, hipFuncSetAttribute((const void*)k_propagate<MODE_MIX, float, 3, 256, false>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)nl));
            HIPCHK(ctx, hipFuncSetAttribute((const void*)k_propagate<MODE_MIX, float, 3, 256, true>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)nl));
            ctx->nf_attr_set = true;
        }
        HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
        if (traj)
            k_propagate<MODE_MIX, float, 3, 256, true><<<ctx->num_cus, 256, nl, s>>>(dp);
        else
            k_propagate<MODE_MIX, float, 3, 256, false><<<ctx->num_cus, 256, nl, s>>>(dp);
    } else {
    HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    if (nested && f32 && layout == CRP_LAYOUT_CORNER && mix)
        launch_propagate<MODE_MIX, float, 6>(nb, bs, lds, s, dp, traj);
    else if (nested && f32 && layout == CRP_LAYOUT_CORNER)
        launch_propagate<MODE_FP64, float, 6>(nb, bs, lds, s, dp, traj);
    else if (nested && f32 && mix)
        launch_propagate<MODE_MIX, float, 5>(nb, bs, lds, s, dp, traj);
    else if (nested && f32)
        launch_propagate<MODE_FP64, float, 5>(nb, bs, lds, s, dp, traj);
    else if (nested && mix)
        launch_propagate<MODE_MIX, double, 5>(nb, bs, lds, s, dp, traj);
    else if (nested)
        launch_propagate<MODE_FP64, double, 5>(nb, bs, lds, s, dp, traj);
    else if (analytic && mix)
        launch_propagate<MODE_MIX, double, 4>(nb, bs, lds, s, dp, traj);
    else if (analytic)
        launch_propagate<MODE_FP64, double, 4>(nb, bs, lds, s, dp, traj);
    else if (!mix && !f32 && layout == CRP_LAYOUT_CORNER)
        launch_propagate<MODE_FP64, double, 2>(nb, bs, lds, s, dp, traj);
    else if (!mix && !f32)
        launch_propagate<MODE_FP64, double, 0>(nb, bs, lds, s, dp, traj);
    else if (!mix && layout == CRP_LAYOUT_CORNER)
        launch_propagate<MODE_FP64, float, 2>(nb, bs, lds, s, dp, traj);
    else if (!mix)
        launch_propagate<MODE_FP64, float, 0>(nb, bs, lds, s, dp, traj);
    else if (!f32 && layout == CRP_LAYOUT_CORNER)
        launch_propagate<MODE_MIX, double, 2>(nb, bs, lds, s, dp, traj);
    else if (!f32)
        launch_propagate<MODE_MIX, double, 0>(nb, bs, lds, s, dp, traj);
    else if (layout == CRP_LAYOUT_CORNER)
        launch_propagate<MODE_MIX, float, 2>(nb, bs, lds, s, dp, traj);
    else
        launch_propagate<MODE_MIX, float, 0>(nb, bs, lds, s, dp, traj);
    }
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(dc, ctx->cnt, sizeof *dc, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_ms = ms;
    ctx->last_launches = 1;
    if (dc->error)
        return fail(ctx, CRP_EDEVICE,
                    "propagation kernel: a wave waited too long for the run to drain");
    return CRP_OK;
}

// Host bookkeeping after a run: record counts, parked candidates become the
// pending queue.
void after_run(crp_ctx* ctx, const DevCounters& dc, bool add_totals)
{
    ctx->fin_unread = (int64_t)std::min<unsigned long long>(dc.fin_n, ctx->fin.cap);
    ctx->neu_unread = (int64_t)std::min<unsigned long long>(dc.neu_n, ctx->neu.cap);
    const int64_t traj_before = ctx->traj_unread;
    ctx->traj_unread = (int64_t)std::min<unsigned long long>(dc.traj_n, ctx->traj.cap);
    if (add_totals) {
        crp_counters& t = ctx->totals;
        t.finished += dc.finished;
        t.observed += dc.observed;
        t.max_traj += dc.max_traj;
        t.energy_floor += dc.energy_floor;
        t.steps += dc.steps;
        t.attempts += dc.attempts;
        t.rejects += dc.rejects;
        t.forced += dc.forced;
        t.events += dc.events;
        t.null_events += dc.null_events;
        t.inter_pi += dc.inter_pi;
        t.inter_n += dc.inter_n;
        t.charged_sec += dc.charged_sec;
        t.neutral_sec += dc.neutral_sec;
        t.queue_deferred += dc.queue_deferred;
        t.neutral_deferred += dc.neutral_deferred;
        t.lane_slots += dc.lane_slots;
        t.boundary += dc.boundary;
        t.traj_points += ctx->traj_unread - traj_before;
        // the cursor started at the unread count (within the capacity) and
        // counted every point; those past the capacity were dropped
        if (dc.traj_n > (unsigned long long)ctx->traj.cap)
            t.traj_dropped += (int64_t)(dc.traj_n - (unsigned long long)ctx->traj.cap);
    }
    ctx->pending = (int64_t)dc.park_n;
    if (dc.park_n > 0) {
        std::swap(ctx->q, ctx->park);
        std::swap(ctx->qmem[0], ctx->qmem[1]);
    }
}

// Copies the first n slots of every array of a queue into another queue
// (planar vectors plane by plane).
hipError_t copy_queue_slots(const QueueSoA& d, const QueueSoA& s, int64_t n, hipStream_t st)
{
    hipError_t e = hipSuccess;
    auto cp = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes)
            e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
    };
    for (int a = 0; a < 3; ++a) {
        cp(d.x + a * d.cap, s.x + a * s.cap, n * 8);
        cp(d.u + a * d.cap, s.u + a * s.cap, n * 8);
        cp(d.u0 + a * d.cap, s.u0 + a * s.cap, n * 8);
    }
    cp(d.E, s.E, n * 8);
    cp(d.L, s.L, n * 8);
    cp(d.Lmax, s.Lmax, n * 8);
    cp(d.hctrl, s.hctrl, n * 8);
    cp(d.tau, s.tau, n * 8);
    cp(d.E0, s.E0, n * 8);
    cp(d.id, s.id, n * 4);
    cp(d.lineage, s.lineage, n * 4);
    cp(d.m, s.m, n * 4);
    cp(d.nsteps, s.nsteps, n * 4);
    cp(d.nrej, s.nrej, n * 4);
    cp(d.A, s.A, n * 4);
    cp(d.Z, s.Z, n * 4);
    return e;
}

// Same for the finished-record buffer.
hipError_t copy_finished_slots(const FinishedSoA& d, const FinishedSoA& s, int64_t n,
                               hipStream_t st)
{
    hipError_t e = hipSuccess;
    auto cp = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes)
            e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
    };
    for (int a = 0; a < 3; ++a) {
        cp(d.x + a * d.cap, s.x + a * s.cap, n * 8);
        cp(d.u + a * d.cap, s.u + a * s.cap, n * 8);
        cp(d.u0 + a * d.cap, s.u0 + a * s.cap, n * 8);
    }
    cp(d.E, s.E, n * 8);
    cp(d.L, s.L, n * 8);
    cp(d.E0, s.E0, n * 8);
    cp(d.id, s.id, n * 4);
    cp(d.lineage, s.lineage, n * 4);
    cp(d.m, s.m, n * 4);
    cp(d.nsteps, s.nsteps, n * 4);
    cp(d.nrej, s.nrej, n * 4);
    cp(d.status, s.status, n * 4);
    cp(d.A, s.A, n * 4);
    cp(d.Z, s.Z, n * 4);
    return e;
}

// Grows the work queue (and its park buffer) to cap slots and the finished-
// record buffer to 2 cap, keeping the pending candidates and the unread
// records.  On failure nothing is changed.
crp_status grow_queue(crp_ctx* ctx, int64_t cap)
{
    if (cap <= ctx->q.cap)
        return CRP_OK;
    hipStream_t s = ctx->stream;
    void* nq[2] = {nullptr, nullptr};
    void* nf = nullptr;
    QueueSoA q2, p2;
    FinishedSoA f2;
    hipError_t e = hipMalloc(&nq[0], queue_layout(nullptr, cap, nullptr));
    if (e == hipSuccess)
        e = hipMalloc(&nq[1], queue_layout(nullptr, cap, nullptr));
    if (e == hipSuccess)
        e = hipMalloc(&nf, finished_layout(nullptr, 2 * cap, nullptr));
    if (e == hipSuccess) {
        queue_layout((char*)nq[0], cap, &q2);
        queue_layout((char*)nq[1], cap, &p2);
        finished_layout((char*)nf, 2 * cap, &f2);
        e = hipMemsetAsync(q2.ready, 0, cap * sizeof(uint32_t), s);
    }
    if (e == hipSuccess)
        e = hipMemsetAsync(p2.ready, 0, cap * sizeof(uint32_t), s);
    if (e == hipSuccess)
        e = copy_queue_slots(q2, ctx->q, ctx->pending, s);
    if (e == hipSuccess)
        e = copy_finished_slots(f2, ctx->fin, ctx->fin_unread, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        for (void* p : {nq[0], nq[1], nf})
            if (p)
                (void)hipFree(p);
        return fail(ctx, e == hipErrorOutOfMemory ? CRP_ENOMEM : CRP_EDEVICE,
                    std::string("queue growth: ") + hipGetErrorString(e));
    }
    for (void* p : {ctx->qmem[0], ctx->qmem[1], ctx->fmem})
        (void)hipFree(p);
    ctx->qmem[0] = nq[0];
    ctx->qmem[1] = nq[1];
    ctx->fmem = nf;
    ctx->q = q2;
    ctx->park = p2;
    ctx->fin = f2;
    return CRP_OK;
}

}  // namespace

// -------------------------------------------------------------------------
// Autotuner cache: one line per tuning, "KEY : block=B blocks_per_cu=C
// refill=R layout=L steps_per_s=S", KEY naming the device, the grid shape and
// element type, the precision and the field mode.
// -------------------------------------------------------------------------
static std::string tune_key(const crp_ctx* ctx)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s grid=%lldx%lldx%lld dtype=%d precision=%d field=%d",
             ctx->device_name.c_str(), (long long)ctx->gn[0], (long long)ctx->gn[1],
             (long long)ctx->gn[2], ctx->grid_dtype, ctx->cfg.precision, ctx->cfg.field_mode);
    return buf;
}

// The latest valid entry for key in the cache file, if any.
static bool tune_cache_lookup(const char* path, const std::string& key, crp_launch* out,
                              double* rate)
{
    FILE* f = fopen(path, "r");
    if (!f)
        return false;
    bool found = false;
    char line[512];
    const std::string prefix = key + " : ";
    while (fgets(line, sizeof line, f)) {
        if (std::strncmp(line, prefix.c_str(), prefix.size()) != 0)
            continue;
        crp_launch l;
        double r = 0.0;
        if (sscanf(line + prefix.size(), "block=%d blocks_per_cu=%d refill=%d layout=%d "
                                         "steps_per_s=%lf",
                   &l.block, &l.blocks_per_cu, &l.refill, &l.layout, &r) == 5 &&
            (l.block == 128 || l.block == 256) && l.blocks_per_cu >= 0 &&
            l.blocks_per_cu <= 64 && l.refill >= 1 && l.refill <= 64 &&
            (l.layout == CRP_LAYOUT_LINEAR || l.layout == CRP_LAYOUT_CORNER)) {
            *out = l;
            *rate = r;
            found = true;
        }
    }
    fclose(f);
    return found;
}

// -------------------------------------------------------------------------
// Field evaluation shared by crp_eval_field and crp_eval_field_noalloc.
// -------------------------------------------------------------------------
static crp_status eval_field_check(crp_ctx* ctx, int32_t mode, const char* who)
{
    const bool neural = mode == 16 + CRP_FIELD_NEURAL;
    const bool analytic = mode == 16 + CRP_FIELD_ANALYTIC;
    if (!(mode == CRP_FP64 || mode == CRP_MIX || neural || analytic))
        return fail(ctx, CRP_EINVAL, std::string(who) + ": bad mode");
    if (analytic ? !ctx->has_analytic : !ctx->has_grid)
        return fail(ctx, CRP_ESTATE, std::string(who) + ": no such field set");
    if (neural && !ctx->nf)
        return fail(ctx, CRP_ESTATE, std::string(who) + ": neural field not initialised");
    return CRP_OK;
}

// Launches the evaluation of n device positions into device B on the
// context stream (mode checked by eval_field_check).
static crp_status eval_field_launch(crp_ctx* ctx, int64_t n, const double* dpos, double* dB,
                                    int32_t mode)
{
    if (mode == 16 + CRP_FIELD_ANALYTIC) {
        k_eval_analytic<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(ctx->ana, n, dpos, dB);
        return CRP_OK;
    }
    if (mode == 16 + CRP_FIELD_NEURAL)
        return nf_eval(ctx->nf, make_view(ctx), n, dpos, dB, ctx->stream);
    GridView g = make_view(ctx);
    const int md = mode == CRP_MIX ? MODE_MIX : MODE_FP64;
    if (ctx->nest.np > 0 && ctx->grid_dtype == CRP_F64)
        k_eval_nested<double><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(g, ctx->nest, n, dpos,
                                                                           dB, md);
    else if (ctx->nest.np > 0)
        k_eval_nested<float><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(g, ctx->nest, n, dpos,
                                                                          dB, md);
    else if (ctx->grid_dtype == CRP_F64)
        k_eval_field<double, 0><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(g, n, dpos, dB, md);
    else if (ctx->launch.layout == CRP_LAYOUT_CORNER && ctx->corner)
        k_eval_field<float, 1><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(g, n, dpos, dB, md);
    else
        k_eval_field<float, 0><<<blocks_for(n, 256), 256, 0, ctx->stream>>>(g, n, dpos, dB, md);
    return CRP_OK;
}

// -------------------------------------------------------------------------
// Static staging for crp_eval_field_noalloc: positions [CRP_EVAL_NOALLOC_MAX][3]
// then fields [CRP_EVAL_NOALLOC_MAX][3], FP64 (12 MiB).  Every GPU the library
// runs on holds its own copy until the process ends.  In host code the array's
// name is not a device address: its address on each device is looked up once,
// at crp_create with that device current, and only that address is used.
// -------------------------------------------------------------------------
static __device__ __align__(256) double scratch[6 * CRP_EVAL_NOALLOC_MAX];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex scratch_mu;
static double* scratch_dev[SCRATCH_MAX_DEVICES];

// Looks up this device's copy of `scratch` (the device must be current).
static hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_dev[device])
        return hipSuccess;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess)
        scratch_dev[device] = (double*)p;
    return e;
}

static double* scratch_ptr(int device)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES)
        return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    return scratch_dev[device];
}

extern "C" {

const char* crp_last_error(const crp_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

crp_status crp_create(const crp_config* cfg, void* stream, crp_ctx** out)
{
    if (!cfg || !out)
        return CRP_EINVAL;
    *out = nullptr;
    const crp_config& c = *cfg;
    if (!(c.precision == CRP_FP64 || c.precision == CRP_MIX) ||
        !(c.field_mode == CRP_FIELD_GRID || c.field_mode == CRP_FIELD_NEURAL ||
          c.field_mode == CRP_FIELD_ANALYTIC) ||
        !(c.charge_sign == -1 || c.charge_sign == 0 || c.charge_sign == 1) ||
        !(c.inject_order == CRP_ORDER_LONGEST_FIRST || c.inject_order == CRP_ORDER_AS_GIVEN) ||
        !(c.boundary_radius >= 0) || !std::isfinite(c.boundary_radius) ||
        !std::isfinite(c.boundary_center[0]) || !std::isfinite(c.boundary_center[1]) ||
        !std::isfinite(c.boundary_center[2]) ||
        !(c.tol > 0) || !(c.hmin > 0) || !(c.hmax >= c.hmin) || !(c.eps_loss > 0) ||
        !std::isfinite(c.tol) || !std::isfinite(c.hmax) || !std::isfinite(c.eps_loss) ||
        !(c.kappa_pi >= 0 && c.kappa_pi < 1) || !(c.e_floor >= 0) || !std::isfinite(c.e_floor) ||
        !(c.obs_radius >= 0) || !std::isfinite(c.obs_radius) || !std::isfinite(c.obs_center[0]) ||
        !std::isfinite(c.obs_center[1]) || !std::isfinite(c.obs_center[2]) ||
        c.queue_capacity <= 0 || c.neutral_capacity <= 0 || c.queue_capacity > (1ll << 40) ||
        c.neutral_capacity > (1ll << 40) ||
        c.traj_every < 0 || c.traj_capacity < 0 || c.traj_capacity > (1ll << 40) ||
        (c.traj_every > 0 && c.traj_capacity == 0) ||
        (c.field_mode == CRP_FIELD_NEURAL && c.precision != CRP_MIX))
        return CRP_EINVAL;
    crp_ctx* ctx = new (std::nothrow) crp_ctx();
    if (!ctx)
        return CRP_ENOMEM;
    ctx->cfg = c;
    ctx->stream = (hipStream_t)stream;
    std::memset(&ctx->totals, 0, sizeof ctx->totals);
    ctx->launch.block = 128;
    ctx->launch.blocks_per_cu = 0;
    ctx->launch.refill = 4;
    ctx->launch.layout = CRP_LAYOUT_LINEAR;
    auto bail = [&](crp_status st, const char* what, hipError_t e) {
        fprintf(stderr, "crp_create: %s: %s\n", what, hipGetErrorString(e));
        crp_destroy(ctx);
        (void)hipGetLastError();   // as in fail()
        return st;
    };
    hipError_t e = hipSetDevice(c.device);
    if (e != hipSuccess)
        return bail(CRP_EDEVICE, "hipSetDevice", e);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, c.device);
    if (e != hipSuccess)
        return bail(CRP_EDEVICE, "hipGetDeviceProperties", e);
    ctx->num_cus = prop.multiProcessorCount;
    ctx->device_name = prop.gcnArchName;
    e = scratch_setup(c.device);
    if (e != hipSuccess)
        return bail(CRP_EDEVICE, "static scratch lookup (hipGetSymbolAddress)", e);
    const int64_t qc = c.queue_capacity;
    for (int b = 0; b < 2; ++b) {
        size_t bytes = queue_layout(nullptr, qc, nullptr);
        e = hipMalloc(&ctx->qmem[b], bytes);
        if (e != hipSuccess)
            return bail(CRP_ENOMEM, "queue allocation", e);
        queue_layout((char*)ctx->qmem[b], qc, b == 0 ? &ctx->q : &ctx->park);
        QueueSoA& qq = b == 0 ? ctx->q : ctx->park;
        e = hipMemset(qq.ready, 0, qc * sizeof(uint32_t));
        if (e != hipSuccess)
            return bail(CRP_EDEVICE, "hipMemset", e);
    }
    {
        size_t bytes = finished_layout(nullptr, 2 * qc, nullptr);
        e = hipMalloc(&ctx->fmem, bytes);
        if (e != hipSuccess)
            return bail(CRP_ENOMEM, "finished-record allocation", e);
        finished_layout((char*)ctx->fmem, 2 * qc, &ctx->fin);
    }
    {
        size_t bytes = neutral_layout(nullptr, c.neutral_capacity, nullptr);
        e = hipMalloc(&ctx->nmem, bytes);
        if (e != hipSuccess)
            return bail(CRP_ENOMEM, "neutral-record allocation", e);
        neutral_layout((char*)ctx->nmem, c.neutral_capacity, &ctx->neu);
    }
    if (c.traj_capacity > 0) {
        size_t bytes = traj_layout(nullptr, c.traj_capacity, nullptr);
        e = hipMalloc(&ctx->tmem, bytes);
        if (e != hipSuccess)
            return bail(CRP_ENOMEM, "trajectory-point allocation", e);
        traj_layout((char*)ctx->tmem, c.traj_capacity, &ctx->traj);
    }
    e = hipMalloc((void**)&ctx->cnt, sizeof(DevCounters));
    if (e != hipSuccess)
        return bail(CRP_ENOMEM, "counter allocation", e);
    e = hipMalloc((void**)&ctx->d_params, sizeof(PropParams));
    if (e != hipSuccess)
        return bail(CRP_ENOMEM, "parameter block allocation", e);
    e = hipMalloc((void**)&ctx->scratch, 64);
    if (e != hipSuccess)
        return bail(CRP_ENOMEM, "scratch allocation", e);
    e = hipEventCreate(&ctx->ev0);
    if (e == hipSuccess)
        e = hipEventCreate(&ctx->ev1);
    if (e != hipSuccess)
        return bail(CRP_EDEVICE, "hipEventCreate", e);
    *out = ctx;
    return CRP_OK;
}

void crp_destroy(crp_ctx* ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->cfg.device);
    if (ctx->stream)
        (void)hipStreamSynchronize(ctx->stream);
    else
        (void)hipDeviceSynchronize();
    nf_destroy(ctx->nf);
    free_patches(ctx);
    lens_free(ctx->lens);
    lens_free_scratch(ctx->lens);
    for (void* p : {ctx->qmem[0], ctx->qmem[1], ctx->fmem, ctx->nmem, ctx->tmem, ctx->obs_mem,
                    (void*)ctx->cnt,
                    (void*)ctx->d_params,
                    (void*)ctx->scratch, ctx->xfer, ctx->order_mem, ctx->grid_owned,
                    (void*)ctx->tab,
                    (void*)ctx->corner, (void*)ctx->corner64})
        if (p)
            (void)hipFree(p);
    if (ctx->ev0)
        (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1)
        (void)hipEventDestroy(ctx->ev1);
    delete ctx;
}

crp_status crp_set_field_grid(crp_ctx* ctx, const void* data, int32_t dtype, int32_t on_device,
                              int64_t nx, int64_t ny, int64_t nz, double spacing_m,
                              const double origin_m[3])
{
    if (!ctx)
        return CRP_EINVAL;
    if (!data || !(dtype == CRP_F32 || dtype == CRP_F64))
        return fail(ctx, CRP_EINVAL, "grid: null data or bad dtype");
    const int64_t lim = 1ll << 20;
    if (nx < 2 || ny < 2 || nz < 2 || nx > lim || ny > lim || nz > lim)
        return fail(ctx, CRP_EINVAL, "grid: each dimension must be in [2, 2^20]");
    if (!(spacing_m > 0) || !std::isfinite(spacing_m))
        return fail(ctx, CRP_EINVAL, "grid: spacing must be positive and finite");
    double org[3] = {0, 0, 0};
    if (origin_m)
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(origin_m[a]))
                return fail(ctx, CRP_EINVAL, "grid: origin must be finite");
            org[a] = origin_m[a];
        }
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const size_t bytes = (size_t)nx * ny * nz * 3 * (dtype == CRP_F32 ? 4 : 8);
    void* owned = nullptr;
    const void* ptr = data;
    if (!on_device) {
        HIPCHK(ctx, hipMalloc(&owned, bytes));
        hipError_t e = hipMemcpy(owned, data, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(owned);
            return fail(ctx, CRP_EDEVICE, std::string("grid upload: ") + hipGetErrorString(e));
        }
        ptr = owned;
    }
    if (ctx->grid_owned)
        (void)hipFree(ctx->grid_owned);
    free_corner(ctx);
    free_patches(ctx);
    ctx->grid_owned = owned;
    ctx->grid = ptr;
    ctx->grid_dtype = dtype;
    ctx->gn[0] = nx;
    ctx->gn[1] = ny;
    ctx->gn[2] = nz;
    ctx->spacing = spacing_m;
    for (int a = 0; a < 3; ++a)
        ctx->origin[a] = org[a];
    ctx->has_grid = true;
    return CRP_OK;
}

crp_status crp_set_field_patches(crp_ctx* ctx, int32_t n, const crp_grid_patch* patches)
{
    if (!ctx || n < 0 || n > MAX_PATCHES || (n > 0 && !patches))
        return CRP_EINVAL;
    if (!ctx->has_grid)
        return fail(ctx, CRP_ESTATE, "patches: set the base grid first");
    const int64_t lim = 1ll << 20;
    for (int k = 0; k < n; ++k) {
        const crp_grid_patch& q = patches[k];
        if (!q.data || !(q.refine == 2 || q.refine == 4 || q.refine == 8 || q.refine == 16))
            return fail(ctx, CRP_EINVAL, "patches: null data or refine not in {2, 4, 8, 16}");
        for (int a = 0; a < 3; ++a)
            if (q.n[a] < 2 || q.n[a] > lim || q.offset[a] < 0 ||
                q.offset[a] * q.refine + q.n[a] - 1 > ctx->gn[a] * q.refine)
                return fail(ctx, CRP_EINVAL,
                            "patches: each patch needs 2..2^20 vertices per axis and must lie "
                            "inside one period of the base grid");
        if (q.n[0] * q.n[1] * q.n[2] >= (1ll << 31) / 3)
            return fail(ctx, CRP_EINVAL, "patches: at most 2^31/3 - 1 vertices per patch");
    }
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    free_patches(ctx);
    NestView nv{};
    const size_t el = ctx->grid_dtype == CRP_F32 ? 4 : 8;
    for (int k = 0; k < n; ++k) {
        const crp_grid_patch& q = patches[k];
        const size_t bytes = (size_t)q.n[0] * q.n[1] * q.n[2] * 3 * el;
        const void* ptr = q.data;
        if (!q.on_device) {
            void* owned = nullptr;
            hipError_t e = hipMalloc(&owned, bytes);
            if (e == hipSuccess)
                e = hipMemcpy(owned, q.data, bytes, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                if (owned)
                    (void)hipFree(owned);
                free_patches(ctx);
                return fail(ctx, e == hipErrorOutOfMemory ? CRP_ENOMEM : CRP_EDEVICE,
                            std::string("patch upload: ") + hipGetErrorString(e));
            }
            ctx->patch_owned[k] = owned;
            ptr = owned;
        }
        PatchView& v = nv.p[k];
        v.data = ptr;
        for (int a = 0; a < 3; ++a) {
            v.n[a] = (int)q.n[a];
            v.off[a] = (int)q.offset[a];
        }
        v.stride[0] = q.n[1] * q.n[2] * 3;
        v.stride[1] = q.n[2] * 3;
        v.refine = (double)q.refine;
    }
    nv.np = n;
    ctx->nest = nv;
    return CRP_OK;
}

crp_status crp_set_field_analytic(crp_ctx* ctx, const crp_analytic_field* f)
{
    if (!ctx || !f)
        return CRP_EINVAL;
    const double vals[] = {f->center[0], f->center[1], f->center[2], f->b_disk, f->b_halo, f->b_x};
    for (double v : vals)
        if (!std::isfinite(v))
            return fail(ctx, CRP_EINVAL, "analytic field: values must be finite");
    const double lens[] = {f->r_disk, f->h_disk, f->r_halo, f->h_halo, f->r_x, f->h_x};
    for (double v : lens)
        if (!(v > 0) || !std::isfinite(v))
            return fail(ctx, CRP_EINVAL, "analytic field: radii and heights must be positive");
    AnalyticParams& a = ctx->ana;
    for (int k = 0; k < 3; ++k)
        a.center[k] = f->center[k];
    a.b_disk = f->b_disk;
    a.r_disk = f->r_disk;
    a.b_halo = f->b_halo;
    a.r_halo = f->r_halo;
    a.b_x = f->b_x;
    a.kd = 1.0 / (f->r_disk * f->r_disk);
    a.ld = 1.0 / (f->h_disk * f->h_disk);
    a.kh = 1.0 / (f->r_halo * f->r_halo);
    a.lh = 1.0 / (f->h_halo * f->h_halo);
    a.ih = 1.0 / f->h_halo;
    a.kx = 1.0 / (f->r_x * f->r_x);
    a.lx = 1.0 / (f->h_x * f->h_x);
    ctx->has_analytic = true;
    return CRP_OK;
}

crp_status crp_set_tables(crp_ctx* ctx, int32_t n, const double* e, const double* tpi,
                          const double* tn, const double* bp)
{
    if (!ctx)
        return CRP_EINVAL;
    if (n < 2 || n > 1024 || !e || !tpi || !tn || !bp)
        return fail(ctx, CRP_EINVAL, "tables: need 2 <= n <= 1024 and non-null arrays");
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(e[i]) || !(e[i] > 0))
            return fail(ctx, CRP_EINVAL, "tables: nodes must be positive and finite");
        if (i > 0 && !(e[i] > e[i - 1]))
            return fail(ctx, CRP_EINVAL, "tables: nodes must be strictly increasing");
        for (const double* v : {tpi, tn, bp})
            if (!std::isfinite(v[i]) || v[i] < 0)
                return fail(ctx, CRP_EINVAL, "tables: values must be finite and >= 0");
    }
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<double> h((size_t)4 * n);
    std::memcpy(h.data(), e, n * sizeof(double));
    std::memcpy(h.data() + n, tpi, n * sizeof(double));
    std::memcpy(h.data() + 2 * n, tn, n * sizeof(double));
    std::memcpy(h.data() + 3 * n, bp, n * sizeof(double));
    if (ctx->tab)
        (void)hipFree(ctx->tab);
    ctx->tab = nullptr;
    ctx->has_tables = false;
    HIPCHK(ctx, hipMalloc((void**)&ctx->tab, h.size() * sizeof(double)));
    HIPCHK(ctx, hipMemcpy(ctx->tab, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    ctx->tab_n = n;
    ctx->lg0 = (float)std::log2(e[0]);
    ctx->lgscale = (float)((double)(n - 1) / (std::log2(e[n - 1]) - std::log2(e[0])));
    ctx->has_tables = true;
    return CRP_OK;
}

static std::string bad_candidate(int64_t i, const int32_t* A, const int32_t* Z, const double* E,
                                 const double* pos, const double* dir, const double* lmax,
                                 double max_extent)
{
    char buf[256];
    if (!(A[i] >= 1 && A[i] <= 255 && Z[i] >= 1 && Z[i] <= A[i]))
        snprintf(buf, sizeof buf, "inject: candidate %lld: need 1 <= Z <= A <= 255 (A=%d Z=%d)",
                 (long long)i, A[i], Z[i]);
    else if (!(std::isfinite(E[i]) && E[i] > 0))
        snprintf(buf, sizeof buf, "inject: candidate %lld: energy must be finite and > 0",
                 (long long)i);
    else if (!(std::isfinite(lmax[i]) && lmax[i] > 0))
        snprintf(buf, sizeof buf, "inject: candidate %lld: lmax must be finite and > 0",
                 (long long)i);
    else {
        double d2 = 0, p2 = 0;
        bool fin = true;
        for (int a = 0; a < 3; ++a) {
            fin = fin && std::isfinite(pos[3 * i + a]) && std::isfinite(dir[3 * i + a]);
            d2 += dir[3 * i + a] * dir[3 * i + a];
            p2 += pos[3 * i + a] * pos[3 * i + a];
        }
        if (!fin)
            snprintf(buf, sizeof buf, "inject: candidate %lld: non-finite position/direction",
                     (long long)i);
        else if (std::fabs(std::sqrt(d2) - 1.0) > 1e-12)
            snprintf(buf, sizeof buf, "inject: candidate %lld: |dir| must be 1 within 1e-12",
                     (long long)i);
        else if (!(std::sqrt(p2) + lmax[i] < max_extent))
            snprintf(buf, sizeof buf,
                     "inject: candidate %lld: |pos| + lmax must stay below 2^30 grid cells",
                     (long long)i);
        else
            snprintf(buf, sizeof buf, "inject: candidate %lld is invalid", (long long)i);
    }
    return buf;
}

// The longest-expected-path-first order of a validated batch (device arrays):
// a stable radix sort of the keys of k_inject_keys; *perm (in the context's
// grow-only buffer) lists the input index of each queue slot in turn.
crp_status inject_order_perm(crp_ctx* ctx, int64_t n, const int32_t* Z, const double* E,
                             const double* lmax, const uint32_t** perm)
{
    const int ni = (int)n;
    size_t tmp = 0;
    HIPCHK(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (unsigned long long*)nullptr,
                                                   (unsigned long long*)nullptr,
                                                   (uint32_t*)nullptr, (uint32_t*)nullptr, ni, 0,
                                                   64, ctx->stream));
    const size_t kb = ((size_t)n * 8 + 255) & ~(size_t)255;
    const size_t ib = ((size_t)n * 4 + 255) & ~(size_t)255;
    const size_t need = 2 * kb + 2 * ib + tmp;
    if (need > ctx->order_bytes) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->order_mem)
            (void)hipFree(ctx->order_mem);
        ctx->order_mem = nullptr;
        ctx->order_bytes = 0;
        HIPCHK(ctx, hipMalloc(&ctx->order_mem, need));
        ctx->order_bytes = need;
    }
    char* p = (char*)ctx->order_mem;
    auto* keys = (unsigned long long*)p;
    auto* keys_sorted = (unsigned long long*)(p + kb);
    auto* idx = (uint32_t*)(p + 2 * kb);
    auto* idx_sorted = (uint32_t*)(p + 2 * kb + ib);
    void* temp = p + 2 * kb + 2 * ib;
    k_inject_keys<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, Z, E, lmax, keys, idx);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipcub::DeviceRadixSort::SortPairs(temp, tmp, keys, keys_sorted, idx, idx_sorted,
                                                   ni, 0, 64, ctx->stream));
    *perm = idx_sorted;
    return CRP_OK;
}

crp_status crp_inject(crp_ctx* ctx, int64_t n, const uint32_t* id, const int32_t* A,
                      const int32_t* Z, const double* E, const double* pos, const double* dir,
                      const double* lmax, int32_t on_device)
{
    if (!ctx)
        return CRP_EINVAL;
    if (n < 0)
        return fail(ctx, CRP_EINVAL, "inject: n must be >= 0");
    if (n == 0)
        return CRP_OK;
    if (!id || !A || !Z || !E || !pos || !dir || !lmax)
        return fail(ctx, CRP_EINVAL, "inject: null array");
    const bool analytic = ctx->cfg.field_mode == CRP_FIELD_ANALYTIC;
    if (analytic ? !ctx->has_analytic : !ctx->has_grid)
        return fail(ctx, CRP_ESTATE, "inject: set the field first");
    if (ctx->pending + n > ctx->q.cap)
        return fail(ctx, CRP_EQUEUE, "inject: queue capacity exceeded");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    // the grid's cell indices bound the reach of a candidate; the analytic
    // field has no such bound
    const double max_extent =
        analytic ? HUGE_VAL : std::ldexp(1.0, 30) * ctx->spacing;
    const uint32_t* d_id = id;
    const int32_t *d_A = A, *d_Z = Z;
    const double *d_E = E, *d_pos = pos, *d_dir = dir, *d_lmax = lmax;
    void* stage = nullptr;
    if (!on_device) {
        for (int64_t i = 0; i < n; ++i) {
            bool ok = A[i] >= 1 && A[i] <= 255 && Z[i] >= 1 && Z[i] <= A[i] &&
                      std::isfinite(E[i]) && E[i] > 0 && std::isfinite(lmax[i]) && lmax[i] > 0;
            double d2 = 0, p2 = 0;
            for (int a = 0; a < 3 && ok; ++a) {
                ok = std::isfinite(pos[3 * i + a]) && std::isfinite(dir[3 * i + a]);
                d2 += dir[3 * i + a] * dir[3 * i + a];
                p2 += pos[3 * i + a] * pos[3 * i + a];
            }
            ok = ok && std::fabs(std::sqrt(d2) - 1.0) <= 1e-12 &&
                 std::sqrt(p2) + lmax[i] < max_extent;
            if (!ok)
                return fail(ctx, CRP_EINVAL, bad_candidate(i, A, Z, E, pos, dir, lmax, max_extent));
        }
        const size_t bytes = (size_t)n * (4 + 4 + 4 + 8 + 24 + 24 + 8) + 7 * 256;
        HIPCHK(ctx, hipMalloc(&stage, bytes));
        Carver cv{(char*)stage};
        uint32_t* s_id = cv.take<uint32_t>(n);
        int32_t* s_A = cv.take<int32_t>(n);
        int32_t* s_Z = cv.take<int32_t>(n);
        double* s_E = cv.take<double>(n);
        double* s_pos = cv.take<double>(3 * n);
        double* s_dir = cv.take<double>(3 * n);
        double* s_lmax = cv.take<double>(n);
        hipError_t e = hipSuccess;
        auto up = [&](void* d, const void* h, size_t b) {
            if (e == hipSuccess)
                e = hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, ctx->stream);
        };
        up(s_id, id, n * 4);
        up(s_A, A, n * 4);
        up(s_Z, Z, n * 4);
        up(s_E, E, n * 8);
        up(s_pos, pos, n * 24);
        up(s_dir, dir, n * 24);
        up(s_lmax, lmax, n * 8);
        if (e != hipSuccess) {
            (void)hipFree(stage);
            return fail(ctx, CRP_EDEVICE, std::string("inject upload: ") + hipGetErrorString(e));
        }
        d_id = s_id;
        d_A = s_A;
        d_Z = s_Z;
        d_E = s_E;
        d_pos = s_pos;
        d_dir = s_dir;
        d_lmax = s_lmax;
    } else {
        const unsigned long long none = ~0ull;
        HIPCHK(ctx, hipMemcpyAsync(ctx->scratch, &none, 8, hipMemcpyHostToDevice, ctx->stream));
        k_validate<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, id, A, Z, E, pos, dir, lmax,
                                                                 max_extent, ctx->scratch);
        HIPCHK(ctx, hipGetLastError());
        unsigned long long bad = 0;
        HIPCHK(ctx, hipMemcpyAsync(&bad, ctx->scratch, 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (bad != ~0ull)
            return fail(ctx, CRP_EINVAL,
                        "inject: candidate " + std::to_string(bad) + " is invalid (device input)");
    }
    const uint32_t* perm = nullptr;
    if (ctx->cfg.inject_order == CRP_ORDER_LONGEST_FIRST && n > 1 && n <= INT32_MAX) {
        const crp_status st = inject_order_perm(ctx, n, d_Z, d_E, d_lmax, &perm);
        if (st != CRP_OK) {
            if (stage)
                (void)hipFree(stage);
            return st;
        }
    }
    k_inject<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(
        ctx->q, ctx->pending, n, d_id, d_A, d_Z, d_E, d_pos, d_dir, d_lmax, perm, ctx->cfg.seed,
        ctx->cfg.hmin, ctx->cfg.precision == CRP_MIX ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (stage)
        (void)hipFree(stage);
    if (e != hipSuccess)
        return fail(ctx, CRP_EDEVICE, std::string("inject: ") + hipGetErrorString(e));
    ctx->pending += n;
    return CRP_OK;
}

crp_status crp_propagate(crp_ctx* ctx, int64_t max_cycles)
{
    if (!ctx)
        return CRP_EINVAL;
    if (!ctx->has_grid && ctx->cfg.field_mode == CRP_FIELD_GRID)
        return fail(ctx, CRP_ESTATE, "propagate: no field grid");
    if (!ctx->has_analytic && ctx->cfg.field_mode == CRP_FIELD_ANALYTIC)
        return fail(ctx, CRP_ESTATE, "propagate: no analytic field");
    if (!ctx->has_tables)
        return fail(ctx, CRP_ESTATE, "propagate: no tables");
    if (ctx->cfg.field_mode == CRP_FIELD_NEURAL && !ctx->nf)
        return fail(ctx, CRP_ESTATE, "propagate: neural field not initialised");
    ctx->last_ms = 0.0;
    ctx->last_launches = 0;
    if (ctx->pending == 0)
        return CRP_OK;
    if (ctx->fin_unread > ctx->q.cap)
        return fail(ctx, CRP_ESTATE, "propagate: read finished records first");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    for (;;) {
        DevCounters dc;
        const crp_status st = run_kernel(ctx, max_cycles, &dc);
        if (st != CRP_OK)
            return st;
        after_run(ctx, dc, true);
        if (dc.neutral_deferred > 0)
            // the neutral records stay until read: the caller drains them
            return fail(ctx, CRP_EOVERFLOW,
                        "propagate: the neutral-record buffer is full (" +
                            std::to_string(dc.neutral_deferred) +
                            " interactions wait for a slot); read neutral records and "
                            "propagate again (nothing was lost)");
        if (dc.queue_deferred == 0)
            break;
        // secondaries found the queue full: their parents wait, parked just
        // before the interaction; double the queue and go on
        const crp_status g = grow_queue(ctx, 2 * ctx->q.cap);
        if (g != CRP_OK)
            return g;
        if (max_cycles > 0)
            break;   // a cycle budget ends the call; the next call resumes
    }
    return ctx->pending > 0 ? CRP_INCOMPLETE : CRP_OK;
}

crp_status crp_read_finished(crp_ctx* ctx, int64_t cap, const crp_finished_soa* out,
                             int64_t* n_out)
{
    if (!ctx || cap < 0 || !n_out)
        return CRP_EINVAL;
    const int64_t k = std::min(cap, ctx->fin_unread);
    const int64_t s = ctx->fin_unread - k;
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    if (out && k > 0) {
        const FinishedSoA& f = ctx->fin;
        HIPCHK(ctx, copy_d2h(out->id, f.id + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->lineage, f.lineage + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->m, f.m + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->nsteps, f.nsteps + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->nrej, f.nrej + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->status, f.status + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->A, f.A + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->Z, f.Z + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->E, f.E + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->L, f.L + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->E0, f.E0 + s, k, ctx->stream));
        if (out->x)
            HIPCHK(ctx, copy_planar(ctx, out->x, f.x, f.cap, s, k));
        if (out->u)
            HIPCHK(ctx, copy_planar(ctx, out->u, f.u, f.cap, s, k));
        if (out->u0)
            HIPCHK(ctx, copy_planar(ctx, out->u0, f.u0, f.cap, s, k));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    ctx->fin_unread -= k;
    *n_out = k;
    return ctx->fin_unread > 0 ? CRP_EOVERFLOW : CRP_OK;
}

crp_status crp_read_neutral(crp_ctx* ctx, int64_t cap, const crp_neutral_soa* out,
                            int64_t* n_out)
{
    if (!ctx || cap < 0 || !n_out)
        return CRP_EINVAL;
    const int64_t k = std::min(cap, ctx->neu_unread);
    const int64_t s = ctx->neu_unread - k;
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    if (out && k > 0) {
        const NeutralSoA& f = ctx->neu;
        HIPCHK(ctx, copy_d2h(out->id, f.id + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->lineage, f.lineage + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->m, f.m + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->chan, f.chan + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->E, f.E + s, k, ctx->stream));
        if (out->x)
            HIPCHK(ctx, copy_planar(ctx, out->x, f.x, f.cap, s, k));
        if (out->u)
            HIPCHK(ctx, copy_planar(ctx, out->u, f.u, f.cap, s, k));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    ctx->neu_unread -= k;
    *n_out = k;
    return ctx->neu_unread > 0 ? CRP_EOVERFLOW : CRP_OK;
}

crp_status crp_read_trajectory(crp_ctx* ctx, int64_t cap, const crp_traj_soa* out,
                               int64_t* n_out)
{
    if (!ctx || cap < 0 || !n_out)
        return CRP_EINVAL;
    const int64_t k = std::min(cap, ctx->traj_unread);
    const int64_t s = ctx->traj_unread - k;
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    if (out && k > 0) {
        const TrajSoA& t = ctx->traj;
        HIPCHK(ctx, copy_d2h(out->id, t.id + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->lineage, t.lineage + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->n, t.n + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->A, t.A + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->L, t.L + s, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->E, t.E + s, k, ctx->stream));
        if (out->x)
            HIPCHK(ctx, copy_planar(ctx, out->x, t.x, t.cap, s, k));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    ctx->traj_unread -= k;
    *n_out = k;
    return ctx->traj_unread > 0 ? CRP_EOVERFLOW : CRP_OK;
}

// ---- observables ----------------------------------------------------------
crp_status crp_set_observables(crp_ctx* ctx, const crp_observables* sp)
{
    if (!ctx || !sp)
        return CRP_EINVAL;
    const crp_observables& o = *sp;
    if (o.n_e < 1 || o.n_e > OBS_MAX_E || o.n_groups < 1 || o.n_groups > OBS_MAX_G ||
        o.n_e * o.n_groups > OBS_MAX_BINS || !o.e_edges || !o.a_edges || o.sky_n < 0 ||
        o.sky_n > 512 || !(o.sky_sign == 1.0 || o.sky_sign == -1.0) || !(o.e_ref > 0) ||
        !std::isfinite(o.e_ref) || !std::isfinite(o.gamma))
        return fail(ctx, CRP_EINVAL, "observables: bad bin counts, edges or parameters");
    for (int i = 0; i <= o.n_e; ++i)
        if (!std::isfinite(o.e_edges[i]) || (i > 0 && !(o.e_edges[i] > o.e_edges[i - 1])))
            return fail(ctx, CRP_EINVAL, "observables: energy edges must increase strictly");
    for (int i = 1; i <= o.n_groups; ++i)
        if (!(o.a_edges[i] > o.a_edges[i - 1]))
            return fail(ctx, CRP_EINVAL, "observables: mass edges must increase strictly");
    const size_t nb = (size_t)o.n_e * (size_t)o.n_groups;
    const size_t nsky = nb * 6 * (size_t)o.sky_n * (size_t)o.sky_n;
    if (nsky > ((size_t)1 << 27))
        return fail(ctx, CRP_EINVAL, "observables: sky map larger than 2^27 entries");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->obs_mem) {
        (void)hipFree(ctx->obs_mem);
        ctx->obs_mem = nullptr;
        ctx->has_obs = false;
    }
    Carver c{nullptr};
    c.take<double>(o.n_e + 1);
    c.take<int32_t>(o.n_groups + 1);
    c.take<unsigned long long>(nb);
    c.take<unsigned long long>(nb);
    c.take<double>(nb);
    c.take<unsigned long long>(nsky);
    c.take<unsigned long long>(1);
    const size_t bytes = c.off;
    HIPCHK(ctx, hipMalloc(&ctx->obs_mem, bytes));
    Carver d{(char*)ctx->obs_mem};
    ObsParams& p = ctx->obs_p;
    p = ObsParams{};
    double* ee = d.take<double>(o.n_e + 1);
    int32_t* ae = d.take<int32_t>(o.n_groups + 1);
    p.e_edges = ee;
    p.a_edges = ae;
    p.counts = d.take<unsigned long long>(nb);
    p.defl = d.take<unsigned long long>(nb);
    p.wsum = d.take<double>(nb);
    p.sky = d.take<unsigned long long>(nsky);
    p.outside = d.take<unsigned long long>(1);
    p.ne = o.n_e;
    p.ng = o.n_groups;
    p.sky_n = o.sky_n;
    p.status_mask = (uint32_t)o.status_mask;
    p.sky_sign = o.sky_sign;
    p.e_ref = o.e_ref;
    p.gamma = o.gamma;
    HIPCHK(ctx, hipMemsetAsync(ctx->obs_mem, 0, bytes, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ee, o.e_edges, (o.n_e + 1) * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ae, o.a_edges, (o.n_groups + 1) * sizeof(int32_t),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->obs = o;
    ctx->obs.e_edges = nullptr;   // the host arrays are not kept
    ctx->obs.a_edges = nullptr;
    ctx->obs_sky_n = nsky;
    ctx->has_obs = true;
    return CRP_OK;
}

crp_status crp_observe(crp_ctx* ctx, double* kernel_ms)
{
    if (!ctx)
        return CRP_EINVAL;
    if (!ctx->has_obs)
        return fail(ctx, CRP_ESTATE, "observe: call crp_set_observables first");
    if (kernel_ms)
        *kernel_ms = 0.0;
    if (ctx->fin_unread == 0)
        return CRP_OK;
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    ObsParams p = ctx->obs_p;
    const FinishedSoA& f = ctx->fin;
    p.E = f.E;
    p.E0 = f.E0;
    p.u = f.u;
    p.u0 = f.u0;
    p.status = f.status;
    p.A = f.A;
    p.cap = f.cap;
    p.n = ctx->fin_unread;
    // enough blocks for 8 waves per SIMD where the records allow; each block
    // flushes its LDS bins once
    const int64_t want = (p.n + 1023) / 1024;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->num_cus * 8));
    const size_t lds = observe_lds_bytes(p.ne, p.ng);
    HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    k_observe<<<nb, 256, lds, ctx->stream>>>(p);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (kernel_ms)
        *kernel_ms = ms;
    return CRP_OK;
}

crp_status crp_read_observables(crp_ctx* ctx, uint64_t* counts, double* wsum, uint64_t* defl,
                                uint64_t* sky, uint64_t* outside)
{
    if (!ctx)
        return CRP_EINVAL;
    if (!ctx->has_obs)
        return fail(ctx, CRP_ESTATE, "read_observables: call crp_set_observables first");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    const ObsParams& p = ctx->obs_p;
    const int64_t nb = (int64_t)p.ne * p.ng;
    HIPCHK(ctx, copy_d2h((unsigned long long*)counts, p.counts, nb, ctx->stream));
    HIPCHK(ctx, copy_d2h(wsum, p.wsum, nb, ctx->stream));
    HIPCHK(ctx, copy_d2h((unsigned long long*)defl, p.defl, nb, ctx->stream));
    HIPCHK(ctx, copy_d2h((unsigned long long*)sky, p.sky, (int64_t)ctx->obs_sky_n, ctx->stream));
    HIPCHK(ctx, copy_d2h((unsigned long long*)outside, p.outside, 1, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return CRP_OK;
}

// ---- galactic lenses --------------------------------------------------------
crp_status crp_lens_build(crp_ctx* ctx, const crp_lens_spec* sp, int64_t* nnz, double* kernel_ms)
{
    if (!ctx || !sp || !nnz)
        return CRP_EINVAL;
    if (sp->n_r < 1 || sp->n_r > 256 || sp->sky_n < 1 || sp->sky_n > 512 || !sp->r_edges)
        return fail(ctx, CRP_EINVAL, "lens: 1 <= n_r <= 256, 1 <= sky_n <= 512, edges needed");
    for (int i = 0; i <= sp->n_r; ++i)
        if (!std::isfinite(sp->r_edges[i]) || (i > 0 && !(sp->r_edges[i] > sp->r_edges[i - 1])))
            return fail(ctx, CRP_EINVAL, "lens: rigidity edges must increase strictly");
    if (ctx->fin_unread > (int64_t)INT32_MAX)
        return fail(ctx, CRP_EINVAL, "lens: at most 2^31 - 1 records");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    double* edges = nullptr;
    HIPCHK(ctx, hipMalloc((void**)&edges, (sp->n_r + 1) * sizeof(double)));
    hipError_t e = hipMemcpyAsync(edges, sp->r_edges, (sp->n_r + 1) * sizeof(double),
                                  hipMemcpyHostToDevice, ctx->stream);
    LensKeyParams kp;
    const FinishedSoA& f = ctx->fin;
    kp.E0 = f.E0;
    kp.u = f.u;
    kp.u0 = f.u0;
    kp.status = f.status;
    kp.Z = f.Z;
    kp.cap = f.cap;
    kp.n = ctx->fin_unread;
    kp.r_edges = edges;
    kp.n_r = sp->n_r;
    kp.sky_n = sp->sky_n;
    kp.npix = 6 * sp->sky_n * sp->sky_n;
    kp.status_mask = (uint32_t)sp->status_mask;
    kp.no_key = (unsigned long long)kp.n_r * (unsigned long long)kp.npix *
                (unsigned long long)kp.npix;
    ctx->has_lens = false;
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = lens_build(ctx->lens, kp, (int64_t)kp.n_r * kp.npix, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess)
        e = hipEventSynchronize(ctx->ev1);
    float ms = 0.f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    (void)hipFree(edges);
    if (e != hipSuccess)
        return fail(ctx, e == hipErrorOutOfMemory ? CRP_ENOMEM : CRP_EDEVICE,
                    std::string("lens build: ") + hipGetErrorString(e));
    ctx->has_lens = true;
    *nnz = ctx->lens.nnz;
    if (kernel_ms)
        *kernel_ms = ms;
    return CRP_OK;
}

crp_status crp_lens_read(crp_ctx* ctx, int64_t* rowptr, int32_t* col, double* val,
                         uint64_t* count)
{
    if (!ctx)
        return CRP_EINVAL;
    if (!ctx->has_lens)
        return fail(ctx, CRP_ESTATE, "lens_read: no lens built");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    const Lens& L = ctx->lens;
    HIPCHK(ctx, copy_d2h(rowptr, L.rowptr, L.nrows + 1, ctx->stream));
    HIPCHK(ctx, copy_d2h(col, L.col, L.nnz, ctx->stream));
    HIPCHK(ctx, copy_d2h(val, L.val, L.nnz, ctx->stream));
    HIPCHK(ctx, copy_d2h((unsigned long long*)count, L.count, L.nnz, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return CRP_OK;
}

crp_status crp_lens_apply(crp_ctx* ctx, int32_t n_maps, const double* x, double* y,
                          int32_t on_device, double* kernel_ms)
{
    if (!ctx || n_maps < 0 || n_maps > 65535 || (n_maps > 0 && (!x || !y)))
        return CRP_EINVAL;
    if (!ctx->has_lens)
        return fail(ctx, CRP_ESTATE, "lens_apply: no lens built");
    if (kernel_ms)
        *kernel_ms = 0.0;
    if (n_maps == 0)
        return CRP_OK;
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    Lens& L = ctx->lens;
    const size_t bytes = (size_t)n_maps * (size_t)L.nrows * sizeof(double);
    const double* dx = x;
    double* dy = y;
    void* stage = nullptr;
    hipError_t e = hipSuccess;
    if (!on_device) {
        HIPCHK(ctx, hipMalloc(&stage, 2 * bytes));
        dx = (const double*)stage;
        dy = (double*)((char*)stage + bytes);
        e = hipMemcpyAsync((void*)dx, x, bytes, hipMemcpyHostToDevice, ctx->stream);
    }
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = lens_apply(L, n_maps, dx, dy, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(y, dy, bytes, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    float ms = 0.f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    if (stage)
        (void)hipFree(stage);
    if (e != hipSuccess)
        return fail(ctx, CRP_EDEVICE, std::string("lens apply: ") + hipGetErrorString(e));
    if (kernel_ms)
        *kernel_ms = ms;
    return CRP_OK;
}

crp_status crp_peek_pending(crp_ctx* ctx, int64_t cap, const crp_finished_soa* out,
                            int64_t* n_out)
{
    if (!ctx || cap < 0 || !n_out)
        return CRP_EINVAL;
    const int64_t k = std::min(cap, ctx->pending);
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    if (out && k > 0) {
        const QueueSoA& q = ctx->q;
        HIPCHK(ctx, copy_d2h(out->id, q.id, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->lineage, q.lineage, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->m, q.m, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->nsteps, q.nsteps, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->nrej, q.nrej, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->A, q.A, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->Z, q.Z, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->E, q.E, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->L, q.L, k, ctx->stream));
        HIPCHK(ctx, copy_d2h(out->E0, q.E0, k, ctx->stream));
        if (out->x)
            HIPCHK(ctx, copy_planar(ctx, out->x, q.x, q.cap, 0, k));
        if (out->u)
            HIPCHK(ctx, copy_planar(ctx, out->u, q.u, q.cap, 0, k));
        if (out->u0)
            HIPCHK(ctx, copy_planar(ctx, out->u0, q.u0, q.cap, 0, k));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (out->status)
            for (int64_t i = 0; i < k; ++i)
                out->status[i] = CRP_ACTIVE;
    }
    *n_out = k;
    return CRP_OK;
}

crp_status crp_counts(crp_ctx* ctx, crp_counters* out)
{
    if (!ctx || !out)
        return CRP_EINVAL;
    *out = ctx->totals;
    out->pending = ctx->pending;
    out->finished_unread = ctx->fin_unread;
    out->neutral_unread = ctx->neu_unread;
    out->traj_unread = ctx->traj_unread;
    return CRP_OK;
}

crp_status crp_reset_counters(crp_ctx* ctx)
{
    if (!ctx)
        return CRP_EINVAL;
    std::memset(&ctx->totals, 0, sizeof ctx->totals);
    return CRP_OK;
}

crp_status crp_eval_field(crp_ctx* ctx, int64_t n, const double* pos, double* B, int32_t mode,
                          int32_t on_device)
{
    if (!ctx || n < 0 || (n > 0 && (!pos || !B)))
        return CRP_EINVAL;
    if (n == 0)
        return CRP_OK;
    crp_status st = eval_field_check(ctx, mode, "eval_field");
    if (st != CRP_OK)
        return st;
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    const double* dpos = pos;
    double* dB = B;
    void* stage = nullptr;
    if (!on_device) {
        HIPCHK(ctx, hipMalloc(&stage, (size_t)n * 48));
        dpos = (const double*)stage;
        dB = (double*)stage + 3 * n;
    }
    hipError_t e = on_device ? hipSuccess
                             : hipMemcpyAsync((void*)dpos, pos, n * 24, hipMemcpyHostToDevice,
                                              ctx->stream);
    if (e == hipSuccess) {
        st = eval_field_launch(ctx, n, dpos, dB, mode);
        if (st != CRP_OK) {
            if (stage)
                (void)hipFree(stage);
            return fail(ctx, st, "eval_field: neural evaluation failed");
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(B, dB, n * 24, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (stage)
        (void)hipFree(stage);
    if (e != hipSuccess)
        return fail(ctx, CRP_EDEVICE, std::string("eval_field: ") + hipGetErrorString(e));
    return CRP_OK;
}

crp_status crp_eval_field_noalloc(crp_ctx* ctx, int64_t n, const double* pos, double* B,
                                  int32_t mode)
{
    if (!ctx || n < 0 || (n > 0 && (!pos || !B)))
        return CRP_EINVAL;
    if (n > CRP_EVAL_NOALLOC_MAX)
        return fail(ctx, CRP_EINVAL,
                    "eval_field_noalloc: more than CRP_EVAL_NOALLOC_MAX (262144) points");
    if (n == 0)
        return CRP_OK;
    crp_status st = eval_field_check(ctx, mode, "eval_field_noalloc");
    if (st != CRP_OK)
        return st;
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    // the device's copy of the static staging array, looked up at crp_create
    double* sp = scratch_ptr(ctx->cfg.device);
    if (!sp)
        return fail(ctx, CRP_EDEVICE, "eval_field_noalloc: static scratch not set up");
    double* dpos = sp;
    double* dB = sp + 3 * CRP_EVAL_NOALLOC_MAX;
    hipError_t e = hipMemcpyAsync(dpos, pos, n * 24, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        st = eval_field_launch(ctx, n, dpos, dB, mode);
        if (st != CRP_OK)
            return fail(ctx, st, "eval_field_noalloc: neural evaluation failed");
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(B, dB, n * 24, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return fail(ctx, CRP_EDEVICE,
                    std::string("eval_field_noalloc: ") + hipGetErrorString(e));
    return CRP_OK;
}

crp_status crp_set_launch(crp_ctx* ctx, const crp_launch* l)
{
    if (!ctx || !l)
        return CRP_EINVAL;
    if (!(l->block == 128 || l->block == 256) || l->blocks_per_cu < 0 ||
        l->blocks_per_cu > 64 || l->refill < 1 || l->refill > 64 ||
        !(l->layout == CRP_LAYOUT_LINEAR || l->layout == CRP_LAYOUT_CORNER))
        return fail(ctx, CRP_EINVAL, "set_launch: invalid launch shape");
    ctx->launch = *l;
    return CRP_OK;
}

crp_status crp_get_launch(crp_ctx* ctx, crp_launch* l)
{
    if (!ctx || !l)
        return CRP_EINVAL;
    *l = ctx->launch;
    return CRP_OK;
}

crp_status crp_last_timing(crp_ctx* ctx, double* kernel_ms, int64_t* launches)
{
    if (!ctx)
        return CRP_EINVAL;
    if (kernel_ms)
        *kernel_ms = ctx->last_ms;
    if (launches)
        *launches = ctx->last_launches;
    return CRP_OK;
}

// ---- diagnostic: the gather pattern alone -------------------------------
crp_status crp_gather_ceiling(crp_ctx* ctx, int32_t iters, double* records_per_s)
{
    if (!ctx || !records_per_s || iters < 1)
        return CRP_EINVAL;
    if (!ctx->has_grid)
        return fail(ctx, CRP_ESTATE, "gather_ceiling: set the grid first");
    if (ctx->gn[0] * ctx->gn[1] * ctx->gn[2] > (int64_t)UINT32_MAX)
        return fail(ctx, CRP_EINVAL, "gather_ceiling: at most 2^32 - 1 cells");
    if (ctx->grid_dtype != CRP_F32)
        return fail(ctx, CRP_EINVAL, "gather_ceiling: FP32 grids only (128-byte records)");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    crp_status st = ensure_corner(ctx);
    if (st != CRP_OK)
        return st;
    const int bpc = ctx->launch.blocks_per_cu > 0 ? ctx->launch.blocks_per_cu : 4;
    const int nb = ctx->num_cus * bpc;
    float* sink = nullptr;
    HIPCHK(ctx, hipMalloc((void**)&sink, (size_t)nb * 128 * sizeof(float)));
    const uint32_t ncell = (uint32_t)(ctx->gn[0] * ctx->gn[1] * ctx->gn[2]);
    hipError_t e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess) {
        k_gather_ceiling<<<nb, 128, 0, ctx->stream>>>(ctx->corner, ncell, iters, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess)
        e = hipEventSynchronize(ctx->ev1);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    (void)hipFree(sink);
    if (e != hipSuccess)
        return fail(ctx, CRP_EDEVICE, std::string("gather_ceiling: ") + hipGetErrorString(e));
    *records_per_s = (double)nb * 128.0 * (double)iters / ((double)ms * 1e-3);
    return CRP_OK;
}

// ---- autotuner ----------------------------------------------------------
crp_status crp_tune(crp_ctx* ctx, int64_t max_cycles, const char* cache_path, crp_launch* best,
                    double* best_rate)
{
    if (!ctx)
        return CRP_EINVAL;
    if (!ctx->has_grid || !ctx->has_tables)
        return fail(ctx, CRP_ESTATE, "tune: set grid and tables first");
    if (ctx->cfg.field_mode != CRP_FIELD_GRID)
        return fail(ctx, CRP_ESTATE, "tune: grid field mode only");
    // a shape tuned earlier for this device, grid, element type, precision
    // and field mode: taken from the cache without trials (the latest entry)
    const std::string key = tune_key(ctx);
    if (cache_path) {
        crp_launch cached;
        double rate = 0.0;
        if (tune_cache_lookup(cache_path, key, &cached, &rate)) {
            ctx->launch = cached;
            if (best)
                *best = cached;
            if (best_rate)
                *best_rate = rate;
            return CRP_OK;
        }
    }
    if (ctx->pending == 0)
        return fail(ctx, CRP_ESTATE, "tune: inject a calibration batch first");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    // back up the pending queue: slots [0, pending) of every array
    const int64_t np = ctx->pending;
    const size_t qbytes = queue_layout(nullptr, ctx->q.cap, nullptr);
    void* backup = nullptr;
    HIPCHK(ctx, hipMalloc(&backup, qbytes));
    {
        hipError_t e =
            hipMemcpyAsync(backup, ctx->qmem[0], qbytes, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            (void)hipFree(backup);
            return fail(ctx, CRP_EDEVICE, std::string("tune: ") + hipGetErrorString(e));
        }
    }
    const crp_launch orig = ctx->launch;
    const int64_t fin0 = ctx->fin_unread, neu0 = ctx->neu_unread, traj0 = ctx->traj_unread;
    crp_launch bestl = orig;
    double bestr = -1.0;
    crp_status st = CRP_OK;
    // every shape is timed twice on the same work and keeps its better rate
    // (a single short trial is too noisy to separate shapes a few % apart)
    auto trial = [&](const crp_launch& l) {
        for (int rep = 0; rep < 2 && st == CRP_OK; ++rep) {
            // restore the queue (the park buffer swap may have moved it)
            ctx->q = QueueSoA();
            queue_layout((char*)ctx->qmem[0], ctx->park.cap, &ctx->q);
            const hipError_t e = hipMemcpyAsync(ctx->qmem[0], backup, qbytes,
                                                hipMemcpyDeviceToDevice, ctx->stream);
            if (e != hipSuccess) {
                st = fail(ctx, CRP_EDEVICE, std::string("tune: ") + hipGetErrorString(e));
                break;
            }
            queue_layout((char*)ctx->qmem[1], ctx->park.cap, &ctx->park);
            ctx->pending = np;
            ctx->fin_unread = fin0;
            ctx->neu_unread = neu0;
            ctx->traj_unread = traj0;
            ctx->launch = l;
            DevCounters dc;
            st = run_kernel(ctx, max_cycles, &dc);
            if (st != CRP_OK)
                break;
            const double rate =
                ctx->last_ms > 0 ? (double)dc.steps / (ctx->last_ms * 1e-3) : 0.0;
            if (rate > bestr) {
                bestr = rate;
                bestl = l;
            }
        }
    };
    // stage 1: block size, occupancy and refill on both layouts (the
    // multi-resolution kernel of an FP64 grid has no corner-record form; a grid
    // whose records do not fit in device memory, or that has 2^32 cells or
    // more, is tuned on the linear layout alone)
    bool corner_ok = ctx->grid_dtype == CRP_F32 || ctx->nest.np == 0;
    if (corner_ok) {
        const crp_status cs = ensure_corner(ctx);
        if (cs == CRP_ENOMEM || cs == CRP_EINVAL) {
            corner_ok = false;
            ctx->err.clear();   // not an error of the tuning
        }
        else if (cs != CRP_OK)
            st = cs;
    }
    for (int layout = 0; layout < (corner_ok ? 2 : 1) && st == CRP_OK; ++layout)
        for (const crp_launch& l : {crp_launch{128, 0, 4, 0}, crp_launch{128, 0, 16, 0},
                                    crp_launch{128, 3, 4, 0}, crp_launch{256, 0, 4, 0},
                                    crp_launch{256, 0, 16, 0}})
            if (st == CRP_OK)
                trial(crp_launch{l.block, l.blocks_per_cu, l.refill, layout});
    // stage 2, around the best: the extreme refill thresholds (claim as soon as
    // one lane idles, or only when the whole wave has) and two blocks per CU
    if (st == CRP_OK) {
        const crp_launch c = bestl;
        for (const crp_launch& l : {crp_launch{c.block, c.blocks_per_cu, 1, c.layout},
                                    crp_launch{c.block, c.blocks_per_cu, 64, c.layout},
                                    crp_launch{c.block, 2, c.refill, c.layout}})
            if (st == CRP_OK && !(l.blocks_per_cu == c.blocks_per_cu && l.refill == c.refill))
                trial(l);
    }
    // restore the pending work exactly as it was
    queue_layout((char*)ctx->qmem[0], ctx->park.cap, &ctx->q);
    queue_layout((char*)ctx->qmem[1], ctx->park.cap, &ctx->park);
    (void)hipMemcpyAsync(ctx->qmem[0], backup, qbytes, hipMemcpyDeviceToDevice, ctx->stream);
    (void)hipMemsetAsync(ctx->q.ready, 0, ctx->q.cap * sizeof(uint32_t), ctx->stream);
    (void)hipMemsetAsync(ctx->park.ready, 0, ctx->park.cap * sizeof(uint32_t), ctx->stream);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(backup);
    ctx->pending = np;
    ctx->fin_unread = fin0;
    ctx->neu_unread = neu0;
    ctx->traj_unread = traj0;
    if (st != CRP_OK) {
        ctx->launch = orig;
        return st;
    }
    ctx->launch = bestl;
    if (best)
        *best = bestl;
    if (best_rate)
        *best_rate = bestr;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s : block=%d blocks_per_cu=%d refill=%d layout=%d steps_per_s=%.6e\n",
                    key.c_str(), bestl.block, bestl.blocks_per_cu, bestl.refill, bestl.layout,
                    bestr);
            fclose(f);
        }
    }
    return CRP_OK;
}

}  // extern "C"

// ---- checkpoint -----------------------------------------------------------
namespace {
const uint64_t kMagic = 0x32504b43505243ull;  // "CRPCKP2"
struct SnapHeader {
    uint64_t magic;
    int64_t pending, fin_unread, neu_unread, traj_unread;
    int32_t precision, pad;
    crp_counters totals;
};

template <class T>
void put(std::vector<char>& b, const T* d, int64_t n, hipStream_t s)
{
    const size_t off = b.size();
    b.resize(off + n * sizeof(T));
    if (n)
        (void)hipMemcpyAsync(b.data() + off, d, n * sizeof(T), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
}

template <class T>
bool get(const char*& p, const char* end, T* d, int64_t n, hipStream_t s)
{
    const size_t b = n * sizeof(T);
    if ((size_t)(end - p) < b)
        return false;
    if (n)
        (void)hipMemcpyAsync(d, p, b, hipMemcpyHostToDevice, s);
    (void)hipStreamSynchronize(s);
    p += b;
    return true;
}
}  // namespace

extern "C" {

crp_status crp_snapshot(crp_ctx* ctx, void** blob, size_t* bytes)
{
    if (!ctx || !blob || !bytes)
        return CRP_EINVAL;
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    std::vector<char> b(sizeof(SnapHeader));
    SnapHeader h;
    std::memset(&h, 0, sizeof h);
    h.magic = kMagic;
    h.pending = ctx->pending;
    h.fin_unread = ctx->fin_unread;
    h.neu_unread = ctx->neu_unread;
    h.traj_unread = ctx->traj_unread;
    h.precision = ctx->cfg.precision;
    h.totals = ctx->totals;
    std::memcpy(b.data(), &h, sizeof h);
    hipStream_t s = ctx->stream;
    const QueueSoA& q = ctx->q;
    const int64_t np = ctx->pending;
    for (int a = 0; a < 3; ++a) {
        put(b, q.x + a * q.cap, np, s);
        put(b, q.u + a * q.cap, np, s);
        put(b, q.u0 + a * q.cap, np, s);
    }
    for (double* p : {q.E, q.L, q.Lmax, q.hctrl, q.tau, q.E0})
        put(b, p, np, s);
    for (uint32_t* p : {q.id, q.lineage, q.m, q.nsteps, q.nrej})
        put(b, p, np, s);
    for (int32_t* p : {q.A, q.Z})
        put(b, p, np, s);
    const FinishedSoA& f = ctx->fin;
    const int64_t nf = ctx->fin_unread;
    for (int a = 0; a < 3; ++a) {
        put(b, f.x + a * f.cap, nf, s);
        put(b, f.u + a * f.cap, nf, s);
        put(b, f.u0 + a * f.cap, nf, s);
    }
    for (double* p : {f.E, f.L, f.E0})
        put(b, p, nf, s);
    for (uint32_t* p : {f.id, f.lineage, f.m, f.nsteps, f.nrej})
        put(b, p, nf, s);
    for (int32_t* p : {f.status, f.A, f.Z})
        put(b, p, nf, s);
    const NeutralSoA& n = ctx->neu;
    const int64_t nn = ctx->neu_unread;
    for (int a = 0; a < 3; ++a) {
        put(b, n.x + a * n.cap, nn, s);
        put(b, n.u + a * n.cap, nn, s);
    }
    put(b, n.E, nn, s);
    for (uint32_t* p : {n.id, n.lineage, n.m})
        put(b, p, nn, s);
    put(b, n.chan, nn, s);
    const TrajSoA& tr = ctx->traj;
    const int64_t nt = ctx->traj_unread;
    for (int a = 0; a < 3; ++a)
        put(b, tr.x + a * tr.cap, nt, s);
    for (double* p : {tr.L, tr.E})
        put(b, p, nt, s);
    for (uint32_t* p : {tr.id, tr.lineage, tr.n})
        put(b, p, nt, s);
    put(b, tr.A, nt, s);
    void* mem = std::malloc(b.size());
    if (!mem)
        return fail(ctx, CRP_ENOMEM, "snapshot: host allocation failed");
    std::memcpy(mem, b.data(), b.size());
    *blob = mem;
    *bytes = b.size();
    return CRP_OK;
}

crp_status crp_restore(crp_ctx* ctx, const void* blob, size_t bytes)
{
    if (!ctx || !blob || bytes < sizeof(SnapHeader))
        return CRP_EINVAL;
    SnapHeader h;
    std::memcpy(&h, blob, sizeof h);
    if (h.magic != kMagic || h.precision != ctx->cfg.precision)
        return fail(ctx, CRP_EINVAL, "restore: not a snapshot of this version / precision");
    if (h.pending < 0 || h.fin_unread < 0 || h.neu_unread < 0 || h.neu_unread > ctx->neu.cap ||
        h.traj_unread > ctx->traj.cap || h.traj_unread < 0)
        return fail(ctx, CRP_EINVAL, "restore: snapshot exceeds this context's capacity");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    {
        // a queue grown in the snapshotted context: grow this one to match
        int64_t cap = ctx->q.cap;
        while (cap < h.pending || 2 * cap < h.fin_unread)
            cap *= 2;
        const int64_t keep_p = ctx->pending, keep_f = ctx->fin_unread;
        ctx->pending = 0;           // nothing of this context's own state is kept
        ctx->fin_unread = 0;
        const crp_status g = grow_queue(ctx, cap);
        ctx->pending = keep_p;
        ctx->fin_unread = keep_f;
        if (g != CRP_OK)
            return g;
    }
    hipStream_t s = ctx->stream;
    const char* p = (const char*)blob + sizeof h;
    const char* end = (const char*)blob + bytes;
    bool ok = true;
    const QueueSoA& q = ctx->q;
    const int64_t np = h.pending;
    for (int a = 0; a < 3; ++a) {
        ok = ok && get(p, end, q.x + a * q.cap, np, s);
        ok = ok && get(p, end, q.u + a * q.cap, np, s);
        ok = ok && get(p, end, q.u0 + a * q.cap, np, s);
    }
    for (double* d : {q.E, q.L, q.Lmax, q.hctrl, q.tau, q.E0})
        ok = ok && get(p, end, d, np, s);
    for (uint32_t* d : {q.id, q.lineage, q.m, q.nsteps, q.nrej})
        ok = ok && get(p, end, d, np, s);
    for (int32_t* d : {q.A, q.Z})
        ok = ok && get(p, end, d, np, s);
    const FinishedSoA& f = ctx->fin;
    const int64_t nf = h.fin_unread;
    for (int a = 0; a < 3; ++a) {
        ok = ok && get(p, end, f.x + a * f.cap, nf, s);
        ok = ok && get(p, end, f.u + a * f.cap, nf, s);
        ok = ok && get(p, end, f.u0 + a * f.cap, nf, s);
    }
    for (double* d : {f.E, f.L, f.E0})
        ok = ok && get(p, end, d, nf, s);
    for (uint32_t* d : {f.id, f.lineage, f.m, f.nsteps, f.nrej})
        ok = ok && get(p, end, d, nf, s);
    for (int32_t* d : {f.status, f.A, f.Z})
        ok = ok && get(p, end, d, nf, s);
    const NeutralSoA& n = ctx->neu;
    const int64_t nn = h.neu_unread;
    for (int a = 0; a < 3; ++a) {
        ok = ok && get(p, end, n.x + a * n.cap, nn, s);
        ok = ok && get(p, end, n.u + a * n.cap, nn, s);
    }
    ok = ok && get(p, end, n.E, nn, s);
    for (uint32_t* d : {n.id, n.lineage, n.m})
        ok = ok && get(p, end, d, nn, s);
    ok = ok && get(p, end, n.chan, nn, s);
    const TrajSoA& tr = ctx->traj;
    const int64_t nt = h.traj_unread;
    for (int a = 0; a < 3; ++a)
        ok = ok && get(p, end, tr.x + a * tr.cap, nt, s);
    for (double* d : {tr.L, tr.E})
        ok = ok && get(p, end, d, nt, s);
    for (uint32_t* d : {tr.id, tr.lineage, tr.n})
        ok = ok && get(p, end, d, nt, s);
    ok = ok && get(p, end, tr.A, nt, s);
    if (!ok || p != end)
        return fail(ctx, CRP_EINVAL, "restore: truncated or oversized snapshot");
    ctx->pending = h.pending;
    ctx->fin_unread = h.fin_unread;
    ctx->neu_unread = h.neu_unread;
    ctx->traj_unread = h.traj_unread;
    ctx->totals = h.totals;
    return CRP_OK;
}

void crp_free(void* p) { std::free(p); }

// ---- neural field entry points (implemented in crp_nf.hip) ---------------
crp_status crp_nf_init(crp_ctx* ctx, const int32_t* freq, const float* params, double b_scale)
{
    if (!ctx || !freq || !params || !(b_scale > 0))
        return CRP_EINVAL;
    if (!ctx->has_grid)
        return fail(ctx, CRP_ESTATE, "nf_init: set the field grid first (period and origin)");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    if (!ctx->nf) {
        ctx->nf = nf_create(ctx->stream);
        if (!ctx->nf)
            return fail(ctx, CRP_ENOMEM, "nf_init: allocation failed");
    }
    const crp_status st = nf_load(ctx->nf, freq, params, b_scale, ctx->err);
    if (st != CRP_OK) {
        nf_destroy(ctx->nf);
        ctx->nf = nullptr;
    }
    return st;
}

crp_status crp_nf_get_params(crp_ctx* ctx, float* params)
{
    if (!ctx || !params)
        return CRP_EINVAL;
    if (!ctx->nf)
        return fail(ctx, CRP_ESTATE, "nf: not initialised");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    return nf_get(ctx->nf, params, ctx->err);
}

crp_status crp_nf_loss_grad(crp_ctx* ctx, int64_t n, const double* pos, const float* target,
                            float* out, float* grad, double* loss)
{
    if (!ctx || n <= 0 || !pos || !target)
        return CRP_EINVAL;
    if (!ctx->nf)
        return fail(ctx, CRP_ESTATE, "nf: not initialised");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    return nf_loss_grad(ctx->nf, make_view(ctx), n, pos, target, out, grad, loss, ctx->err);
}

crp_status crp_nf_train(crp_ctx* ctx, int64_t steps, int64_t batch, double lr0, double lr1,
                        uint64_t seed, float* loss_out)
{
    if (!ctx || steps < 0 || batch <= 0 || !(lr0 > 0) || !(lr1 > 0))
        return CRP_EINVAL;
    if (!ctx->nf)
        return fail(ctx, CRP_ESTATE, "nf: not initialised");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    return nf_train(ctx->nf, make_view(ctx), steps, batch, lr0, lr1, seed, loss_out, ctx->err);
}

crp_status crp_nf_adam_step(crp_ctx* ctx, const float* grad, double lr)
{
    if (!ctx || !grad || !(lr > 0) || !std::isfinite(lr))
        return CRP_EINVAL;
    if (!ctx->nf)
        return fail(ctx, CRP_ESTATE, "nf: not initialised");
    for (int i = 0; i < CRP_NF_NPARAM; ++i)
        if (!std::isfinite(grad[i]))
            return fail(ctx, CRP_EINVAL, "nf_adam_step: non-finite gradient");
    HIPCHK(ctx, hipSetDevice(ctx->cfg.device));
    return nf_adam_step(ctx->nf, grad, lr, ctx->err);
}

}  // extern "C"

