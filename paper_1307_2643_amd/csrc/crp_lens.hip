// Galactic lenses of libcrp for gfx950 (the lensing technique of the paper's
// section 4: per-energy transformation matrices mapping directions at the
// border of the Galaxy to directions observed at Earth; definitions in crp.h).
//
// Construction from the finished records of a backtracking run: one key per
// record (rigidity bin, Earth pixel of u0, border pixel of u), a device radix
// sort and run-length encoding give the distinct (row, column) entries with
// their counts in CSR order; a binary search per row gives the row pointers
// and an integer sum per row the normalisation.
//
// Application: a sparse matrix times border maps, one group of LPR lanes per
// row (LPR sized for about four entries per lane), the group's partial sums
// combined by lane shuffles; up to four maps in one pass over the matrix, more
// maps interleaved by pixel first and applied sixteen per pass.  The time goes
// to each row's dependent loads and to the per-map shuffle reductions rather
// than to the bytes streamed.
#include <hipcub/hipcub.hpp>

#include "crp_lens.hpp"

namespace crp {

// Cube-map pixel (as in crp.h for the observables), -1 for a zero vector.
__device__ inline int64_t lens_pixel(double v0, double v1, double v2, int n)
{
    const double a0 = fabs(v0), a1 = fabs(v1), a2 = fabs(v2);
    int m = 0;
    double big = a0, vm = v0, vp = v1, vq = v2;
    if (a1 > big) {
        m = 1;
        big = a1;
        vm = v1;
        vp = v0;
        vq = v2;
    }
    if (a2 > big) {
        m = 2;
        big = a2;
        vm = v2;
        vp = v0;
        vq = v1;
    }
    if (!(big > 0.0))
        return -1;
    const double s = vp / big, t = vq / big;
    double fi = floor(((s + 1.0) * 0.5) * (double)n);
    double fj = floor(((t + 1.0) * 0.5) * (double)n);
    if (fi > (double)(n - 1))
        fi = (double)(n - 1);
    if (fj > (double)(n - 1))
        fj = (double)(n - 1);
    const int64_t face = 2 * m + (vm < 0.0 ? 1 : 0);
    return (face * n + (int64_t)fi) * n + (int64_t)fj;
}

// Key (r Np + i) Np + j of every record, or no_key (one past the largest) if
// it takes no part, so that the sort needs only the key's significant bits.
__global__ void k_lens_keys(LensKeyParams p, unsigned long long* keys)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n)
        return;
    unsigned long long key = p.no_key;
    const int32_t st = p.status[k];
    if (st >= 0 && st <= 31 && ((p.status_mask >> st) & 1u) != 0u) {
        const double R = p.E0[k] / (double)p.Z[k];
        int r = -1;
        if (R >= p.r_edges[0] && R < p.r_edges[p.n_r]) {
            int lo = 0, hi = p.n_r;   // r_edges[lo] <= R < r_edges[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (p.r_edges[mid] <= R)
                    lo = mid;
                else
                    hi = mid;
            }
            r = lo;
        }
        const int64_t cap = p.cap;
        const int64_t i = lens_pixel(p.u0[k], p.u0[cap + k], p.u0[2 * cap + k], p.sky_n);
        const int64_t j = lens_pixel(p.u[k], p.u[cap + k], p.u[2 * cap + k], p.sky_n);
        if (r >= 0 && i >= 0 && j >= 0)
            key = ((unsigned long long)(r * p.npix + i)) * (unsigned long long)p.npix +
                  (unsigned long long)j;
    }
    keys[k] = key;
}

// Row pointers: the first entry whose key is at least row * Np (entries are
// sorted); an entry past nvalid holds the no-key marker.  Then each row's total
// count and every entry's column and value.
__global__ void k_lens_rows(const unsigned long long* ukeys, int64_t nvalid, int64_t nrows,
                            int npix, int64_t* rowptr)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row > nrows)
        return;
    const unsigned long long target = (unsigned long long)row * (unsigned long long)npix;
    int64_t lo = 0, hi = nvalid;   // first index with key >= target
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ukeys[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    rowptr[row] = lo;
}

__global__ void k_lens_rowsum(const uint32_t* counts, const int64_t* rowptr, int64_t nrows,
                              unsigned long long* tot)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nrows)
        return;
    unsigned long long s = 0;
    for (int64_t q = rowptr[row]; q < rowptr[row + 1]; ++q)
        s += counts[q];
    tot[row] = s;
}

__global__ void k_lens_values(const unsigned long long* ukeys, const uint32_t* counts,
                              const unsigned long long* tot, int64_t nvalid, int npix,
                              int32_t* col, double* val, unsigned long long* count)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nvalid)
        return;
    const unsigned long long key = ukeys[e];
    const int64_t row = (int64_t)(key / (unsigned long long)npix);
    col[e] = (int32_t)(key % (unsigned long long)npix);
    val[e] = (double)counts[e] / (double)tot[row];
    count[e] = counts[e];
}

// y[m][row] = sum over the row's entries of val * x[m][r Np + col], row = r Np + i,
// for LENS_MAPS maps m0, m0 + 1, ... at once (blockIdx.y = m0 / LENS_MAPS): the
// row's columns and values are read once for all of them.  Every map's sum
// has the same order whatever the number of maps applied together.
constexpr int LENS_MAPS = 4;

template <int LPR>
__global__ void __launch_bounds__(256) k_lens_apply(LensApplyParams p)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (LPR - 1);
    const int64_t group = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPR;
    const int64_t m0 = (int64_t)blockIdx.y * LENS_MAPS;
    const int nm = (int)(p.n_maps - m0 < LENS_MAPS ? p.n_maps - m0 : LENS_MAPS);
    const bool live = group < p.nrows;
    const int64_t row = live ? group : 0;
    const int64_t base = (row / p.npix) * p.npix;     // first column of this rigidity's block
    const double* x = p.x + m0 * p.map_len + base;
    double acc[LENS_MAPS] = {0.0, 0.0, 0.0, 0.0};
    if (live) {
        const int64_t e1 = p.rowptr[row + 1];
        for (int64_t e = p.rowptr[row] + sub; e < e1; e += LPR) {
            const double v = p.val[e];
            const int64_t c = p.col[e];
#pragma unroll
            for (int k = 0; k < LENS_MAPS; ++k)
                if (k < nm)
                    acc[k] += v * x[k * p.map_len + c];
        }
    }
#pragma unroll
    for (int k = 0; k < LENS_MAPS; ++k) {
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1)
            acc[k] += __shfl_xor(acc[k], o, LPR);
    }
    if (live && sub == 0) {
#pragma unroll
        for (int k = 0; k < LENS_MAPS; ++k)
            if (k < nm)
                p.y[(m0 + k) * p.map_len + row] = acc[k];
    }
}

template __global__ void k_lens_apply<4>(LensApplyParams);
template __global__ void k_lens_apply<8>(LensApplyParams);
template __global__ void k_lens_apply<16>(LensApplyParams);
template __global__ void k_lens_apply<32>(LensApplyParams);
template __global__ void k_lens_apply<64>(LensApplyParams);

// More than LENS_MAPS maps: the border maps are first interleaved by pixel,
// xt[pixel][k] for the LENS_GROUP maps of a group (128 bytes per pixel, zero
// past the last map), so that an entry's gathers for all maps of the group are
// one contiguous line instead of one request per map.  Each map's sums keep
// the order of k_lens_apply, so both paths give the same bits.
constexpr int LENS_GROUP = 16;

__global__ void k_lens_interleave(const double* __restrict__ x, int64_t map_len, int64_t m0,
                                  int nm, double* __restrict__ xt)
{
    const int64_t n = map_len * LENS_GROUP;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const int64_t i = t / LENS_GROUP;
        const int k = (int)(t - i * LENS_GROUP);
        xt[t] = k < nm ? x[(m0 + k) * map_len + i] : 0.0;
    }
}

template <int LPR>
__global__ void __launch_bounds__(256) k_lens_apply_group(LensApplyParams p, const double* xt,
                                                          int64_t m0, int nm)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int sub = lane & (LPR - 1);
    const int64_t group = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPR;
    const bool live = group < p.nrows;
    const int64_t row = live ? group : 0;
    const int64_t base = (row / p.npix) * p.npix;     // first column of this rigidity's block
    double acc[LENS_GROUP];
#pragma unroll
    for (int k = 0; k < LENS_GROUP; ++k)
        acc[k] = 0.0;
    if (live) {
        const int64_t e1 = p.rowptr[row + 1];
        for (int64_t e = p.rowptr[row] + sub; e < e1; e += LPR) {
            const double v = p.val[e];
            const double2* xp = (const double2*)(xt + (base + p.col[e]) * LENS_GROUP);
#pragma unroll
            for (int h = 0; h < LENS_GROUP / 2; ++h) {
                const double2 xv = xp[h];
                acc[2 * h] += v * xv.x;
                acc[2 * h + 1] += v * xv.y;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < LENS_GROUP; ++k) {
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1)
            acc[k] += __shfl_xor(acc[k], o, LPR);
    }
    if (live && sub == 0) {
#pragma unroll
        for (int k = 0; k < LENS_GROUP; ++k)
            if (k < nm)
                p.y[(m0 + k) * p.map_len + row] = acc[k];
    }
}

// ---- host side ---------------------------------------------------------------

namespace {
int blocks(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }
}

// Carves the construction buffers out of the lens's grow-only scratch.
static hipError_t lens_scratch(Lens& L, int64_t n, size_t tmp_bytes, int64_t nrows,
                               unsigned long long** keys, unsigned long long** sorted,
                               unsigned long long** ukeys, uint32_t** counts, int64_t** nruns,
                               unsigned long long** tot, void** tmp)
{
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_keys = up(n * sizeof(unsigned long long));
    const size_t b_counts = up(n * sizeof(uint32_t));
    const size_t b_nruns = up(sizeof(int64_t));
    const size_t b_tot = up(nrows * sizeof(unsigned long long));
    const size_t need = 3 * b_keys + b_counts + b_nruns + b_tot + up(tmp_bytes);
    if (need > L.scratch_bytes) {
        lens_free_scratch(L);
        hipError_t e = hipMalloc(&L.scratch, need);
        if (e != hipSuccess)
            return e;
        L.scratch_bytes = need;
    }
    char* p = (char*)L.scratch;
    *keys = (unsigned long long*)p;
    p += b_keys;
    *sorted = (unsigned long long*)p;
    p += b_keys;
    *ukeys = (unsigned long long*)p;
    p += b_keys;
    *counts = (uint32_t*)p;
    p += b_counts;
    *nruns = (int64_t*)p;
    p += b_nruns;
    *tot = (unsigned long long*)p;
    p += b_tot;
    *tmp = (void*)p;
    return hipSuccess;
}

// Grows a matrix buffer to at least n elements (contents not kept).
template <class T>
static hipError_t lens_grow(T** p, int64_t n, int64_t& cap)
{
    if (n <= cap && *p)
        return hipSuccess;
    if (*p)
        (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void**)p, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
    if (e == hipSuccess)
        cap = n;
    return e;
}

hipError_t lens_build(Lens& L, const LensKeyParams& kp, int64_t nrows, hipStream_t s)
{
    L.nnz = 0;
    const int64_t n = kp.n;
    L.nrows = nrows;
    L.npix = kp.npix;
    L.n_r = kp.n_r;
    hipError_t e = hipSuccess;
    auto done = [&](hipError_t r) {
        if (r != hipSuccess)
            lens_free(L);
        return r;
    };
#define LCHK(x)                  \
    do {                         \
        e = (x);                 \
        if (e != hipSuccess)     \
            return done(e);      \
    } while (0)
    {
        int64_t cap = L.cap_rows;
        LCHK(lens_grow(&L.rowptr, nrows + 1, cap));
        L.cap_rows = cap;
    }
    if (n == 0) {
        LCHK(hipMemsetAsync(L.rowptr, 0, (size_t)(nrows + 1) * sizeof(int64_t), s));
        LCHK(hipStreamSynchronize(s));
        L.nnz = 0;
        return done(hipSuccess);
    }
    // the sort needs the bits of the largest key (no_key) only
    int nbits = 1;
    while (nbits < 64 && (kp.no_key >> nbits) != 0ull)
        ++nbits;
    size_t tmp_sort = 0, tmp_rle = 0;
    LCHK(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_sort, (unsigned long long*)nullptr,
                                           (unsigned long long*)nullptr, (int)n, 0, nbits, s));
    LCHK(hipcub::DeviceRunLengthEncode::Encode(nullptr, tmp_rle, (unsigned long long*)nullptr,
                                               (unsigned long long*)nullptr, (uint32_t*)nullptr,
                                               (int64_t*)nullptr, (int)n, s));
    size_t tmp_bytes = std::max(tmp_sort, tmp_rle);
    unsigned long long *keys, *sorted, *ukeys, *tot;
    uint32_t* counts;
    int64_t* nruns_d;
    void* tmp;
    LCHK(lens_scratch(L, n, tmp_bytes, nrows, &keys, &sorted, &ukeys, &counts, &nruns_d, &tot,
                      &tmp));
    k_lens_keys<<<blocks(n, 256), 256, 0, s>>>(kp, keys);
    LCHK(hipGetLastError());
    LCHK(hipcub::DeviceRadixSort::SortKeys(tmp, tmp_sort, keys, sorted, (int)n, 0, nbits, s));
    LCHK(hipcub::DeviceRunLengthEncode::Encode(tmp, tmp_rle, sorted, ukeys, counts, nruns_d,
                                               (int)n, s));
    int64_t nruns = 0;
    unsigned long long last = 0;
    LCHK(hipMemcpyAsync(&nruns, nruns_d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LCHK(hipStreamSynchronize(s));
    if (nruns > 0) {
        LCHK(hipMemcpyAsync(&last, ukeys + nruns - 1, sizeof(last), hipMemcpyDeviceToHost, s));
        LCHK(hipStreamSynchronize(s));
    }
    const int64_t nvalid = (nruns > 0 && last == kp.no_key) ? nruns - 1 : nruns;
    L.nnz = nvalid;
    k_lens_rows<<<blocks(nrows + 1, 256), 256, 0, s>>>(ukeys, nvalid, nrows, kp.npix, L.rowptr);
    LCHK(hipGetLastError());
    if (nvalid > 0) {
        if (nvalid > L.cap_nnz || !L.col || !L.val || !L.count) {
            int64_t c1 = 0, c2 = 0, c3 = 0;   // zero capacities: reallocate all three
            L.cap_nnz = 0;
            LCHK(lens_grow(&L.col, nvalid, c1));
            LCHK(lens_grow(&L.val, nvalid, c2));
            LCHK(lens_grow(&L.count, nvalid, c3));
            L.cap_nnz = nvalid;
        }
        k_lens_rowsum<<<blocks(nrows, 256), 256, 0, s>>>(counts, L.rowptr, nrows, tot);
        LCHK(hipGetLastError());
        k_lens_values<<<blocks(nvalid, 256), 256, 0, s>>>(ukeys, counts, tot, nvalid, kp.npix,
                                                          L.col, L.val, L.count);
        LCHK(hipGetLastError());
    }
    LCHK(hipStreamSynchronize(s));
    // lanes per row: the power of two nearest above a quarter of the mean
    // filled-row length, so a lane sums ~4 entries and the cross-lane
    // reduction of each map's sum stays short (measured on 44-entry rows:
    // 16 lanes twice as fast as 64 for 1 and for 16 maps)
    L.lpr = 4;
    if (nvalid > 0) {
        const double mean = (double)nvalid / (double)std::min<int64_t>(nrows, nvalid);
        while (L.lpr < 64 && 4 * L.lpr < mean)
            L.lpr *= 2;
    }
#undef LCHK
    return done(hipSuccess);
}

hipError_t lens_apply(Lens& L, int n_maps, const double* x, double* y, hipStream_t s)
{
    LensApplyParams p;
    p.rowptr = L.rowptr;
    p.col = L.col;
    p.val = L.val;
    p.x = x;
    p.y = y;
    p.nrows = L.nrows;
    p.npix = L.npix;
    p.map_len = L.nrows;
    p.n_maps = n_maps;
    // the grouped path stages 128 bytes per row; lens sets whose staging would
    // pass 1 GiB take the four-map passes instead
    const int64_t need = L.nrows * LENS_GROUP;
    if (n_maps > LENS_MAPS && need <= (int64_t)((1ll << 30) / sizeof(double))) {
        if (need > L.xt_cap) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                return e;
            if (L.xt)
                (void)hipFree(L.xt);
            L.xt = nullptr;
            L.xt_cap = 0;
            e = hipMalloc((void**)&L.xt, (size_t)need * sizeof(double));
            if (e != hipSuccess)
                return e;
            L.xt_cap = need;
        }
        const unsigned nb = (unsigned)((L.nrows * L.lpr + 255) / 256);
        const int ib = (int)std::min<int64_t>((need + 255) / 256, 65536);
        for (int64_t m0 = 0; m0 < n_maps; m0 += LENS_GROUP) {
            const int nm = (int)std::min<int64_t>(LENS_GROUP, n_maps - m0);
            k_lens_interleave<<<ib, 256, 0, s>>>(x, L.nrows, m0, nm, L.xt);
            switch (L.lpr) {
            case 4: k_lens_apply_group<4><<<nb, 256, 0, s>>>(p, L.xt, m0, nm); break;
            case 8: k_lens_apply_group<8><<<nb, 256, 0, s>>>(p, L.xt, m0, nm); break;
            case 16: k_lens_apply_group<16><<<nb, 256, 0, s>>>(p, L.xt, m0, nm); break;
            case 32: k_lens_apply_group<32><<<nb, 256, 0, s>>>(p, L.xt, m0, nm); break;
            default: k_lens_apply_group<64><<<nb, 256, 0, s>>>(p, L.xt, m0, nm); break;
            }
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    const dim3 grid((unsigned)((L.nrows * L.lpr + 255) / 256),
                    (unsigned)((n_maps + LENS_MAPS - 1) / LENS_MAPS));
    switch (L.lpr) {
    case 4: k_lens_apply<4><<<grid, 256, 0, s>>>(p); break;
    case 8: k_lens_apply<8><<<grid, 256, 0, s>>>(p); break;
    case 16: k_lens_apply<16><<<grid, 256, 0, s>>>(p); break;
    case 32: k_lens_apply<32><<<grid, 256, 0, s>>>(p); break;
    default: k_lens_apply<64><<<grid, 256, 0, s>>>(p); break;
    }
    return hipGetLastError();
}

void lens_free_scratch(Lens& L)
{
    if (L.scratch)
        (void)hipFree(L.scratch);
    L.scratch = nullptr;
    L.scratch_bytes = 0;
    if (L.xt)
        (void)hipFree(L.xt);
    L.xt = nullptr;
    L.xt_cap = 0;
}

void lens_free(Lens& L)
{
    for (void* q : {(void*)L.rowptr, (void*)L.col, (void*)L.val, (void*)L.count})
        if (q)
            (void)hipFree(q);
    L.rowptr = nullptr;
    L.col = nullptr;
    L.val = nullptr;
    L.count = nullptr;
    L.nnz = 0;
    L.cap_rows = 0;
    L.cap_nnz = 0;
}

}  // namespace crp
