// Galactic lenses: device buffers and kernel parameters shared by the lens
// kernels (crp_lens.hip) and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crp {

// A lens set in CSR form: row r Np + i (rigidity bin r, Earth pixel i), columns
// the border pixels j in increasing order.
struct Lens {
    int64_t* rowptr = nullptr;          // [nrows + 1]
    int32_t* col = nullptr;             // [nnz]
    double* val = nullptr;              // [nnz]
    unsigned long long* count = nullptr;   // [nnz] records behind each entry
    int64_t nrows = 0, nnz = 0;
    int npix = 0, n_r = 0;
    int lpr = 4;                        // lanes per row of the application kernel
    // construction scratch, kept (grow-only) between builds, and the matrix
    // buffers' capacities (also grow-only)
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    int64_t cap_rows = 0, cap_nnz = 0;
    // application scratch (grow-only): border maps interleaved by pixel
    double* xt = nullptr;
    int64_t xt_cap = 0;                 // doubles
};

struct LensKeyParams {
    const double *E0, *u, *u0;          // finished records (u, u0 planar [3][cap])
    const int32_t *status, *Z;
    int64_t cap, n;
    const double* r_edges;              // device [n_r + 1]
    int n_r, sky_n, npix;
    uint32_t status_mask;
    unsigned long long no_key;          // n_r Np Np: the key of a record that takes no part
};

struct LensApplyParams {
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
    const double* x;                    // [n_maps][nrows]
    double* y;                          // [n_maps][nrows]
    int64_t nrows, map_len;
    int64_t npix;
    int64_t n_maps;
};

hipError_t lens_build(Lens& L, const LensKeyParams& kp, int64_t nrows, hipStream_t s);
hipError_t lens_apply(Lens& L, int n_maps, const double* x, double* y, hipStream_t s);
void lens_free(Lens& L);           // the matrix buffers
void lens_free_scratch(Lens& L);   // construction and application scratch

}  // namespace crp
