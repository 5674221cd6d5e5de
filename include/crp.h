/*
 * crp.h -- C-ABI of the MI355X propagation library (libcrp.so).
 *
 * The library steps cosmic-ray candidates (nuclei) through a periodic
 * magnetic-field grid on one GPU.  Each candidate carries all of its own
 * state (paper, section 3, "cosmic ray candidate and modules"), so candidates
 * are independent lanes of one persistent GPU kernel.  Every cycle of a
 * candidate runs, in the order of Fig. 1 of the paper:
 *   1. integration: an adaptive Cash-Karp 4(5) step of the Lorentz force
 *      dx/ds = u, du/ds = (Z c / E) u x B(x), with B from periodic trilinear
 *      interpolation of the grid;
 *   2. interactions: a continuous relative energy loss (pair-production-like)
 *      and stochastic interactions decided per step by an optical-depth clock
 *      that is reset after every interaction (section 3);
 *   3. boundary / observer checks: detection inside an observer sphere, the
 *      maximum trajectory length, an energy floor; the active flag is checked
 *      after each cycle.
 * Secondaries: a nucleon-loss event spawns a charged proton candidate that is
 * propagated in the same run; a pion-like event emits a neutral record.
 * Field sources: the periodic grid (optionally with refinement patches: a
 * multi-resolution grid), an analytic galactic field for backtracking
 * (section 4), or a learned neural field.  Outputs: finished and neutral
 * records, per-step trajectory points, observable sums (spectra, deflection,
 * sky maps) and galactic lenses built from backtracked records (section 4).
 *
 * Units at this ABI: metres, eV, tesla; rates in 1/m.
 * Threading: one context per host thread; calls on one context must not
 * overlap.  All functions return a crp_status; no C++ exception crosses the
 * ABI.  After an error, crp_last_error(ctx) describes it.
 */
#ifndef CRP_H
#define CRP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRP_OK = 0,
    CRP_INCOMPLETE = 1,   /* propagate: cycle budget used up with candidates left */
    CRP_EOVERFLOW = 2,    /* read: more records remain than fit in the buffer;
                             propagate: stopped with the neutral-record buffer
                             full (read neutral records, then propagate again) */
    CRP_EINVAL = -1,      /* invalid argument (nothing was changed)               */
    CRP_EDEVICE = -2,     /* HIP runtime error                                    */
    CRP_ENOMEM = -3,      /* device allocation failed                             */
    CRP_ESTATE = -4,      /* call not valid in this state (e.g. no field/tables)  */
    CRP_EQUEUE = -5       /* inject: queue capacity exceeded                       */
} crp_status;

enum { CRP_FP64 = 0, CRP_MIX = 1 };                     /* stage precision        */
enum { CRP_FIELD_GRID = 0, CRP_FIELD_NEURAL = 1, CRP_FIELD_ANALYTIC = 2 }; /* field source */
enum { CRP_F32 = 0, CRP_F64 = 1 };                      /* grid element type      */
enum { CRP_LAYOUT_LINEAR = 0, CRP_LAYOUT_CORNER = 1 };  /* grid layout in HBM     */
enum { CRP_ACTIVE = 0, CRP_OBSERVED = 1, CRP_MAX_TRAJ = 2, CRP_ENERGY_FLOOR = 3,
       CRP_BOUNDARY = 4 };
enum { CRP_CHAN_PI = 0, CRP_CHAN_N = 1 };
enum { CRP_ORDER_LONGEST_FIRST = 0, CRP_ORDER_AS_GIVEN = 1 };   /* crp_config.inject_order */

/* Run configuration (copied at crp_create). */
typedef struct {
    int32_t precision;        /* CRP_FP64: every operation FP64.  CRP_MIX: RK stage
                                 increments, field interpolation and direction in
                                 FP32; position, length, step control, energy and
                                 interactions in FP64. */
    int32_t field_mode;       /* CRP_FIELD_GRID, CRP_FIELD_NEURAL (needs crp_nf_init and
                                 precision CRP_MIX) or CRP_FIELD_ANALYTIC (needs
                                 crp_set_field_analytic) */
    int32_t renormalize;      /* 1: |u| renormalised after every accepted step */
    int32_t device;           /* HIP device ordinal */
    double tol;               /* direction error tolerance per step */
    double hmin, hmax;        /* step-size controller bounds, m (0 < hmin <= hmax) */
    double eps_loss;          /* max relative continuous loss per step (> 0) */
    double kappa_pi;          /* energy fraction of one nucleon lost in a pion-like event */
    double e_floor;           /* candidates below this energy (eV) stop */
    double obs_center[3];     /* observer sphere centre, m */
    double obs_radius;        /* observer radius, m; 0 disables the observer */
    uint64_t seed;            /* Philox4x64-10 key word 0 */
    int64_t queue_capacity;   /* initial work-queue capacity: pending + spawned
                                 candidates (> 0).  Injection beyond it is refused;
                                 secondaries that do not fit make the queue double
                                 during crp_propagate (their parents wait) */
    int64_t neutral_capacity; /* max undrained neutral records (> 0) */
    int32_t charge_sign;      /* +1 (or 0): forward tracking; -1: backtracking, i.e. the
                                 antiparticle (charge -Z) from the observer along the
                                 reversed arrival direction (section 4) */
    int32_t inject_order;     /* CRP_ORDER_LONGEST_FIRST (0): crp_inject queues each
                                 batch in order of decreasing lmax * Z / E (the path
                                 length in units of the rigidity, which grows with the
                                 number of curvature-limited steps), so that the
                                 persistent kernel starts the longest trajectories
                                 first; CRP_ORDER_AS_GIVEN (1): in the caller's order.
                                 Results do not depend on it. */
    double boundary_center[3];/* spherical boundary centre, m */
    double boundary_radius;   /* m; 0 disables it.  A candidate at or beyond the radius
                                 after a cycle stops with status CRP_BOUNDARY */
    int32_t traj_every;       /* per-step trajectory output (section 3: output modules
                                 can record a candidate after every step): a point is
                                 recorded after the cycle of every traj_every-th
                                 accepted step and after the cycle that ends the
                                 candidate; 0 disables it (>= 0) */
    uint32_t traj_ids;        /* only candidates with id < traj_ids are recorded */
    int64_t traj_capacity;    /* max undrained trajectory points (> 0 if traj_every > 0);
                                 points beyond it are dropped and counted */
} crp_config;

/* Analytic galactic field (section 4: the code offers analytic field models;
 * the JF12 fit parameters are not available, so this is a synthetic model of
 * the same disk / halo / X-field structure with rational profiles).
 * Cylindrical coordinates about `center`, axis z; tesla and metres:
 *   disk toroidal  B_phi = b_disk (r/r_disk) / ((1 + r^2/r_disk^2)(1 + z^2/h_disk^2))
 *   halo toroidal  B_phi = b_halo (z/h_halo)(r/r_halo) / ((1 + r^2/r_halo^2)(1 + z^2/h_halo^2)^2)
 *   X-field        B = curl(A_phi e_phi), A_phi = b_x r / (2 D),
 *                  D = 1 + r^2/r_x^2 + z^2/h_x^2
 * evaluated in FP64 (the precision form rounds the result to FP32). */
typedef struct {
    double center[3];
    double b_disk, r_disk, h_disk;
    double b_halo, r_halo, h_halo;
    double b_x, r_x, h_x;
} crp_analytic_field;

/* Kernel launch shape of the persistent propagation kernel. */
typedef struct {
    int32_t block;            /* threads per block: 128 or 256 */
    int32_t blocks_per_cu;    /* persistent blocks per compute unit (1..64), or 0:
                                 as many as the kernel's occupancy lets one
                                 compute unit hold at once */
    int32_t refill;           /* a wave claims new candidates once this many of its
                                 64 lanes are idle (1..64) */
    int32_t layout;           /* CRP_LAYOUT_LINEAR or CRP_LAYOUT_CORNER */
} crp_launch;

/* Caller-allocated host arrays for finished candidates ([n] or [n][3]). */
typedef struct {
    uint32_t *id, *lineage, *m, *nsteps, *nrej;
    int32_t *status, *A, *Z;
    double *E, *x, *u, *L, *u0, *E0;
} crp_finished_soa;

/* Caller-allocated host arrays for neutral secondary records. */
typedef struct {
    uint32_t *id, *lineage, *m;
    int32_t* chan;
    double *E, *x, *u;
} crp_neutral_soa;

/* Caller-allocated host arrays for trajectory points ([n] or [n][3]): the
 * candidate key (id, lineage), n = its accepted steps so far, its mass number,
 * trajectory length, energy and position after that step's cycle. */
typedef struct {
    uint32_t *id, *lineage, *n;
    int32_t* A;
    double *L, *E, *x;
} crp_traj_soa;

/* Observables of finished records (the reductions of the paper's section 5
 * application: energy spectrum, mean deflection against energy, sky maps).
 * A record with status s takes part if bit s of status_mask is set.  Its
 * energy bin e has e_edges[e] <= E < e_edges[e + 1] and its mass group g has
 * a_edges[g] <= A < a_edges[g + 1]; records outside either range (or with a
 * zero direction when there is a sky map) are only counted in `outside`.
 * Per (g, e) the library sums: the record count; the weight (E0 / e_ref)^gamma
 * (E0 the source energy: gamma reweights the injected spectrum, FP64 sum in
 * an unspecified order); the deflection, the angle between the initial and
 * final directions a = u/|u|, b = u0/|u0|, 2 atan2(|a - b|, |a + b|), as
 * floor(angle * 2^32) in 64-bit fixed point (order-independent); and, with
 * sky_n > 0, a cube-map sky map of v = sky_sign * u: face 2m + (v_m < 0) for
 * the axis m of largest |v_m| (the lowest on ties), on it s = v_p / |v_m| and
 * t = v_q / |v_m| for the other two axes p < q, pixel
 * (i, j) = (floor(((s + 1) / 2) sky_n), floor(((t + 1) / 2) sky_n)) clamped
 * to sky_n - 1, index (face * sky_n + i) * sky_n + j. */
typedef struct {
    int32_t n_e;              /* energy bins, 1..256 */
    int32_t n_groups;         /* mass groups, 1..16; n_e * n_groups <= 1024 */
    const double* e_edges;    /* [n_e + 1] eV, strictly increasing (host) */
    const int32_t* a_edges;   /* [n_groups + 1], strictly increasing (host) */
    int32_t status_mask;      /* bit s: records with status s take part */
    int32_t sky_n;            /* cube-map face resolution 0..512 (0: no sky map);
                                 n_groups * n_e * 6 sky_n^2 <= 2^27 */
    double sky_sign;          /* +1 or -1 (-1: the arrival direction -u) */
    double e_ref;             /* > 0, eV */
    double gamma;             /* finite */
} crp_observables;

/* Cumulative integer bookkeeping since crp_create (or crp_reset_counters). */
typedef struct {
    int64_t finished, observed, max_traj, energy_floor;
    int64_t steps, attempts, rejects, forced;
    int64_t events, null_events, inter_pi, inter_n;
    int64_t charged_sec, neutral_sec;
    int64_t queue_deferred;   /* interactions whose secondary found the queue full:
                                 the parent waited (parked just before the
                                 interaction) and finished its cycle after the
                                 queue grew; nothing is dropped */
    int64_t neutral_deferred; /* interactions that found the neutral-record buffer
                                 full: the parent waits until the records are read */
    int64_t pending;          /* candidates waiting for the next propagate */
    int64_t finished_unread, neutral_unread;
    int64_t lane_slots;       /* 64 x wave iterations of the propagation kernel:
                                 attempts / lane_slots is the fraction of lanes
                                 that carried a candidate */
    int64_t boundary;         /* candidates stopped by the spherical boundary */
    int64_t traj_points;      /* trajectory points recorded */
    int64_t traj_dropped;     /* trajectory points dropped (capacity) */
    int64_t traj_unread;      /* recorded points not yet read */
} crp_counters;

typedef struct crp_ctx crp_ctx;

/* Creates a context on cfg->device.  stream: a hipStream_t borrowed for all
 * work of this context (NULL: the default stream).  The library allocates and
 * owns every device buffer it uses.  Errors: CRP_EINVAL (bad config),
 * CRP_EDEVICE, CRP_ENOMEM. */
crp_status crp_create(const crp_config* cfg, void* stream, crp_ctx** out);
void crp_destroy(crp_ctx* ctx);

/* Field grid: [nx][ny][nz][3] tesla, C order, vertex (i,j,k) at
 * origin + (i,j,k) * spacing, periodic with period n * spacing on each axis
 * (section 4 of the paper: precomputed grids for fast lookup; trilinear
 * interpolation is this library's reading).  dtype: CRP_F32 or CRP_F64.
 * on_device = 0: host data is copied.  on_device = 1: the device pointer is
 * used in place until replaced or the context is destroyed (the caller keeps
 * it alive).  Errors: CRP_EINVAL (dims < 2, > 2^20, bad dtype/spacing),
 * CRP_ENOMEM. */
crp_status crp_set_field_grid(crp_ctx* ctx, const void* data, int32_t dtype, int32_t on_device,
                              int64_t nx, int64_t ny, int64_t nz, double spacing_m,
                              const double origin_m[3]);

/* Refinement patch of a multi-resolution grid (section 4: multi-resolution
 * grids give fast access to precomputed fields over a larger dynamic range).
 * A patch is a non-periodic vertex grid [n0][n1][n2][3] of the base grid's
 * element type with spacing spacing_m / refine; its vertex (0,0,0) sits on
 * base vertex `offset`, and the whole patch lies inside one period of the
 * base grid: offset[a] * refine + n[a] - 1 <= base_n[a] * refine.  It
 * repeats with the base grid's period. */
typedef struct {
    const void* data;         /* [n0][n1][n2][3] tesla, C order, the base grid's dtype */
    int64_t n[3];             /* vertices per axis, 2 .. 2^20 */
    int64_t offset[3];        /* base-grid vertex index of the patch's vertex (0,0,0), >= 0 */
    int32_t refine;           /* base cells per patch cell along each axis: 2, 4, 8 or 16 */
    int32_t on_device;        /* 0: host data, copied; 1: device pointer used in place (the
                                 caller keeps it alive while the patches are set) */
} crp_grid_patch;

/* Sets the refinement patches of the current field grid (replacing earlier
 * ones; n = 0 removes them; crp_set_field_grid removes them too).  Level
 * selection: a position p is located in the base grid (wrapped vertex index
 * i0 and offset t in cell units, as for the plain grid); patch k sees it at
 * r = ((i0 - offset) + t) * refine and holds it if 0 <= r < n - 1 on every
 * axis; the last such patch in list order gives the field, by trilinear
 * interpolation of its own vertices at r (same arithmetic as the base grid),
 * else the base grid does.  With CRP_LAYOUT_CORNER (FP32 grids) every patch
 * gets corner records too (128 bytes per patch vertex, built on first use) and
 * the wave gathers each lane's record from whichever level it selected.
 * 0 <= n <= 4.  Errors: CRP_EINVAL (limits above), CRP_ESTATE (no grid),
 * CRP_ENOMEM. */
crp_status crp_set_field_patches(crp_ctx* ctx, int32_t n, const crp_grid_patch* patches);

/* Analytic field for CRP_FIELD_ANALYTIC (model above); copied.  Radii and
 * heights must be positive and every value finite.  Errors: CRP_EINVAL. */
crp_status crp_set_field_analytic(crp_ctx* ctx, const crp_analytic_field* field);

/* Interaction tables per nucleon at eps = E/A on n strictly increasing nodes
 * (eV): pion-like rate, nucleon-loss-like rate, proton relative loss rate
 * (all 1/m, >= 0).  A nucleus (A, Z) uses R_pi = A t_pi(E/A),
 * R_N = A t_n(E/A) if A >= 2 else 0, beta = Z^2/A beta_p(E/A); values are
 * linear in E between nodes and clamped outside.  2 <= n <= 1024.  Copied.
 * Errors: CRP_EINVAL. */
crp_status crp_set_tables(crp_ctx* ctx, int32_t n, const double* e_nodes_eV,
                          const double* t_pi_per_m, const double* t_n_per_m,
                          const double* beta_p_per_m);

/* Appends n candidates (all-or-nothing) to the pending queue: id (unique per
 * context, the caller's contract), 1 <= Z <= A <= 255, E > 0 (eV), pos [n][3]
 * (m), dir [n][3] with | |dir| - 1 | <= 1e-12, lmax > 0 (m, trajectory
 * length limit); values finite; |pos| + lmax < 2^30 grid cells.  Pointers are
 * host memory (on_device = 0) or device memory (on_device = 1).  Injected
 * candidates start with L = 0, step h_min, event count 0, lineage 0.  The
 * batch is queued in the order crp_config.inject_order selects (sorted on the
 * device by a stable radix sort, in a grow-only buffer of 24 bytes per
 * candidate kept by the context; batches of 2^31 or more are queued as given).
 * Errors: CRP_EINVAL (first bad index in crp_last_error; only checked for
 * host input), CRP_EQUEUE (capacity), CRP_ESTATE (no field yet).  With the
 * analytic field the grid-cell bound on |pos| + lmax does not apply. */
crp_status crp_inject(crp_ctx* ctx, int64_t n, const uint32_t* id, const int32_t* A,
                      const int32_t* Z, const double* E_eV, const double* pos_m,
                      const double* dir, const double* lmax_m, int32_t on_device);

/* Propagates every pending candidate, and every secondary spawned meanwhile,
 * until it stops or has run max_cycles cycles in this call (max_cycles <= 0:
 * no limit).  Runs on the context stream and returns after it completes.
 * Nothing is dropped: a candidate whose interaction product (a secondary, or
 * a neutral record) finds no slot keeps its state from just before the
 * interaction and waits; for secondaries the queue (and the finished-record
 * buffer) doubles and the run goes on (with a cycle budget, the next call goes
 * on).  Returns CRP_INCOMPLETE if candidates remain pending (call again to
 * continue; the result is identical to an uninterrupted run), CRP_EOVERFLOW if
 * candidates wait because the neutral-record buffer is full (read neutral
 * records, then call again; the result is again identical).
 * Errors: CRP_ESTATE (no field or tables), CRP_ENOMEM (the queue could not
 * grow; the pending work is kept), CRP_EDEVICE. */
crp_status crp_propagate(crp_ctx* ctx, int64_t max_cycles);

/* Copies up to cap finished records into out and removes them from the
 * library; *n_out receives the count.  Order is unspecified: records are keyed
 * by (id, lineage).  Returns CRP_EOVERFLOW (informational) if more remain. */
crp_status crp_read_finished(crp_ctx* ctx, int64_t cap, const crp_finished_soa* out,
                             int64_t* n_out);

/* Same for neutral records, keyed by (id, lineage, m). */
crp_status crp_read_neutral(crp_ctx* ctx, int64_t cap, const crp_neutral_soa* out,
                            int64_t* n_out);

/* Copies up to cap trajectory points into out and removes them from the
 * library; *n_out receives the count.  Order is unspecified: points are keyed
 * by (id, lineage, n).  Returns CRP_EOVERFLOW (informational) if more remain. */
crp_status crp_read_trajectory(crp_ctx* ctx, int64_t cap, const crp_traj_soa* out,
                               int64_t* n_out);

/* Sets the observable binning (copied) and clears the sums; the sums live in
 * device memory owned by the context.  Errors: CRP_EINVAL (limits above),
 * CRP_ENOMEM. */
crp_status crp_set_observables(crp_ctx* ctx, const crp_observables* spec);

/* Adds every unread finished record to the observable sums, on the context
 * stream; the records stay unread.  kernel_ms (nullable) receives the
 * reduction kernel's duration.  Errors: CRP_ESTATE (no crp_set_observables). */
crp_status crp_observe(crp_ctx* ctx, double* kernel_ms);

/* Copies the sums (host arrays, each nullable): counts, wsum and defl
 * [n_groups][n_e]; sky [n_groups][n_e][6 sky_n^2]; *outside. */
crp_status crp_read_observables(crp_ctx* ctx, uint64_t* counts, double* wsum, uint64_t* defl,
                                uint64_t* sky, uint64_t* outside);

/* Galactic lenses (section 4: the lensing technique maps the directions of
 * cosmic rays at the border of the Galaxy to directions observed at Earth
 * with one transformation matrix per energy range).  Built here from the
 * unread finished records of a backtracking run (charge_sign = -1, a
 * spherical boundary): a record with status s takes part if bit s of
 * status_mask is set and its rigidity E0 / Z lies in a bin
 * r_edges[r] <= E0 / Z < r_edges[r + 1].  Its Earth pixel i is the cube-map
 * pixel (the map of crp_observables, sky_n x sky_n per face, Np = 6 sky_n^2)
 * of its launch direction u0 (the arrival direction) and its border pixel j
 * that of its final direction u (the direction it came from, seen at the
 * border).  Lens r: L_r[i][j] = c_r(i, j) / sum_j' c_r(i, j') with c_r the
 * number of such records; rows without records are zero. */
typedef struct {
    int32_t n_r;              /* rigidity bins, 1..256 */
    int32_t sky_n;            /* cube-map face resolution, 1..512 */
    const double* r_edges;    /* [n_r + 1] rigidity edges (eV per unit charge), strictly
                                 increasing (host) */
    int32_t status_mask;      /* normally 1 << CRP_BOUNDARY */
    int32_t pad_;
} crp_lens_spec;

/* Builds the lens set from the unread finished records (they stay unread),
 * replacing an earlier one; the lenses live in device memory owned by the
 * context, as one CSR matrix of n_r * Np rows (row r * Np + i), Np columns,
 * entries of a row in increasing column order, FP64 values.  *nnz receives
 * the number of entries; kernel_ms (nullable) the device time of the build.
 * Errors: CRP_EINVAL (spec; more than 2^31 - 1 records), CRP_ENOMEM,
 * CRP_EDEVICE. */
crp_status crp_lens_build(crp_ctx* ctx, const crp_lens_spec* spec, int64_t* nnz,
                          double* kernel_ms);

/* Copies the lens set to host arrays (each nullable): rowptr [n_r Np + 1],
 * col [nnz], val [nnz], count [nnz] (records behind each entry).
 * Errors: CRP_ESTATE (no lens built). */
crp_status crp_lens_read(crp_ctx* ctx, int64_t* rowptr, int32_t* col, double* val,
                         uint64_t* count);

/* Applies the lenses to n_maps border maps: x [n_maps][n_r][Np] gives
 * y [n_maps][n_r][Np], y[m][r][i] = sum_j L_r[i][j] x[m][r][j] (FP64; the
 * order of the sum over j is unspecified).  Pointers are host (on_device = 0)
 * or device memory; kernel_ms (nullable) receives the kernel's duration.
 * Errors: CRP_ESTATE (no lens), CRP_EINVAL. */
crp_status crp_lens_apply(crp_ctx* ctx, int32_t n_maps, const double* x, double* y,
                          int32_t on_device, double* kernel_ms);

/* Copies up to cap pending (interrupted) candidates as records with status
 * CRP_ACTIVE, without removing them. */
crp_status crp_peek_pending(crp_ctx* ctx, int64_t cap, const crp_finished_soa* out,
                            int64_t* n_out);

crp_status crp_counts(crp_ctx* ctx, crp_counters* out);
crp_status crp_reset_counters(crp_ctx* ctx);

/* Field at n positions pos [n][3] (m) into B [n][3] (T), with the stepper's
 * own interpolation: mode CRP_FP64 (FP64 weights), CRP_MIX (FP32 weights and
 * sums), CRP_FIELD_NEURAL + 16 (the trained network) or CRP_FIELD_ANALYTIC + 16
 * (the analytic field, FP64).  Pointers are host (on_device = 0) or device
 * memory.  Errors: CRP_ESTATE, CRP_EINVAL. */
crp_status crp_eval_field(crp_ctx* ctx, int64_t n, const double* pos_m, double* B_T,
                          int32_t mode, int32_t on_device);

/* For callers that cannot allocate device memory during a call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * crp_eval_field for host arrays pos [n][3] (m) and B [n][3] (T), same modes
 * and the same kernels, bitwise the same results, staged through a static
 * device array of the library instead of a per-call allocation.  It calls no
 * hipMalloc, hipFree or other allocating routine.  Limit: n <=
 * CRP_EVAL_NOALLOC_MAX points (the static array holds 12 MiB per GPU the
 * library runs on, kept until the process ends); larger n is CRP_EINVAL with
 * nothing evaluated.  All calls on one GPU share that array: calls that
 * overlap on one GPU (from several contexts or threads) race and must be
 * serialised by the caller.  Errors: CRP_EINVAL, CRP_ESTATE, CRP_EDEVICE. */
#define CRP_EVAL_NOALLOC_MAX 262144
crp_status crp_eval_field_noalloc(crp_ctx* ctx, int64_t n, const double* pos_m, double* B_T,
                                  int32_t mode);

/* Launch shape of the propagation kernel (validated; CRP_EINVAL otherwise).
 * A new context starts with {128, 0, 4, CRP_LAYOUT_LINEAR}.
 * CRP_LAYOUT_CORNER keeps, beside the linear grid, one record per cell with
 * the cell's 8 corner vectors in the grid's element type (built on first use,
 * at most 2^32 - 1 cells): 128 bytes per cell for an FP32 grid (24 floats and
 * a pad), 192 bytes for an FP64 grid (24 doubles).  The field values read are
 * the same in either layout, so results do not depend on it.  An FP64 grid
 * with refinement patches is read from the linear arrays in either layout. */
crp_status crp_set_launch(crp_ctx* ctx, const crp_launch* launch);
crp_status crp_get_launch(crp_ctx* ctx, crp_launch* launch);

/* Autotuner: times candidate launch shapes, each twice, in two stages: block
 * 128 / 256, as many blocks per compute unit as fit or 3, refill 4 / 16, on
 * the linear and the corner layout (the corner layout only where its records
 * can be built: they fit in device memory, the grid has fewer than 2^32
 * cells, and it is not an FP64 grid with refinement patches); then, around
 * the fastest of those, refill
 * 1 and 64 and 2 blocks per compute unit.  The trials run on a copy of the
 * pending queue (restored after each trial, so the
 * pending work is unchanged) run for max_cycles cycles (<= 0: to completion),
 * keeps the fastest in the context and appends it to cache_path (NULL: no
 * file) under a key of (device name, grid shape, dtype, precision, field
 * mode).  If cache_path already holds an entry for this key, its latest shape
 * is taken without trials.  best_rate: accepted steps per second of the chosen
 * shape (from the cache when taken from it).  Needs pending work unless the
 * cache answers.  Errors: CRP_ESTATE (no grid, tables or pending work; not the
 * grid field mode), CRP_EDEVICE. */
crp_status crp_tune(crp_ctx* ctx, int64_t max_cycles, const char* cache_path,
                    crp_launch* best, double* best_rate);

/* Timing of the last crp_propagate: summed duration of its propagation
 * kernel launches (HIP events on the context stream), ms, and launch count. */
crp_status crp_last_timing(crp_ctx* ctx, double* kernel_ms, int64_t* launches);

/* Diagnostic, not a step of the method: times the field-gather pattern alone
 * (the cooperative corner-record gather of the propagation kernel) on this
 * context's corner records (built on first use, as for CRP_LAYOUT_CORNER),
 * `iters` random records per lane with the context's blocks per CU (block
 * 128).  records_per_s: gathered records per second, the practical ceiling of
 * the field evaluation.  CRP_ESTATE without a grid, CRP_EINVAL for an FP64 grid,
 * a grid of more than 2^32 - 1 cells or iters < 1. */
crp_status crp_gather_ceiling(crp_ctx* ctx, int32_t iters, double* records_per_s);

/* Checkpoint: pending candidates, undrained finished / neutral records,
 * unread trajectory points and counters (not the observable sums or lenses,
 * which are rebuilt from records).  The blob is allocated by the library and
 * released with crp_free; a blob of an earlier layout is rejected. */
crp_status crp_snapshot(crp_ctx* ctx, void** blob, size_t* bytes);
crp_status crp_restore(crp_ctx* ctx, const void* blob, size_t bytes);
void crp_free(void* p);

/* ---- neural field (learned stand-in for the trilinear gather) ----------
 * Network: xhat = frac((x - origin) / (n * spacing)); gamma = [cos 2pi F xhat,
 * sin 2pi F xhat] (F: 64 x 3 integers); four 128-wide ReLU layers; linear 3
 * outputs; B = b_scale * out.  Weights are FP32 masters, used as bfloat16 in
 * the matrix products with FP32 accumulation.  Parameter order in flat
 * buffers: W1 [128][128], b1 [128], ..., W4, b4, W5 [3][128], b5 [3]. */
#define CRP_NF_NPARAM 66435
crp_status crp_nf_init(crp_ctx* ctx, const int32_t* freq_64x3, const float* params,
                       double b_scale_T);
crp_status crp_nf_get_params(crp_ctx* ctx, float* params);
/* Forward and MSE gradient at n points (host arrays): target in units of
 * b_scale; writes out [n][3] and grad [CRP_NF_NPARAM]; loss = mean |out - t|^2. */
crp_status crp_nf_loss_grad(crp_ctx* ctx, int64_t n, const double* pos_m, const float* target,
                            float* out, float* grad, double* loss);
/* One Adam update (Kingma & Ba 2015: beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrections with the context's step count, which crp_nf_init resets and
 * every update advances) of the FP32 masters with a caller-given gradient:
 * grad [CRP_NF_NPARAM] host FP32 in the flat parameter order, e.g. the sum of
 * per-GPU crp_nf_loss_grad gradients in data-parallel training.  Errors:
 * CRP_EINVAL (non-finite gradient or lr <= 0; nothing changed), CRP_ESTATE. */
crp_status crp_nf_adam_step(crp_ctx* ctx, const float* grad, double lr);
/* Trains on points drawn uniformly in one period of the grid with targets from
 * the grid's trilinear field: steps Adam updates (beta1 0.9, beta2 0.999,
 * eps 1e-8) of batch points, cosine learning rate lr0 -> lr1.  loss_out[steps]
 * (nullable) receives each step's loss. */
crp_status crp_nf_train(crp_ctx* ctx, int64_t steps, int64_t batch, double lr0, double lr1,
                        uint64_t seed, float* loss_out);

const char* crp_last_error(const crp_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CRP_H */
