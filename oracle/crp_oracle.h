/*
 * CPU oracle of the 3D cosmic-ray propagation hot path -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, FP64 (and, for the precision form, mixed FP32/FP64) reference
 * implementation of the module cycle of the paper's section 3 (Fig. 1):
 * integration (Cash-Karp Lorentz-force step), continuous loss, stochastic
 * interactions with a reset of the interaction state after every event,
 * then boundary / observer break conditions checked after each cycle.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
 * load this library.  It shares no code with the GPU library.
 *
 * Units: metres, eV, tesla, rates in 1/m.
 */
#ifndef CRP_ORACLE_H
#define CRP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_FP64 = 0, OR_MIX = 1 };
enum { OR_GRID_F32 = 0, OR_GRID_F64 = 1 };
enum { OR_ACTIVE = 0, OR_OBSERVED = 1, OR_MAX_TRAJ = 2, OR_ENERGY_FLOOR = 3, OR_BOUNDARY = 4 };
enum { OR_CHAN_PI = 0, OR_CHAN_N = 1 };

typedef struct {
    int32_t precision;      /* OR_FP64 or OR_MIX */
    int32_t renormalize;    /* 1: |u| renormalised after each accepted step */
    double tol;             /* direction error tolerance per step */
    double hmin, hmax;      /* controller step bounds, m */
    double eps_loss;        /* max relative continuous loss per step */
    double kappa_pi;        /* inelasticity of the pion-like channel */
    double e_floor;         /* energy floor, eV */
    double obs[3];          /* observer centre, m */
    double obs_r;           /* observer radius, m (0: no observer) */
    uint64_t seed;          /* Philox key word 0 */
    int64_t max_cycles;     /* per-candidate cycle cap (<= 0: none) */
    int32_t charge_sign;    /* +1 forward tracking, -1 backtracking (charge -Z) */
    int32_t pad_;
    double bnd_center[3];   /* spherical boundary centre, m */
    double bnd_r;           /* boundary radius, m (0: none); leaving it ends a candidate */
    int32_t traj_every;     /* per-step output: every k-th accepted step (0: none) */
    uint32_t traj_ids;      /* per-step output only for candidates with id < traj_ids */
} or_config;

/* Synthetic analytic galactic field (section 4, galactic propagation: the
 * code offers analytic field models; the JF12 parameters are not available,
 * so this is a disk/halo/X-field model of the same structure with rational
 * profiles).  Cylindrical coordinates about `center`, axis z:
 *   disk toroidal  B_phi = b_disk (r/r_disk) / ((1 + r^2/r_disk^2)(1 + z^2/h_disk^2))
 *   halo toroidal  B_phi = b_halo (z/h_halo)(r/r_halo) / ((1 + r^2/r_halo^2)(1 + z^2/h_halo^2)^2)
 *   X-field        B = curl(A_phi e_phi), A_phi = b_x r / (2 D),
 *                  D = 1 + r^2/r_x^2 + z^2/h_x^2.
 * Every part is divergence-free. */
typedef struct {
    double center[3];
    double b_disk, r_disk, h_disk;
    double b_halo, r_halo, h_halo;
    double b_x, r_x, h_x;
} or_analytic;

/* Refinement patch of a multi-resolution grid (section 4: multi-resolution
 * grids give fast access to precomputed fields over a larger dynamic range).
 * A patch is a non-periodic vertex grid [n0][n1][n2][3] of the base grid's
 * element type with spacing base_spacing / refine; its vertex (0,0,0) sits on
 * base vertex `offset`, and it lies inside one period of the base grid.  It
 * repeats with the base grid's period.  Level selection: a position uses the
 * last patch (in list order) whose cells contain it, else the base grid. */
typedef struct {
    const void* data;
    int64_t n[3];
    int64_t offset[3];      /* base-grid vertex index of the patch's vertex (0,0,0) */
    int32_t refine;         /* base cells per patch cell along each axis: 2, 4, 8 or 16 */
    int32_t pad_;
} or_patch;

typedef struct {
    const void* data;       /* [nx][ny][nz][3] tesla, C order */
    int32_t dtype;          /* OR_GRID_F32 / OR_GRID_F64 */
    int32_t pad_;
    int64_t n[3];
    double spacing;         /* m */
    double origin[3];       /* m */
    const or_analytic* analytic;   /* non-NULL: this analytic field instead of the grid */
    int32_t n_patches;      /* refinement patches (0: a single-resolution grid) */
    int32_t pad2_;
    const or_patch* patches;
    /* non-NULL: a caller-supplied field instead of the grid (and of
     * `analytic`): B (T, FP64) at one position p (m); the precision form
     * rounds it to FP32.  A propagation with it runs on one thread. */
    void (*field_cb)(void* user, const double p[3], double B[3]);
    void* cb_user;
} or_grid;

typedef struct {
    int32_t n;
    int32_t pad_;
    const double* e;        /* nodes, eV, strictly increasing */
    const double* tpi;      /* pion-like rate per nucleon, 1/m */
    const double* tn;       /* nucleon-loss-like rate per nucleon, 1/m */
    const double* bp;       /* proton relative loss rate, 1/m */
} or_tables;

typedef struct {            /* finished (or, with max_cycles, still active) candidates */
    int64_t cap;
    uint32_t *id, *lineage, *m, *nsteps, *nrej;
    int32_t *status, *A, *Z;
    double *E, *x, *u, *L, *u0, *E0;   /* x, u, u0: n x 3 */
} or_finished;

typedef struct {            /* neutral secondaries (pion-like channel products) */
    int64_t cap;
    uint32_t *id, *lineage, *m;
    int32_t* chan;
    double *E, *x, *u;                 /* x, u: n x 3 */
} or_neutral;

/* Per-step trajectory output (section 3: output modules may record the
 * candidate after every step).  A point is recorded after the cycle of every
 * traj_every-th accepted step and after the cycle that ends the candidate;
 * the injection point itself is not recorded. */
typedef struct {
    int64_t cap;
    uint32_t *id, *lineage, *n;        /* n: accepted steps so far */
    int32_t* A;
    double *L, *E, *x;                 /* x: n x 3 */
} or_traj;

typedef struct {
    int64_t finished, observed, max_traj, energy_floor, still_active;
    int64_t steps, attempts, rejects, forced;
    int64_t events, null_events, inter_pi, inter_n;
    int64_t charged_sec, neutral_sec;
    int64_t fin_dropped, neu_dropped;
    int64_t boundary;
    int64_t traj_dropped;              /* trajectory points beyond the capacity */
} or_counts;

/* Propagate n injected candidates to completion (or max_cycles). Returns the
 * number of OpenMP threads used. */
int oracle_propagate(const or_config* cfg, const or_grid* grid, const or_tables* tab,
                     int64_t n, const uint32_t* id, const int32_t* A, const int32_t* Z,
                     const double* E, const double* pos, const double* dir,
                     const double* lmax, int nthreads,
                     or_finished* fin, or_neutral* neu, or_counts* counts,
                     int64_t* n_fin, int64_t* n_neu);

/* As oracle_propagate, also recording per-step trajectory points into traj
 * (config traj_every / traj_ids); *n_traj receives the number recorded. */
int oracle_propagate_traj(const or_config* cfg, const or_grid* grid, const or_tables* tab,
                          int64_t n, const uint32_t* id, const int32_t* A, const int32_t* Z,
                          const double* E, const double* pos, const double* dir,
                          const double* lmax, int nthreads,
                          or_finished* fin, or_neutral* neu, or_counts* counts,
                          int64_t* n_fin, int64_t* n_neu, or_traj* traj, int64_t* n_traj);

/* Field at n positions; mode OR_FP64 or OR_MIX (MIX results are FP32 values). */
void oracle_eval_field(const or_grid* grid, int32_t mode, int64_t n, const double* pos,
                       double* B);

/* One Cash-Karp attempt from (x,u) with curvature factor kappa = Z c / E and
 * step h. Outputs the 5th-order state and the embedded direction error. */
void oracle_ck_attempt(const or_grid* grid, int32_t mode, const double x[3], const double u[3],
                       double kappa, double h, double x5[3], double u5[3], double* err);

/* Philox4x64-10 block for counter ctr and key. */
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Table value by linear interpolation between the bracketing nodes. */
double oracle_table_lookup(const or_tables* tab, int32_t which, double eps);

/* Species-scaled rates (R_pi, R_N, R, beta) at total energy E. */
void oracle_rates(const or_tables* tab, int32_t A, int32_t Z, double E, double out[4]);

/* Optical-depth draw from a 64-bit word. */
double oracle_texp(uint64_t w);

/* Step-size factor numerator k (factor = k / 1024) for error ratio r > 0. */
int32_t oracle_ctrl_k(double r);

#ifdef __cplusplus
}
#endif
#endif
