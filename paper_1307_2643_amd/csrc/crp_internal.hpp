// Internal layout of the device buffers and kernel parameter blocks shared by
// the host runtime and the kernels of libcrp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crp_device.hpp"

namespace crp {

// Candidate queue, structure of arrays (one entry per candidate slot).
// Vectors are planar: x + q * cap holds component q.
struct QueueSoA {
    double *x, *u, *u0;
    double *E, *L, *Lmax, *hctrl, *tau, *E0;
    uint32_t *id, *lineage, *m, *nsteps, *nrej;
    int32_t *A, *Z;
    uint32_t* ready;     // publication flag of slots written during a run
    int64_t cap;
};

struct FinishedSoA {
    double *x, *u, *u0;  // planar [3][cap]
    double *E, *L, *E0;
    uint32_t *id, *lineage, *m, *nsteps, *nrej;
    int32_t *status, *A, *Z;
    int64_t cap;
};

struct NeutralSoA {
    double *x, *u;       // planar [3][cap]
    double* E;
    uint32_t *id, *lineage, *m;
    int32_t* chan;
    int64_t cap;
};

// Per-step trajectory points (planar x).
struct TrajSoA {
    double *x, *L, *E;
    uint32_t *id, *lineage, *n;
    int32_t* A;
    int64_t cap;
};

// Device counter block (all 64-bit, updated with device-scope atomics).
struct DevCounters {
    unsigned long long head;                // claim cursor of slots written before the run
    unsigned long long tail;                // append cursor (end of written slots)
    unsigned long long head1;               // claim cursor of slots appended during the run
    unsigned long long fin_n, neu_n, park_n;
    unsigned long long steps, attempts, rejects, forced;
    unsigned long long events, null_events, inter_pi, inter_n;
    unsigned long long charged_sec, neutral_sec;
    unsigned long long finished, observed, max_traj, energy_floor;
    unsigned long long queue_deferred, neutral_deferred;   // interactions that found no slot
    unsigned long long lane_slots;          // 64 x wave iterations
    unsigned long long boundary;            // stopped by the spherical boundary
    unsigned long long traj_n;              // trajectory-point append cursor (may pass the
                                            // capacity: the excess was dropped)
    unsigned long long error;               // nonzero: a wave gave up waiting
};

struct TableParams {
    const double* e;
    const double* v[3];
    int n;
    float lg0, scale;    // log2 of the first node, (n - 1) / log2 span of the nodes
};

struct StepParams {
    double tol, hmin, hmax, eps_loss, kappa_pi, e_floor;
    double obs[3], obs_r;
    uint64_t seed;
    int renorm;
    int charge_sign;             // +1 forward, -1 backtracking
    double bnd[3], bnd_r;        // spherical boundary (bnd_r = 0: none)
    uint32_t traj_every;         // per-step output every k-th step (0: none)
    uint32_t traj_ids;           // ... of candidates with id below this
};


// Neural-field source of the propagation kernel: the network image in global
// memory (staged into LDS by every block) and the grid period it was fit on.
struct NFProp {
    const char* img;
    double origin[3];
    double inv_box[3];
    float b_scale;
};

struct PropParams {
    QueueSoA q;
    QueueSoA park;
    FinishedSoA fin;
    NeutralSoA neu;
    TrajSoA traj;
    DevCounters* cnt;
    GridView grid;
    TableParams tab;
    StepParams sp;
    int64_t max_cycles;          // <= 0: no limit
    unsigned long long tail0;    // slots below were written before the launch
    unsigned long long fin0;     // finished-record count at the launch
    int refill;                  // idle lanes that trigger a claim (1..64)
    NFProp nf;                   // used by the neural-field instantiation only
    AnalyticParams ana;          // used by the analytic-field instantiation only
    NestView nest;               // used by the multi-resolution instantiation only
};

// Observable reduction over finished records (definitions in crp.h).
constexpr int OBS_MAX_BINS = 1024;      // n_groups * n_e
constexpr int OBS_MAX_E = 256;
constexpr int OBS_MAX_G = 16;
struct ObsParams {
    const double *E, *E0, *u, *u0;      // u, u0 planar [3][cap]
    const int32_t *status, *A;
    int64_t cap, n;
    const double* e_edges;              // device [ne + 1]
    const int32_t* a_edges;             // device [ng + 1]
    int ne, ng, sky_n;
    uint32_t status_mask;
    double sky_sign, e_ref, gamma;
    unsigned long long *counts, *defl, *sky, *outside;
    double* wsum;
};

enum { MODE_FP64 = 0, MODE_MIX = 1 };

}  // namespace crp
