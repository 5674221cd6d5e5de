// Propagation kernels of libcrp for gfx950 (CDNA4, wave64).
//
// One lane holds one candidate in registers (the candidate carries all of its
// propagation state, paper section 3).  Waves are persistent: idle lanes claim
// candidates from a device queue, every loop iteration performs exactly one
// Cash-Karp attempt for all busy lanes (so the expensive part -- six field
// gathers -- is executed by the whole wave together), and lanes whose
// attempt is accepted finish their cycle: continuous loss, the stochastic
// interaction clock (reset after each event, section 3), then the
// observer / trajectory / energy-floor checks after the cycle (Fig. 1).
// Finished records, neutral records, spawned secondaries and budget-parked
// candidates are appended with one atomic per wave (ballot + prefix count).
#include "crp_internal.hpp"
#include "crp_nf_device.hpp"

namespace crp {

enum { LIM_CTRL = 0, LIM_TRAJ = 1, LIM_INTER = 2, LIM_LOSS = 3, LIM_OBS = 4 };
// interaction channel chosen in a cycle: none due, a null event (no channel
// open at this energy), pion-like (neutral record), nucleon loss (secondary)
enum { CH_NONE = -1, CH_PI = 0, CH_N = 1, CH_NULL = 2 };

// A parked candidate whose cycle stopped just before its interaction (no
// slot for the product) carries -(1 + step-limit flag) as its optical depth:
// a stored optical depth is otherwise always positive (an interaction resets
// it to at least 2^-24, and without one it stayed above zero).
__device__ inline double event_due_marker(int flag) { return -1.0 - (double)flag; }
__device__ inline int event_due_flag(double tau) { return (int)(-tau) - 1; }
enum { ST_ACTIVE = 0, ST_OBSERVED = 1, ST_MAX_TRAJ = 2, ST_ENERGY_FLOOR = 3, ST_BOUNDARY = 4 };

struct Cand {
    double x[3], u[3], u0[3];
    double E, L, Lmax, hctrl, tau, E0;
    uint32_t id, lineage, m, nsteps, nrej;
    int A, Z;
};

__device__ inline void store_cand(const QueueSoA& q, int64_t i, const Cand& c)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.x[a * q.cap + i] = c.x[a];
        q.u[a * q.cap + i] = c.u[a];
        q.u0[a * q.cap + i] = c.u0[a];
    }
    q.E[i] = c.E;
    q.L[i] = c.L;
    q.Lmax[i] = c.Lmax;
    q.hctrl[i] = c.hctrl;
    q.tau[i] = c.tau;
    q.E0[i] = c.E0;
    q.id[i] = c.id;
    q.lineage[i] = c.lineage;
    q.m[i] = c.m;
    q.nsteps[i] = c.nsteps;
    q.nrej[i] = c.nrej;
    q.A[i] = c.A;
    q.Z[i] = c.Z;
}

// Bookkeeping: block counters in LDS; the per-iteration counts (attempts,
// accepts, forced accepts) are added once per wave from a ballot, rare events
// with an LDS atomic where they happen.
enum {
    WC_STEPS = 0, WC_ATTEMPTS, WC_REJECTS, WC_FORCED, WC_EVENTS, WC_NULL, WC_PI, WC_N,
    WC_FINISHED, WC_OBSERVED, WC_MAXTRAJ, WC_EFLOOR, WC_QDEFER, WC_NDEFER, WC_LANES, WC_BOUNDARY,
    WC_COUNT
};
enum : uint32_t { EV_ATTEMPT = 1u << 0, EV_ACCEPT = 1u << 1, EV_FORCED = 1u << 2, EV_FIN = 1u << 3 };

__device__ inline unsigned long long count_bit(uint32_t ev, uint32_t bit)
{
    return (unsigned long long)__popcll(__ballot((ev & bit) != 0u));
}

// Adds a wave-uniform count to the block's LDS counter.
__device__ inline void add_count(unsigned long long* bc, int i, unsigned long long v)
{
    if (v != 0ull && lane_id() == 0)
        atomicAdd(bc + i, v);
}

// Destination of each block counter in the device counter block.
__device__ inline unsigned long long* count_dst(DevCounters* cnt, int i)
{
    switch (i) {
    case WC_STEPS: return &cnt->steps;
    case WC_ATTEMPTS: return &cnt->attempts;
    case WC_REJECTS: return &cnt->rejects;
    case WC_FORCED: return &cnt->forced;
    case WC_EVENTS: return &cnt->events;
    case WC_NULL: return &cnt->null_events;
    case WC_PI: return &cnt->inter_pi;
    case WC_N: return &cnt->inter_n;
    case WC_FINISHED: return &cnt->finished;
    case WC_OBSERVED: return &cnt->observed;
    case WC_MAXTRAJ: return &cnt->max_traj;
    case WC_EFLOOR: return &cnt->energy_floor;
    case WC_QDEFER: return &cnt->queue_deferred;
    case WC_NDEFER: return &cnt->neutral_deferred;
    case WC_LANES: return &cnt->lane_slots;
    default: return &cnt->boundary;
    }
}

__device__ inline void flush_counts(DevCounters* cnt, const unsigned long long* bc)
{
    const int i = (int)threadIdx.x;
    if (i < WC_COUNT && bc[i] != 0ull) {
        atomicAdd(count_dst(cnt, i), bc[i]);
        // every pion-like event emits one neutral secondary, every nucleon-loss
        // event one charged secondary
        if (i == WC_PI)
            atomicAdd(&cnt->neutral_sec, bc[i]);
        if (i == WC_N)
            atomicAdd(&cnt->charged_sec, bc[i]);
    }
}

// Claims up to `want` slots of the region written before the launch with one
// atomicAdd (overshoot past tail0 is harmless: that region does not grow).
__device__ inline void claim_initial(DevCounters* cnt, unsigned long long tail0, int want,
                                     unsigned long long& base, unsigned long long& take,
                                     bool& left)
{
    const unsigned long long b = atomicAdd(&cnt->head, (unsigned long long)want);
    base = b;
    take = 0;
    left = false;
    if (b < tail0) {
        take = tail0 - b < (unsigned long long)want ? tail0 - b : (unsigned long long)want;
        left = b + take < tail0;
    }
}

// True once every candidate of this run is finished or parked: then none is
// active, so no secondary can be appended any more.  The done counts are read
// (acquire) before the append cursor; all three only grow and done never
// exceeds the written slots, so equality means that at the last read every
// written slot was done.  Slots past the queue capacity are never written.
// `done` receives the finished + parked count that was read.
__device__ inline bool run_drained(DevCounters* cnt, unsigned long long fin0,
                                   unsigned long long cap, unsigned long long& done)
{
    const unsigned long long f =
        __hip_atomic_load(&cnt->fin_n, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long p =
        __hip_atomic_load(&cnt->park_n, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long t = __hip_atomic_load(&cnt->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t > cap)
        t = cap;
    done = (f - fin0) + p;
    return done == t;
}

// A wave with nothing to do sleeps in units of s_sleep 127 (~3.4 us), one
// unit more per idle iteration up to IDLE_BACKOFF (its polls of the queue
// must not load the memory system that busy waves use).  If IDLE_SLEEP_LIMIT
// units (about 28 s) pass with no candidate of the run finishing anywhere and
// the run not drained, it records an error and leaves.
constexpr uint32_t IDLE_BACKOFF = 16u;
constexpr uint32_t IDLE_SLEEP_LIMIT = 1u << 23;

// Per-lane candidate state that is not needed inside a Cash-Karp attempt,
// kept in LDS (structure of arrays over the block's lanes) so that only the
// position, direction, step and curvature occupy registers in the attempt.
template <int BS>
struct LaneShared {
    double E[BS], L[BS], Lmax[BS], hctrl[BS], tau[BS], R[BS], beta[BS];
    uint32_t id[BS], lineage[BS], m[BS], nsteps[BS], nrej[BS], cycles[BS];
    uint32_t azf[BS];   // A | Z << 8 | step-limit flag << 16
};

__device__ inline int unpack_A(uint32_t v) { return (int)(v & 0xffu); }
__device__ inline int unpack_Z(uint32_t v) { return (int)((v >> 8) & 0xffu); }
__device__ inline int unpack_flag(uint32_t v) { return (int)((v >> 16) & 0xffu); }
__device__ inline uint32_t pack_azf(int A, int Z, int flag)
{
    return (uint32_t)A | ((uint32_t)Z << 8) | ((uint32_t)flag << 16);
}

// Hides a pointer's value from the optimiser so that loads through it stay
// inside the (rarely taken) branch that needs them instead of being hoisted
// out of the persistent loop into scalar registers.
template <class T>
__device__ inline const T* opaque(const T* p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// Field source of a layout: 0 linear grid, 1 corner records (per lane),
// 2 corner records gathered by the whole wave, 3 the neural field, 4 the
// analytic galactic field, 5 the multi-resolution grid (linear base grid and
// refinement patches), 6 the multi-resolution grid from corner records
// gathered by the whole wave.
template <class GT, int LAYOUT>
struct FieldOf {
    using T = GridField<GT, LAYOUT>;
};
template <class GT>
struct FieldOf<GT, 3> {
    using T = NeuralFieldSrc;
};
template <class GT>
struct FieldOf<GT, 4> {
    using T = AnalyticFieldSrc;
};
template <class GT>
struct FieldOf<GT, 5> {
    using T = NestedField<GT>;
};
template <class GT>
struct FieldOf<GT, 6> {
    using T = NestedField<GT, true>;
};

// Layouts whose field values are gathered by the whole wave together.
template <int LAYOUT>
constexpr bool wave_gather = LAYOUT == 2 || LAYOUT == 6;

template <int MODE>
struct DirType {
    using T = double;
};
template <>
struct DirType<MODE_MIX> {
    using T = float;
};

// Minimum waves per SIMD the register allocation targets (occupancy vs
// spills), per precision form.  Measured on the 1e7 batch, 1024^3 grid: both
// forms are fastest at 2 (8 waves per CU, no spills); at 3 the precision form
// spills (1.36 s vs 1.30 s per batch) and the FP64 form spills inside the
// attempt.
#ifndef CRP_WAVES_MIX
#define CRP_WAVES_MIX 2
#endif
#ifndef CRP_WAVES_FP64
#define CRP_WAVES_FP64 2
#endif
// The analytic field has no memory traffic to overlap: its waves hide the
// latency of FP64 arithmetic instead.
#ifndef CRP_WAVES_ANALYTIC
#define CRP_WAVES_ANALYTIC 2
#endif

template <int MODE, int LAYOUT>
constexpr int min_waves = LAYOUT == 3   ? 1
                          : LAYOUT == 4 ? CRP_WAVES_ANALYTIC
                                        : (MODE == MODE_MIX ? CRP_WAVES_MIX : CRP_WAVES_FP64);

// TRAJ: the variant with the per-step output module compiled in (a run without
// trajectory output uses the variant without it, whose loop carries no trace
// of it).
template <int MODE, class GT, int LAYOUT, int BS, bool TRAJ>
__global__ void __launch_bounds__(BS, (min_waves<MODE, LAYOUT>))
    k_propagate(const PropParams* __restrict__ PP)
{
    using UT = typename DirType<MODE>::T;   // direction storage: FP64 or FP32
    // interaction tables, then (neural field) the network image, whose 16-byte
    // operand loads need 16-byte alignment whatever the static LDS size
    extern __shared__ __attribute__((aligned(16))) double lds[];
    __shared__ LaneShared<BS> S;              // per-lane cold state
    __shared__ unsigned long long bc[WC_COUNT];   // block bookkeeping counters
    // LDS staging of the wave-cooperative corner gather (LAYOUT 2 and 6 only)
    __shared__ float4 stage_mem[wave_gather<LAYOUT> ? BS / 64 * coop_stage_float4<GT> : 1];
    // patch table of the multi-resolution grid (LAYOUT 5 only)
    __shared__ PatchView nest_lds[LAYOUT == 5 || LAYOUT == 6 ? MAX_PATCHES : 1];
    const int t = (int)threadIdx.x;
    const int ntab = PP->tab.n;
    {
        const TableParams tp = PP->tab;
        for (int i = t; i < ntab; i += BS) {
            lds[i] = tp.e[i];
            lds[ntab + i] = tp.v[0][i];
            lds[2 * ntab + i] = tp.v[1][i];
            lds[3 * ntab + i] = tp.v[2][i];
        }
    }
    if (t < WC_COUNT)
        bc[t] = 0ull;
    if constexpr (LAYOUT == 5 || LAYOUT == 6) {
        if (t < PP->nest.np)
            nest_lds[t] = PP->nest.p[t];
    }
    __syncthreads();
    TableView T;
    T.e = lds;
    T.v[0] = lds + ntab;
    T.v[1] = lds + 2 * ntab;
    T.v[2] = lds + 3 * ntab;
    T.n = ntab;
    T.lg0 = PP->tab.lg0;
    T.scale = PP->tab.scale;

    typename FieldOf<GT, LAYOUT>::T F;
    if constexpr (LAYOUT == 3) {
        // the network image follows the tables in dynamic LDS
        char* img = (char*)(lds + 4 * ntab);
        nf_stage_lds(img, PP->nf.img);
        __syncthreads();
        F.v = nf_view_lds(img, PP->nf.origin, PP->nf.inv_box, PP->nf.b_scale);
    } else if constexpr (LAYOUT == 4) {
        F.a = PP->ana;
    } else if constexpr (LAYOUT == 5 || LAYOUT == 6) {
        F.g = PP->grid;
        F.P = nest_lds;
        F.np = PP->nest.np;
        F.set_first(PP->nest.p[0]);
        if constexpr (LAYOUT == 6)
            F.stage = (float*)(stage_mem + (t >> 6) * COOP_STAGE_FLOAT4);
    } else {
        F.g = PP->grid;
        F.stage = (float*)(stage_mem + (LAYOUT == 2 ? (t >> 6) * coop_stage_float4<GT> : 0));
    }
    const StepParams sp = PP->sp;
    const int lane = lane_id();
    const unsigned long long qcap = (unsigned long long)PP->q.cap;
    const unsigned long long tail0 = PP->tail0;
    const int refill = PP->refill;
    const int64_t max_cycles = PP->max_cycles;
    DevCounters* const cnt = PP->cnt;

    // registers through the attempt: position, direction, step, curvature
    double x[3] = {0.0, 0.0, 0.0};
    UT u[3] = {0, 0, 0};
    double h = 0.0, kappa = 0.0;
    int64_t slot = 0;
    bool active = false, fresh = true;
    // the lane holds a candidate whose last cycle stopped just before an
    // interaction for want of an output slot: it finishes that cycle first
    bool resume = false;
    // field at the current position, kept for the retry after a rejection
    using BT = typename DirType<MODE>::T;
    BT b1[3] = {0, 0, 0};
    bool reuse = false;
    // cooperative layout: the field at the position an accepted attempt moved
    // to is fetched while the rest of its cycle runs, for the next attempt
    bool pref = false;
    bool initial_left = true;
    // this wave's reservation of appended slots [rb, re): taken with one
    // atomicAdd, handed to idle lanes as their producers publish them
    unsigned long long rb = 0, re = 0;
    uint32_t sleeps = 0, backoff = 0;
    unsigned long long seen_done = 0;   // progress of the run seen while idle
    const unsigned long long fin0 = PP->fin0;

    for (;;) {
        // ---- refill idle lanes from the queue -------------------------------
        const uint64_t idle = __ballot(!active);
        const int nidle = __popcll(idle);
        if (idle == ~0ull || nidle >= refill) {
            const int rank = lanes_below(idle);
            unsigned long long base = 0, take = 0;
            if (initial_left) {
                bool left = false;
                if (lane == 0)
                    claim_initial(cnt, tail0, nidle, base, take, left);
                base = __shfl(base, 0);
                take = __shfl(take, 0);
                initial_left = __shfl((int)left, 0) != 0;
            } else {
                if (rb >= re) {
                    unsigned long long b = 0;
                    if (lane == 0)
                        b = atomicAdd(&cnt->head1, (unsigned long long)nidle);
                    rb = __shfl(b, 0);
                    re = rb + (unsigned long long)nidle;
                }
                // idle lane of rank r looks at slot rb + r; the published
                // prefix of the reservation is handed out in order
                const unsigned long long sl = rb + (unsigned long long)rank;
                const bool mine = !active && sl < re;
                bool pub = false;
                if (mine && sl < qcap)
                    pub = __hip_atomic_load(opaque(PP)->q.ready + sl, __ATOMIC_ACQUIRE,
                                            __HIP_MEMORY_SCOPE_AGENT) != 0u;
                const uint64_t gap = __ballot(mine && !pub);
                if (gap)
                    take = (unsigned long long)__popcll(idle & ((1ull << __builtin_ctzll(gap)) - 1ull));
                else
                    take = re - rb < (unsigned long long)nidle ? re - rb : (unsigned long long)nidle;
                base = rb;
                rb += take;
            }
            if (!active && (unsigned long long)rank < take) {
                const QueueSoA& q = opaque(PP)->q;
                slot = (int64_t)(base + (unsigned long long)rank);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    x[a] = q.x[a * q.cap + slot];
                    u[a] = (UT)q.u[a * q.cap + slot];
                }
                S.E[t] = q.E[slot];
                S.L[t] = q.L[slot];
                S.Lmax[t] = q.Lmax[slot];
                S.hctrl[t] = q.hctrl[slot];
                S.tau[t] = q.tau[slot];
                S.id[t] = q.id[slot];
                S.lineage[t] = q.lineage[slot];
                S.m[t] = q.m[slot];
                S.nsteps[t] = q.nsteps[slot];
                S.nrej[t] = q.nrej[slot];
                S.cycles[t] = 0u;
                resume = S.tau[t] < 0.0;
                // a resumed cycle keeps the step limit its step had
                S.azf[t] = pack_azf(q.A[slot], q.Z[slot],
                                    resume ? event_due_flag(S.tau[t]) : LIM_CTRL);
                if ((unsigned long long)slot >= tail0)
                    q.ready[slot] = 0u;   // clean for the next run
                active = true;
                fresh = !resume;
                reuse = false;
                pref = false;
            }
        }
        if (__ballot(active) == 0ull) {
            // nothing to do: leave once the run has drained, else wait for
            // secondaries that busy waves may still append
            if (!initial_left) {
                bool drained = false;
                unsigned long long done = 0;
                if (lane == 0)
                    drained = run_drained(cnt, fin0, qcap, done);
                if (__shfl((int)drained, 0))
                    break;
                done = __shfl(done, 0);
                if (done != seen_done) {   // the run is progressing: keep waiting
                    seen_done = done;
                    sleeps = 0;
                }
            }
            if (backoff < IDLE_BACKOFF)
                ++backoff;
            for (uint32_t k = 0; k < backoff; ++k)
                __builtin_amdgcn_s_sleep(127);
            sleeps += backoff;
            if (sleeps >= IDLE_SLEEP_LIMIT) {
                if (lane == 0)
                    atomicAdd(&cnt->error, 1ull);
                break;
            }
            continue;
        }
        backoff = 0;

        // ---- start of a cycle: rates and step proposal -----------------------
        if (active && fresh) {
            const uint32_t azf = S.azf[t];
            const int A = unpack_A(azf), Z = unpack_Z(azf);
            const double E = S.E[t];
            const Rates rt = species_rates(T, A, Z, E);
            const double R = rt.r, beta = rt.beta;
            const double L = S.L[t], Lmax = S.Lmax[t], tau = S.tau[t];
            int flag = LIM_CTRL;
            h = S.hctrl[t];
            if (Lmax - L < h) {
                h = Lmax - L;
                flag = LIM_TRAJ;
            }
            if (R > 0.0 && tau / R < h) {
                h = tau / R;
                flag = LIM_INTER;
            }
            if (beta > 0.0 && sp.eps_loss / beta < h) {
                h = sp.eps_loss / beta;
                flag = LIM_LOSS;
            }
            if (sp.obs_r > 0.0) {
                const double d[3] = {x[0] - sp.obs[0], x[1] - sp.obs[1], x[2] - sp.obs[2]};
                const double dist = sqrt(dot3(d, d));
                const double half = 0.5 * sp.obs_r;
                double hob = dist - half;
                if (hob < half)
                    hob = half;
                if (hob < h) {
                    h = hob;
                    flag = LIM_OBS;
                }
            }
            // backtracking follows the antiparticle: charge -Z
            kappa = ((double)(sp.charge_sign * Z) * kC) / E;
            S.R[t] = R;
            S.beta[t] = beta;
            S.azf[t] = pack_azf(A, Z, flag);
            fresh = false;
        }

        // ---- the first-stage field of this position may already be on its way
        if constexpr (wave_gather<LAYOUT>) {
            if (__ballot(pref) != 0ull) {
                BT bp[3];
                if constexpr (MODE == MODE_FP64)
                    F.fp64_prefetched(x, bp);
                else
                    F.fp32_prefetched(x, bp);
                if (pref) {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        b1[q] = bp[q];
                    reuse = true;
                }
                pref = false;
            }
        }

        // ---- one Cash-Karp attempt -------------------------------------------
        uint32_t ev = 0u;
        int status = ST_ACTIVE;
        bool park = false, rec = false;
        // lanes that step in this iteration (a resumed lane only finishes its
        // interrupted cycle)
        const bool stepping = active && !resume;
        // with the cooperative gather every lane of the wave takes part in the
        // attempt (idle lanes on a harmless cell); results are used only by
        // busy lanes
        double x5[3];
        UT u5[3];
        double err = 0.0;
        if (stepping || wave_gather<LAYOUT> || LAYOUT == 3) {
            if constexpr (MODE == MODE_FP64) {
                const double y[6] = {x[0], x[1], x[2], u[0], u[1], u[2]};
                double y5[6];
                err = ck_attempt_fp64(F, kappa, y, h, y5, stepping, reuse, b1);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    x5[q] = y5[q];
                    u5[q] = y5[3 + q];
                }
            } else {
                if constexpr (LAYOUT == 3)
                    err = ck_attempt_mix_rolled(F, kappa, x, u, h, x5, u5);
                else
                    err = ck_attempt_mix_f(F, kappa, x, u, h, x5, u5, stepping, reuse, b1);
            }
        }
        if constexpr (wave_gather<LAYOUT>) {
            // accepted lanes move to x5: start fetching B(x5) now, so that the
            // loads overlap the rest of the cycle
            const bool acc = stepping && (err / sp.tol <= 1.0 || h <= sp.hmin);
            if (__ballot(acc) != 0ull)
                F.prefetch(x5, acc);
            pref = acc;
        }
        // the cycle's energy and optical depth after the step, and whether an
        // interaction is due
        double E = 0.0, tau = 0.0;
        bool evt = false, cycle = false;
        if (stepping) {
            ev |= EV_ATTEMPT;
            const double r = err / sp.tol;
            if (r <= 1.0 || h <= sp.hmin) {
                ev |= EV_ACCEPT;
                reuse = false;
                if (r > 1.0)
                    ev |= EV_FORCED;
                double fac = 5.0;
                if (r > 0.0) {
                    fac = (double)ctrl_k(r) / 1024.0;
                    if (fac > 5.0)
                        fac = 5.0;
                }
                double hn = h * fac;
                if (hn < sp.hmin)
                    hn = sp.hmin;
                if (hn > sp.hmax)
                    hn = sp.hmax;
                S.hctrl[t] = hn;
                // integration module: position, direction, trajectory length
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    x[q] = x5[q];
                if (sp.renorm) {
                    if constexpr (MODE == MODE_FP64) {
                        const double nrm = sqrt(dot3(u5, u5));
#pragma unroll
                        for (int q = 0; q < 3; ++q)
                            u[q] = u5[q] / nrm;
                    } else {
                        const float nrm = sqrtf(dot3f(u5, u5));
#pragma unroll
                        for (int q = 0; q < 3; ++q)
                            u[q] = u5[q] / nrm;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        u[q] = u5[q];
                }
                const double L = S.L[t] + h;
                S.L[t] = L;
                S.nsteps[t] += 1u;
                // continuous loss: (2,2) Pade form of exp(-beta h)
                E = S.E[t];
                {
                    const double z = S.beta[t] * h;
                    const double z2 = z * z;
                    const double num = (12.0 - 6.0 * z) + z2;
                    const double den = (12.0 + 6.0 * z) + z2;
                    E = E * (num / den);
                }
                // stochastic interactions: optical-depth clock
                tau = S.tau[t] - S.R[t] * h;
                evt = unpack_flag(S.azf[t]) == LIM_INTER || tau <= 0.0;
                cycle = true;
            } else {
                reuse = true;             // same position: b1 holds its field
                S.nrej[t] += 1u;
                double fac = (double)ctrl_k(r) / 1024.0;
                if (fac < 0.1)
                    fac = 0.1;
                h = h * fac;
                if (h < sp.hmin)
                    h = sp.hmin;
                S.azf[t] = (S.azf[t] & 0xffffu) | ((uint32_t)LIM_CTRL << 16);
            }
        }
        if (resume) {
            // the interrupted cycle: its step and loss are done, its
            // interaction is due (the clock value is replaced after it)
            E = S.E[t];
            evt = true;
            cycle = true;
            resume = false;
        }

        // ---- interaction: channel first, then a slot for its product --------
        // (one atomic per wave for each kind of product); a lane that finds no
        // slot keeps its state as before the interaction and is parked, to
        // finish the cycle in a later run: nothing is lost
        int chan = CH_NONE;
        U64x4 w = {{0ull, 0ull, 0ull, 0ull}};
        double dE = 0.0, Esec = 0.0;
        if (evt) {
            w = event_draw(sp.seed, S.id[t], S.lineage[t], S.m[t] + 1u);
            const uint32_t azf = S.azf[t];
            const Rates ri = species_rates(T, unpack_A(azf), unpack_Z(azf), E);
            const double Ptot = ri.rpi + ri.rn;
            chan = !(Ptot > 0.0) ? CH_NULL : (unit_uniform(w.w[0]) * Ptot < ri.rpi ? CH_PI : CH_N);
        }
        bool defer = false;
        unsigned long long slot_n = 0, slot_pi = 0;
        {
            const uint64_t mk = __ballot(chan == CH_N);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&cnt->tail, (unsigned long long)__popcll(mk));
                slot_n = __shfl(base, 0) + (unsigned long long)lanes_below(mk);
                defer = chan == CH_N && slot_n >= qcap;
            }
        }
        {
            const uint64_t mk = __ballot(chan == CH_PI);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&cnt->neu_n, (unsigned long long)__popcll(mk));
                slot_pi = __shfl(base, 0) + (unsigned long long)lanes_below(mk);
                defer = defer || (chan == CH_PI &&
                                  slot_pi >= (unsigned long long)opaque(PP)->neu.cap);
            }
        }
        if (defer) {
            atomicAdd(&bc[chan == CH_N ? WC_QDEFER : WC_NDEFER], 1ull);
            S.E[t] = E;
            S.tau[t] = event_due_marker(unpack_flag(S.azf[t]));
            park = true;
        } else if (cycle) {
            if (evt) {
                const uint32_t m = S.m[t] + 1u;
                S.m[t] = m;
                const uint32_t azf = S.azf[t];
                int A = unpack_A(azf), Z = unpack_Z(azf);
                const double Eint = E;
                atomicAdd(&bc[WC_EVENTS], 1ull);
                if (chan == CH_PI) {
                    dE = (sp.kappa_pi * Eint) / (double)A;
                    E = Eint - dE;
                    atomicAdd(&bc[WC_PI], 1ull);
                    const NeutralSoA& nq = opaque(PP)->neu;
                    const int64_t k = (int64_t)slot_pi;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        nq.x[a * nq.cap + k] = x[a];
                        nq.u[a * nq.cap + k] = (double)u[a];
                    }
                    nq.E[k] = dE;
                    nq.id[k] = S.id[t];
                    nq.lineage[k] = S.lineage[t];
                    nq.m[k] = m;
                    nq.chan[k] = 0;
                } else if (chan == CH_N) {
                    const int pout = (2 * Z > A) ? 1 : 0;
                    Esec = Eint / (double)A;
                    Z -= pout;
                    A -= 1;
                    E = Eint - Esec;
                    S.azf[t] = pack_azf(A, Z, unpack_flag(azf));
                    atomicAdd(&bc[WC_N], 1ull);
                    // the secondary proton: a new candidate in the queue
                    const QueueSoA& q = opaque(PP)->q;
                    const int64_t k = (int64_t)slot_n;
                    const uint32_t id = S.id[t];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        q.x[a * q.cap + k] = x[a];
                        q.u[a * q.cap + k] = (double)u[a];
                        q.u0[a * q.cap + k] = q.u0[a * q.cap + slot];
                    }
                    q.E[k] = Esec;
                    q.L[k] = S.L[t];
                    q.Lmax[k] = S.Lmax[t];
                    q.hctrl[k] = sp.hmin;
                    q.E0[k] = q.E0[slot];
                    q.id[k] = id;
                    q.lineage[k] = m;
                    q.m[k] = 0u;
                    q.nsteps[k] = 0u;
                    q.nrej[k] = 0u;
                    q.A[k] = 1;
                    q.Z[k] = 1;
                    q.tau[k] = optical_depth(event_draw(sp.seed, id, m, 0u).w[1]);
                    __hip_atomic_store(q.ready + k, 1u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    atomicAdd(&bc[WC_NULL], 1ull);
                }
                // all interaction state is reset after an interaction
                tau = optical_depth(w.w[1]);
            }
            S.E[t] = E;
            S.tau[t] = tau;
            // boundary and observer modules, checked after the cycle
            const uint32_t cyc = S.cycles[t] + 1u;
            S.cycles[t] = cyc;
            if (sp.obs_r > 0.0) {
                const double d[3] = {x[0] - sp.obs[0], x[1] - sp.obs[1], x[2] - sp.obs[2]};
                if (sqrt(dot3(d, d)) <= sp.obs_r)
                    status = ST_OBSERVED;
            }
            if (status == ST_ACTIVE && sp.bnd_r > 0.0) {
                const double d[3] = {x[0] - sp.bnd[0], x[1] - sp.bnd[1], x[2] - sp.bnd[2]};
                if (sqrt(dot3(d, d)) >= sp.bnd_r)
                    status = ST_BOUNDARY;
            }
            if (status == ST_ACTIVE &&
                (unpack_flag(S.azf[t]) == LIM_TRAJ || S.L[t] >= S.Lmax[t]))
                status = ST_MAX_TRAJ;
            if (status == ST_ACTIVE && E < sp.e_floor)
                status = ST_ENERGY_FLOOR;
            if (status != ST_ACTIVE) {
                ev |= EV_FIN;
                atomicAdd(&bc[WC_FINISHED], 1ull);
                atomicAdd(&bc[status == ST_OBSERVED   ? WC_OBSERVED
                              : status == ST_BOUNDARY ? WC_BOUNDARY
                              : status == ST_MAX_TRAJ ? WC_MAXTRAJ
                                                      : WC_EFLOOR],
                          1ull);
            } else if (max_cycles > 0 && (int64_t)cyc >= max_cycles) {
                park = true;
            }
            // output module: every traj_every-th step and the last one
            if constexpr (TRAJ) {
                // read here rather than kept in scalar registers all loop long
                const StepParams& spp = opaque(PP)->sp;
                const uint32_t every = spp.traj_every;
                if (every != 0u && S.id[t] < spp.traj_ids)
                    rec = S.nsteps[t] % every == 0u || status != ST_ACTIVE;
            }
            fresh = true;
        }
        const bool fin = (ev & EV_FIN) != 0u;

        // ---- appends: one atomic per wave for each kind ----------------------
        if constexpr (TRAJ) {
            const uint64_t mk = __ballot(rec);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&cnt->traj_n, (unsigned long long)__popcll(mk));
                base = __shfl(base, 0);
                if (rec) {
                    const TrajSoA& tq = opaque(PP)->traj;
                    const unsigned long long i = base + (unsigned long long)lanes_below(mk);
                    if (i < (unsigned long long)tq.cap) {
                        const int64_t k = (int64_t)i;
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            tq.x[a * tq.cap + k] = x[a];
                        tq.L[k] = S.L[t];
                        tq.E[k] = S.E[t];
                        tq.id[k] = S.id[t];
                        tq.lineage[k] = S.lineage[t];
                        tq.n[k] = S.nsteps[t];
                        tq.A[k] = unpack_A(S.azf[t]);
                    }   // points past the capacity are counted by the host
                }
            }
        }
        {
            const uint64_t mk = __ballot(fin);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&cnt->fin_n, (unsigned long long)__popcll(mk));
                base = __shfl(base, 0);
                if (fin) {
                    const unsigned long long i = base + (unsigned long long)lanes_below(mk);
                    const PropParams* Q = opaque(PP);
                    if (i < (unsigned long long)Q->fin.cap) {
                        const FinishedSoA& f = Q->fin;
                        const int64_t k = (int64_t)i;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            f.x[a * f.cap + k] = x[a];
                            f.u[a * f.cap + k] = (double)u[a];
                            f.u0[a * f.cap + k] = Q->q.u0[a * Q->q.cap + slot];
                        }
                        f.E[k] = S.E[t];
                        f.L[k] = S.L[t];
                        f.E0[k] = Q->q.E0[slot];
                        f.id[k] = S.id[t];
                        f.lineage[k] = S.lineage[t];
                        f.m[k] = S.m[t];
                        f.nsteps[k] = S.nsteps[t];
                        f.nrej[k] = S.nrej[t];
                        f.status[k] = status;
                        f.A[k] = unpack_A(S.azf[t]);
                        f.Z[k] = unpack_Z(S.azf[t]);
                    }
                    active = false;
                }
            }
        }
        {
            const uint64_t mk = __ballot(park);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&cnt->park_n, (unsigned long long)__popcll(mk));
                base = __shfl(base, 0);
                if (park) {
                    const unsigned long long i = base + (unsigned long long)lanes_below(mk);
                    const PropParams* Q = opaque(PP);
                    if (i < (unsigned long long)Q->park.cap) {
                        const QueueSoA& pq = Q->park;
                        const int64_t k = (int64_t)i;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            pq.x[a * pq.cap + k] = x[a];
                            pq.u[a * pq.cap + k] = (double)u[a];
                            pq.u0[a * pq.cap + k] = Q->q.u0[a * Q->q.cap + slot];
                        }
                        pq.E[k] = S.E[t];
                        pq.L[k] = S.L[t];
                        pq.Lmax[k] = S.Lmax[t];
                        pq.hctrl[k] = S.hctrl[t];
                        pq.tau[k] = S.tau[t];
                        pq.E0[k] = Q->q.E0[slot];
                        pq.id[k] = S.id[t];
                        pq.lineage[k] = S.lineage[t];
                        pq.m[k] = S.m[t];
                        pq.nsteps[k] = S.nsteps[t];
                        pq.nrej[k] = S.nrej[t];
                        pq.A[k] = unpack_A(S.azf[t]);
                        pq.Z[k] = unpack_Z(S.azf[t]);
                    }
                    active = false;
                }
            }
        }

        // ---- bookkeeping: the frequent counts by wave ballot (rare events were
        // counted with LDS atomics where they happened) ------------------------
        {
            const unsigned long long att = count_bit(ev, EV_ATTEMPT);
            const unsigned long long acc = count_bit(ev, EV_ACCEPT);
            const unsigned long long frc = count_bit(ev, EV_FORCED);
            add_count(bc, WC_ATTEMPTS, att);
            add_count(bc, WC_STEPS, acc);
            add_count(bc, WC_REJECTS, att - acc);
            add_count(bc, WC_FORCED, frc);
            add_count(bc, WC_LANES, 64ull);
        }
    }
    __syncthreads();   // every wave of the block has left the loop
    flush_counts(cnt, bc);
}

// Explicit instantiations: FP64 / mixed stage arithmetic x grid element type x
// grid layout (per-lane corner records and multi-resolution corner records
// exist for FP32 grids only).
#define CRP_INST(MODE, GT, LAYOUT)                                                          \
    template __global__ void k_propagate<MODE, GT, LAYOUT, 128, false>(const PropParams*); \
    template __global__ void k_propagate<MODE, GT, LAYOUT, 256, false>(const PropParams*); \
    template __global__ void k_propagate<MODE, GT, LAYOUT, 128, true>(const PropParams*);  \
    template __global__ void k_propagate<MODE, GT, LAYOUT, 256, true>(const PropParams*);
CRP_INST(MODE_FP64, double, 0)
CRP_INST(MODE_FP64, double, 2)
CRP_INST(MODE_FP64, double, 4)
CRP_INST(MODE_FP64, double, 5)
CRP_INST(MODE_FP64, float, 5)
CRP_INST(MODE_MIX, double, 5)
CRP_INST(MODE_MIX, float, 5)
CRP_INST(MODE_MIX, float, 6)
CRP_INST(MODE_FP64, float, 6)
CRP_INST(MODE_MIX, double, 4)
CRP_INST(MODE_FP64, float, 0)
CRP_INST(MODE_FP64, float, 2)
CRP_INST(MODE_MIX, double, 0)
CRP_INST(MODE_MIX, double, 2)
CRP_INST(MODE_MIX, float, 0)
CRP_INST(MODE_MIX, float, 2)
#undef CRP_INST
// neural field (precision form, one block of 256 per CU: the network fills LDS)
template __global__ void k_propagate<MODE_MIX, float, 3, 256, false>(const PropParams*);
template __global__ void k_propagate<MODE_MIX, float, 3, 256, true>(const PropParams*);

// -------------------------------------------------------------------------
// Injection: validation (first bad index) and slot initialisation.
// -------------------------------------------------------------------------
__global__ void k_validate(int64_t n, const uint32_t* id, const int32_t* A, const int32_t* Z,
                           const double* E, const double* pos, const double* dir,
                           const double* lmax, double max_extent,
                           unsigned long long* first_bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    bool ok = A[i] >= 1 && A[i] <= 255 && Z[i] >= 1 && Z[i] <= A[i];
    ok = ok && isfinite(E[i]) && E[i] > 0.0 && isfinite(lmax[i]) && lmax[i] > 0.0;
    double d2 = 0.0, p2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        ok = ok && isfinite(pos[3 * i + a]) && isfinite(dir[3 * i + a]);
        d2 += dir[3 * i + a] * dir[3 * i + a];
        p2 += pos[3 * i + a] * pos[3 * i + a];
    }
    ok = ok && fabs(sqrt(d2) - 1.0) <= 1e-12;
    ok = ok && (sqrt(p2) + lmax[i] < max_extent);
    (void)id;
    if (!ok)
        atomicMin(first_bad, (unsigned long long)i);
}

// Queue slot base + i takes input candidate perm[i] (perm null: candidate i).
__global__ void k_inject(QueueSoA q, int64_t base, int64_t n, const uint32_t* id,
                         const int32_t* A, const int32_t* Z, const double* E,
                         const double* pos, const double* dir, const double* lmax,
                         const uint32_t* perm, uint64_t seed, double hmin, int mix)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t s = perm ? (int64_t)perm[i] : i;
    Cand c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.x[a] = pos[3 * s + a];
        const double d = dir[3 * s + a];
        c.u[a] = mix ? (double)(float)d : d;
        c.u0[a] = c.u[a];
    }
    c.E = E[s];
    c.E0 = E[s];
    c.L = 0.0;
    c.Lmax = lmax[s];
    c.hctrl = hmin;
    c.id = id[s];
    c.lineage = 0;
    c.m = 0;
    c.nsteps = 0;
    c.nrej = 0;
    c.A = A[s];
    c.Z = Z[s];
    c.tau = optical_depth(event_draw(seed, c.id, 0, 0).w[1]);
    store_cand(q, base + i, c);
}

// Sort keys of the longest-expected-path-first injection order: w = lmax * Z / E
// (> 0 and finite for a validated candidate) descending, i.e. the bitwise
// complement of w's IEEE pattern ascending (positive doubles order like their
// bit patterns); idx = 0..n-1, the payload the sort permutes.
__global__ void k_inject_keys(int64_t n, const int32_t* Z, const double* E, const double* lmax,
                              unsigned long long* keys, uint32_t* idx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double w = lmax[i] * (double)Z[i] / E[i];
    keys[i] = ~(unsigned long long)__double_as_longlong(w);
    idx[i] = (uint32_t)i;
}

// -------------------------------------------------------------------------
// Field evaluation at arbitrary points (mode 0: FP64 weights, 1: FP32).
// -------------------------------------------------------------------------
template <class GT, int LAYOUT>
__global__ void k_eval_field(GridView g, int64_t n, const double* pos, double* B, int mode)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const GridField<GT, LAYOUT> F{g};
    const double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    if (mode == MODE_FP64) {
        double b[3];
        F.fp64(p, b);
        B[3 * i] = b[0];
        B[3 * i + 1] = b[1];
        B[3 * i + 2] = b[2];
    } else {
        float b[3];
        F.fp32(p, b);
        B[3 * i] = (double)b[0];
        B[3 * i + 1] = (double)b[1];
        B[3 * i + 2] = (double)b[2];
    }
}

template __global__ void k_eval_field<double, 0>(GridView, int64_t, const double*, double*, int);

// The multi-resolution grid at n positions (patch table staged in LDS).
template <class GT>
__global__ void k_eval_nested(GridView g, NestView nv, int64_t n, const double* pos, double* B,
                              int mode)
{
    __shared__ PatchView P[MAX_PATCHES];
    if ((int)threadIdx.x < nv.np)
        P[threadIdx.x] = nv.p[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    NestedField<GT> F;
    F.g = g;
    F.P = P;
    F.np = nv.np;
    const double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    if (mode == MODE_FP64) {
        double b[3];
        F.fp64(p, b);
        B[3 * i] = b[0];
        B[3 * i + 1] = b[1];
        B[3 * i + 2] = b[2];
    } else {
        float b[3];
        F.fp32(p, b);
        B[3 * i] = (double)b[0];
        B[3 * i + 1] = (double)b[1];
        B[3 * i + 2] = (double)b[2];
    }
}
template __global__ void k_eval_nested<double>(GridView, NestView, int64_t, const double*, double*,
                                               int);
template __global__ void k_eval_nested<float>(GridView, NestView, int64_t, const double*, double*,
                                              int);
template __global__ void k_eval_field<float, 0>(GridView, int64_t, const double*, double*, int);
template __global__ void k_eval_field<float, 1>(GridView, int64_t, const double*, double*, int);

// -------------------------------------------------------------------------
// The analytic field at n positions (FP64).
__global__ void k_eval_analytic(AnalyticParams a, int64_t n, const double* __restrict__ pos,
                                double* __restrict__ B)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    AnalyticFieldSrc F;
    F.a = a;
    const double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    double b[3];
    F.fp64(p, b);
    B[3 * i] = b[0];
    B[3 * i + 1] = b[1];
    B[3 * i + 2] = b[2];
}

// -------------------------------------------------------------------------
// Diagnostic (not a step of the method): the field-gather pattern alone.
// Every wave repeatedly gathers the corner records of 64 pseudo-random cells
// with the propagation kernel's cooperative gather and folds one value of
// each into a checksum, so the rate it reaches is the practical ceiling of
// the field evaluation on this buffer.
// -------------------------------------------------------------------------
__device__ inline uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(128) k_gather_ceiling(const float* corner, uint32_t ncell,
                                                        int iters, float* sink)
{
    __shared__ float4 stage[2 * COOP_STAGE_FLOAT4];
    const int t = (int)threadIdx.x;
    float* st = (float*)(stage + (t >> 6) * COOP_STAGE_FLOAT4);
    uint32_t s = mix32((uint32_t)blockIdx.x * 128u + (uint32_t)t + 0x9e3779b9u);
    float acc = 0.0f;
    for (int it = 0; it < iters; ++it) {
        s = mix32(s + 0x9e3779b9u);
        const uint32_t cell = (uint32_t)(((uint64_t)s * ncell) >> 32);   // < ncell
        float v[8][3];
        gather_corner_coop(corner, cell, st, v, true);
        acc += v[t & 7][0];
    }
    sink[(int64_t)blockIdx.x * 128 + t] = acc;
}

// -------------------------------------------------------------------------
// Corner-replicated layout: record of cell (i,j,k) = the 8 corner vectors
// (c = dx + 2 dy + 4 dz) of the linear grid, as 24 values of the grid's
// element type: FP32 padded to 128 bytes (32 floats), FP64 unpadded (192 bytes).
template <class GT>
__global__ void k_corner_relayout(GridView g, GT* out)
{
    constexpr int RL = sizeof(GT) == 8 ? 24 : 32;   // elements per record
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const GT* G = (const GT*)g.data;
    for (int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cell < ncell;
         cell += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(cell % g.n[2]);
        const int j = (int)((cell / g.n[2]) % g.n[1]);
        const int i = (int)(cell / ((int64_t)g.n[1] * g.n[2]));
        GT rec[RL];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ii = (i + (c & 1)) % g.n[0];
            const int jj = (j + ((c >> 1) & 1)) % g.n[1];
            const int kk = (k + ((c >> 2) & 1)) % g.n[2];
            const GT* p = G + (int64_t)ii * g.stride[0] + (int64_t)jj * g.stride[1] +
                          (int64_t)kk * 3;
            rec[3 * c] = p[0];
            rec[3 * c + 1] = p[1];
            rec[3 * c + 2] = p[2];
        }
#pragma unroll
        for (int q = 24; q < RL; ++q)
            rec[q] = (GT)0;
        if constexpr (sizeof(GT) == 8) {
            double2* o = (double2*)(out + cell * RL);
#pragma unroll
            for (int q = 0; q < RL / 2; ++q)
                o[q] = make_double2(rec[2 * q], rec[2 * q + 1]);
        } else {
            float4* o = (float4*)(out + cell * RL);
#pragma unroll
            for (int q = 0; q < RL / 4; ++q)
                o[q] = make_float4(rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]);
        }
    }
}
template __global__ void k_corner_relayout<float>(GridView, float*);
template __global__ void k_corner_relayout<double>(GridView, double*);

}  // namespace crp
