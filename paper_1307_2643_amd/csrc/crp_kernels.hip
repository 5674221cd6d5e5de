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

namespace crp {

enum { LIM_CTRL = 0, LIM_TRAJ = 1, LIM_INTER = 2, LIM_LOSS = 3, LIM_OBS = 4 };
enum { ST_ACTIVE = 0, ST_OBSERVED = 1, ST_MAX_TRAJ = 2, ST_ENERGY_FLOOR = 3 };

struct Cand {
    double x[3], u[3], u0[3];
    double E, L, Lmax, hctrl, tau, E0;
    uint32_t id, lineage, m, nsteps, nrej;
    int A, Z;
};

__device__ inline void load_cand(const QueueSoA& q, int64_t i, Cand& c)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.x[a] = q.x[a * q.cap + i];
        c.u[a] = q.u[a * q.cap + i];
        c.u0[a] = q.u0[a * q.cap + i];
    }
    c.E = q.E[i];
    c.L = q.L[i];
    c.Lmax = q.Lmax[i];
    c.hctrl = q.hctrl[i];
    c.tau = q.tau[i];
    c.E0 = q.E0[i];
    c.id = q.id[i];
    c.lineage = q.lineage[i];
    c.m = q.m[i];
    c.nsteps = q.nsteps[i];
    c.nrej = q.nrej[i];
    c.A = q.A[i];
    c.Z = q.Z[i];
}

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

__device__ inline void store_finished(const FinishedSoA& f, int64_t i, const Cand& c,
                                      int status)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f.x[a * f.cap + i] = c.x[a];
        f.u[a * f.cap + i] = c.u[a];
        f.u0[a * f.cap + i] = c.u0[a];
    }
    f.E[i] = c.E;
    f.L[i] = c.L;
    f.E0[i] = c.E0;
    f.id[i] = c.id;
    f.lineage[i] = c.lineage;
    f.m[i] = c.m;
    f.nsteps[i] = c.nsteps;
    f.nrej[i] = c.nrej;
    f.status[i] = status;
    f.A[i] = c.A;
    f.Z[i] = c.Z;
}

struct LaneCount {
    uint32_t steps, attempts, rejects, forced;
    uint32_t events, null_events, inter_pi, inter_n;
    uint32_t charged_sec, neutral_sec;
    uint32_t finished, observed, max_traj, energy_floor;
    uint32_t queue_dropped, neutral_dropped;
};

__device__ inline unsigned long long wave_sum(uint32_t v)
{
    unsigned long long s = v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off);
    return s;
}

__device__ inline void flush_counts(DevCounters* cnt, const LaneCount& lc)
{
    const uint32_t* v = (const uint32_t*)&lc;
    unsigned long long* d = &cnt->steps;
    const int nf = (int)(sizeof(LaneCount) / sizeof(uint32_t));
    // steps .. neutral_sec map to consecutive device fields; the rest below
    unsigned long long sums[sizeof(LaneCount) / sizeof(uint32_t)];
#pragma unroll
    for (int i = 0; i < nf; ++i)
        sums[i] = wave_sum(v[i]);
    if (lane_id() == 0) {
#pragma unroll
        for (int i = 0; i < 10; ++i)
            if (sums[i])
                atomicAdd(d + i, sums[i]);
        if (sums[10])
            atomicAdd(&cnt->finished, sums[10]);
        if (sums[11])
            atomicAdd(&cnt->observed, sums[11]);
        if (sums[12])
            atomicAdd(&cnt->max_traj, sums[12]);
        if (sums[13])
            atomicAdd(&cnt->energy_floor, sums[13]);
        if (sums[14])
            atomicAdd(&cnt->queue_dropped, sums[14]);
        if (sums[15])
            atomicAdd(&cnt->neutral_dropped, sums[15]);
    }
}

// Claims up to `want` queue slots in [head, min(tail, cap)).
__device__ inline void claim_slots(DevCounters* cnt, unsigned long long cap, int want,
                                   unsigned long long& base, unsigned long long& take)
{
    unsigned long long h = __hip_atomic_load(&cnt->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        unsigned long long t =
            __hip_atomic_load(&cnt->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t > cap)
            t = cap;
        if (h >= t) {
            base = h;
            take = 0;
            return;
        }
        unsigned long long n = t - h;
        if (n > (unsigned long long)want)
            n = (unsigned long long)want;
        if (__hip_atomic_compare_exchange_strong(&cnt->head, &h, h + n, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            base = h;
            take = n;
            return;
        }
    }
}

// Waits until a slot appended during this run is published.  The producer
// writes the slot and publishes it in the same straight-line code right after
// reserving it, so the wait is short; it is bounded all the same.
__device__ inline bool wait_published(uint32_t* flag, DevCounters* cnt)
{
    for (uint32_t spin = 0; spin < (1u << 26); ++spin) {
        if (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            *flag = 0u;   // clean for the next run
            return true;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    atomicAdd(&cnt->error, 1ull);
    return false;
}

template <int MODE, class GT, int LAYOUT>
__global__ void __launch_bounds__(512) k_propagate(PropParams P)
{
    extern __shared__ double lds_tab[];
    const int ntab = P.tab.n;
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) {
        lds_tab[i] = P.tab.e[i];
        lds_tab[ntab + i] = P.tab.v[0][i];
        lds_tab[2 * ntab + i] = P.tab.v[1][i];
        lds_tab[3 * ntab + i] = P.tab.v[2][i];
    }
    __syncthreads();
    TableView T;
    T.e = lds_tab;
    T.v[0] = lds_tab + ntab;
    T.v[1] = lds_tab + 2 * ntab;
    T.v[2] = lds_tab + 3 * ntab;
    T.n = ntab;
    T.lg0 = P.tab.lg0;
    T.scale = P.tab.scale;

    const GridField<GT, LAYOUT> F{P.grid};
    const StepParams S = P.sp;
    const int lane = lane_id();
    const unsigned long long qcap = (unsigned long long)P.q.cap;

    bool active = false;
    bool fresh = true;
    Cand c;
    int64_t cycles = 0;
    double h = 0.0, kappa = 0.0, R = 0.0, beta = 0.0;
    int flag = LIM_CTRL;
    LaneCount lc = {};
    int iter = 0;
    bool dry = false;

    for (;;) {
        // ---- refill idle lanes from the queue -------------------------------
        const uint64_t idle = __ballot(!active);
        if (idle != 0ull && (idle == ~0ull || (!dry && iter % P.quantum == 0))) {
            const int want = __popcll(idle);
            unsigned long long base = 0, take = 0;
            if (lane == 0)
                claim_slots(P.cnt, qcap, want, base, take);
            base = __shfl(base, 0);
            take = __shfl(take, 0);
            dry = take < (unsigned long long)want;
            if (!active) {
                const int rank = lanes_below(idle);
                if ((unsigned long long)rank < take) {
                    const unsigned long long slot = base + (unsigned long long)rank;
                    bool ok = true;
                    if (slot >= P.tail0)
                        ok = wait_published(P.q.ready + slot, P.cnt);
                    if (ok) {
                        load_cand(P.q, (int64_t)slot, c);
                        active = true;
                        fresh = true;
                        cycles = 0;
                    }
                }
            }
            if (__ballot(active) == 0ull)
                break;
        }
        ++iter;

        // ---- start of a cycle: rates and step proposal -----------------------
        if (active && fresh) {
            const Rates rt = species_rates(T, c.A, c.Z, c.E);
            R = rt.r;
            beta = rt.beta;
            h = c.hctrl;
            flag = LIM_CTRL;
            if (c.Lmax - c.L < h) {
                h = c.Lmax - c.L;
                flag = LIM_TRAJ;
            }
            if (R > 0.0 && c.tau / R < h) {
                h = c.tau / R;
                flag = LIM_INTER;
            }
            if (beta > 0.0 && S.eps_loss / beta < h) {
                h = S.eps_loss / beta;
                flag = LIM_LOSS;
            }
            if (S.obs_r > 0.0) {
                const double d[3] = {c.x[0] - S.obs[0], c.x[1] - S.obs[1], c.x[2] - S.obs[2]};
                const double dist = sqrt(dot3(d, d));
                const double half = 0.5 * S.obs_r;
                double hob = dist - half;
                if (hob < half)
                    hob = half;
                if (hob < h) {
                    h = hob;
                    flag = LIM_OBS;
                }
            }
            kappa = ((double)c.Z * kC) / c.E;
            fresh = false;
        }

        // ---- one Cash-Karp attempt and, if accepted, the rest of the cycle ---
        bool fin = false, neutral = false, spawn = false, park = false;
        int status = ST_ACTIVE;
        double dE = 0.0, Esec = 0.0;
        if (active) {
            double x5[3], u5[3], err;
            if constexpr (MODE == MODE_FP64) {
                const double y[6] = {c.x[0], c.x[1], c.x[2], c.u[0], c.u[1], c.u[2]};
                double y5[6];
                err = ck_attempt_fp64(F, kappa, y, h, y5);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    x5[q] = y5[q];
                    u5[q] = y5[3 + q];
                }
            } else {
                err = ck_attempt_mix(F, kappa, c.x, c.u, h, x5, u5);
            }
            lc.attempts++;
            const double r = err / S.tol;
            if (r <= 1.0 || h <= S.hmin) {
                if (r > 1.0)
                    lc.forced++;
                double fac = 5.0;
                if (r > 0.0) {
                    fac = (double)ctrl_k(r) / 1024.0;
                    if (fac > 5.0)
                        fac = 5.0;
                }
                double hn = h * fac;
                if (hn < S.hmin)
                    hn = S.hmin;
                if (hn > S.hmax)
                    hn = S.hmax;
                c.hctrl = hn;
                // integration module: position, direction, trajectory length
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    c.x[q] = x5[q];
                if (S.renorm) {
                    if constexpr (MODE == MODE_FP64) {
                        const double nrm = sqrt(dot3(u5, u5));
#pragma unroll
                        for (int q = 0; q < 3; ++q)
                            c.u[q] = u5[q] / nrm;
                    } else {
                        const float uf[3] = {(float)u5[0], (float)u5[1], (float)u5[2]};
                        const float nrm = sqrtf(dot3f(uf, uf));
#pragma unroll
                        for (int q = 0; q < 3; ++q)
                            c.u[q] = (double)(uf[q] / nrm);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        c.u[q] = u5[q];
                }
                c.L = c.L + h;
                c.nsteps++;
                lc.steps++;
                // continuous loss: (2,2) Pade form of exp(-beta h)
                {
                    const double z = beta * h;
                    const double z2 = z * z;
                    const double num = (12.0 - 6.0 * z) + z2;
                    const double den = (12.0 + 6.0 * z) + z2;
                    c.E = c.E * (num / den);
                }
                // stochastic interactions: optical-depth clock
                c.tau = c.tau - R * h;
                if (flag == LIM_INTER || c.tau <= 0.0) {
                    c.m++;
                    const U64x4 w = event_draw(S.seed, c.id, c.lineage, c.m);
                    const double Eint = c.E;
                    const Rates ri = species_rates(T, c.A, c.Z, Eint);
                    const double Ptot = ri.rpi + ri.rn;
                    lc.events++;
                    if (Ptot > 0.0) {
                        const double Uc = unit_uniform(w.w[0]);
                        if (Uc * Ptot < ri.rpi) {
                            dE = (S.kappa_pi * Eint) / (double)c.A;
                            c.E = Eint - dE;
                            lc.inter_pi++;
                            lc.neutral_sec++;
                            neutral = true;
                        } else {
                            const int pout = (2 * c.Z > c.A) ? 1 : 0;
                            const int Aold = c.A;
                            Esec = Eint / (double)Aold;
                            c.Z -= pout;
                            c.A -= 1;
                            c.E = Eint - Esec;
                            lc.inter_n++;
                            lc.charged_sec++;
                            spawn = true;
                        }
                    } else {
                        lc.null_events++;
                    }
                    // all interaction state is reset after an interaction
                    c.tau = optical_depth(w.w[1]);
                }
                // boundary and observer modules, checked after the cycle
                ++cycles;
                if (S.obs_r > 0.0) {
                    const double d[3] = {c.x[0] - S.obs[0], c.x[1] - S.obs[1],
                                         c.x[2] - S.obs[2]};
                    if (sqrt(dot3(d, d)) <= S.obs_r)
                        status = ST_OBSERVED;
                }
                if (status == ST_ACTIVE && (flag == LIM_TRAJ || c.L >= c.Lmax))
                    status = ST_MAX_TRAJ;
                if (status == ST_ACTIVE && c.E < S.e_floor)
                    status = ST_ENERGY_FLOOR;
                if (status != ST_ACTIVE) {
                    fin = true;
                    lc.finished++;
                    if (status == ST_OBSERVED)
                        lc.observed++;
                    else if (status == ST_MAX_TRAJ)
                        lc.max_traj++;
                    else
                        lc.energy_floor++;
                } else if (P.max_cycles > 0 && cycles >= P.max_cycles) {
                    park = true;
                }
                fresh = true;
            } else {
                lc.rejects++;
                c.nrej++;
                double fac = (double)ctrl_k(r) / 1024.0;
                if (fac < 0.1)
                    fac = 0.1;
                h = h * fac;
                if (h < S.hmin)
                    h = S.hmin;
                flag = LIM_CTRL;
            }
        }

        // ---- appends: one atomic per wave for each kind ----------------------
        {
            const uint64_t mk = __ballot(neutral);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&P.cnt->neu_n, (unsigned long long)__popcll(mk));
                base = __shfl(base, 0);
                if (neutral) {
                    const unsigned long long i = base + (unsigned long long)lanes_below(mk);
                    if (i < (unsigned long long)P.neu.cap) {
                        const int64_t k = (int64_t)i;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            P.neu.x[a * P.neu.cap + k] = c.x[a];
                            P.neu.u[a * P.neu.cap + k] = c.u[a];
                        }
                        P.neu.E[k] = dE;
                        P.neu.id[k] = c.id;
                        P.neu.lineage[k] = c.lineage;
                        P.neu.m[k] = c.m;
                        P.neu.chan[k] = 0;
                    } else {
                        lc.neutral_dropped++;
                    }
                }
            }
        }
        {
            const uint64_t mk = __ballot(spawn);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&P.cnt->tail, (unsigned long long)__popcll(mk));
                base = __shfl(base, 0);
                if (spawn) {
                    const unsigned long long i = base + (unsigned long long)lanes_below(mk);
                    if (i < qcap) {
                        Cand s;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            s.x[a] = c.x[a];
                            s.u[a] = c.u[a];
                            s.u0[a] = c.u0[a];
                        }
                        s.E = Esec;
                        s.L = c.L;
                        s.Lmax = c.Lmax;
                        s.hctrl = S.hmin;
                        s.E0 = c.E0;
                        s.id = c.id;
                        s.lineage = c.m;
                        s.m = 0;
                        s.nsteps = 0;
                        s.nrej = 0;
                        s.A = 1;
                        s.Z = 1;
                        s.tau = optical_depth(event_draw(S.seed, s.id, s.lineage, 0).w[1]);
                        store_cand(P.q, (int64_t)i, s);
                        __hip_atomic_store(P.q.ready + i, 1u, __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        lc.queue_dropped++;
                    }
                }
            }
        }
        {
            const uint64_t mk = __ballot(fin);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&P.cnt->fin_n, (unsigned long long)__popcll(mk));
                base = __shfl(base, 0);
                if (fin) {
                    const unsigned long long i = base + (unsigned long long)lanes_below(mk);
                    if (i < (unsigned long long)P.fin.cap)
                        store_finished(P.fin, (int64_t)i, c, status);
                    active = false;
                }
            }
        }
        {
            const uint64_t mk = __ballot(park);
            if (mk) {
                unsigned long long base = 0;
                if (lane == 0)
                    base = atomicAdd(&P.cnt->park_n, (unsigned long long)__popcll(mk));
                base = __shfl(base, 0);
                if (park) {
                    const unsigned long long i = base + (unsigned long long)lanes_below(mk);
                    if (i < (unsigned long long)P.park.cap)
                        store_cand(P.park, (int64_t)i, c);
                    active = false;
                }
            }
        }
    }
    flush_counts(P.cnt, lc);
}

// Explicit instantiations: FP64 / mixed stage arithmetic x grid element type x
// grid layout (corner records exist for FP32 grids only).
template __global__ void k_propagate<MODE_FP64, double, 0>(PropParams);
template __global__ void k_propagate<MODE_FP64, float, 0>(PropParams);
template __global__ void k_propagate<MODE_FP64, float, 1>(PropParams);
template __global__ void k_propagate<MODE_MIX, double, 0>(PropParams);
template __global__ void k_propagate<MODE_MIX, float, 0>(PropParams);
template __global__ void k_propagate<MODE_MIX, float, 1>(PropParams);

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

__global__ void k_inject(QueueSoA q, int64_t base, int64_t n, const uint32_t* id,
                         const int32_t* A, const int32_t* Z, const double* E,
                         const double* pos, const double* dir, const double* lmax,
                         uint64_t seed, double hmin, int mix)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    Cand c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.x[a] = pos[3 * i + a];
        const double d = dir[3 * i + a];
        c.u[a] = mix ? (double)(float)d : d;
        c.u0[a] = c.u[a];
    }
    c.E = E[i];
    c.E0 = E[i];
    c.L = 0.0;
    c.Lmax = lmax[i];
    c.hctrl = hmin;
    c.id = id[i];
    c.lineage = 0;
    c.m = 0;
    c.nsteps = 0;
    c.nrej = 0;
    c.A = A[i];
    c.Z = Z[i];
    c.tau = optical_depth(event_draw(seed, c.id, 0, 0).w[1]);
    store_cand(q, base + i, c);
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
template __global__ void k_eval_field<float, 0>(GridView, int64_t, const double*, double*, int);
template __global__ void k_eval_field<float, 1>(GridView, int64_t, const double*, double*, int);

// -------------------------------------------------------------------------
// Corner-replicated layout: record of cell (i,j,k) = the 8 corner vectors
// (c = dx + 2 dy + 4 dz) of an FP32 linear grid, padded to 128 bytes.
// -------------------------------------------------------------------------
__global__ void k_corner_relayout(GridView g, float* out)
{
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const float* G = (const float*)g.data;
    for (int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cell < ncell;
         cell += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(cell % g.n[2]);
        const int j = (int)((cell / g.n[2]) % g.n[1]);
        const int i = (int)(cell / ((int64_t)g.n[1] * g.n[2]));
        float rec[32];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ii = (i + (c & 1)) % g.n[0];
            const int jj = (j + ((c >> 1) & 1)) % g.n[1];
            const int kk = (k + ((c >> 2) & 1)) % g.n[2];
            const float* p = G + (int64_t)ii * g.stride[0] + (int64_t)jj * g.stride[1] +
                             (int64_t)kk * 3;
            rec[3 * c] = p[0];
            rec[3 * c + 1] = p[1];
            rec[3 * c + 2] = p[2];
        }
#pragma unroll
        for (int q = 24; q < 32; ++q)
            rec[q] = 0.0f;
        float4* o = (float4*)(out + cell * 32);
#pragma unroll
        for (int q = 0; q < 8; ++q)
            o[q] = make_float4(rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]);
    }
}

}  // namespace crp
