/*
 * Exercises the CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built and run by tests/test_oracle_sanitizers.py; test infrastructure).
 *
 * Every path of the oracle is driven with small synthetic inputs made here
 * from a splitmix64 stream: FP64 and precision forms on FP64 and FP32 grids,
 * interactions with secondaries and full record buffers, an observer, a fixed
 * step that flings candidates far beyond the box, refinement patches, the
 * analytic galactic field with backtracking and a boundary, per-step output
 * past its capacity, cycle caps, and the single-call entry points at special
 * values (non-finite and far positions, NaN and infinite error ratios, the
 * extreme random words, table ends).  It prints one line of integer counters
 * per scenario and a checksum of every output, so the same program built
 * without sanitizers must print the same text.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "crp_oracle.h"

#define MPC 3.0856775814913673e22
#define KPC 3.0856775814913673e19
#define PC 3.0856775814913673e16

static uint64_t sm_state = 0x243F6A8885A308D3ull;
static uint64_t splitmix(void)
{
    uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double unif(void) { return (double)(splitmix() >> 11) * 0x1p-53; }
static double gauss(void)
{
    double a = unif(), b = unif();
    return sqrt(-2.0 * log(a + 1e-300)) * cos(6.283185307179586 * b);
}

/* checksum of doubles by their bits, order-independent (records come in
 * thread order) */
static uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    return x;
}
static uint64_t sum_bits(const double* v, int64_t n)
{
    uint64_t s = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t b;
        memcpy(&b, &v[i], 8);
        s += mix64(b);
    }
    return s;
}

typedef struct {
    int64_t n;
    uint32_t* id;
    int32_t *A, *Z;
    double *E, *pos, *dir, *lmax;
} inj_t;

static inj_t make_inj(int64_t n, double e_lo, double e_hi, double pos_scale, double lmax)
{
    static const int sp[4][2] = {{1, 1}, {4, 2}, {14, 7}, {56, 26}};
    inj_t j;
    j.n = n;
    j.id = malloc(n * sizeof *j.id);
    j.A = malloc(n * sizeof *j.A);
    j.Z = malloc(n * sizeof *j.Z);
    j.E = malloc(n * sizeof *j.E);
    j.pos = malloc(3 * n * sizeof *j.pos);
    j.dir = malloc(3 * n * sizeof *j.dir);
    j.lmax = malloc(n * sizeof *j.lmax);
    for (int64_t i = 0; i < n; ++i) {
        j.id[i] = (uint32_t)i;
        j.A[i] = sp[i % 4][0];
        j.Z[i] = sp[i % 4][1];
        j.E[i] = e_lo * pow(e_hi / e_lo, unif());
        double d[3] = {gauss(), gauss(), gauss()};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int q = 0; q < 3; ++q) {
            j.dir[3 * i + q] = d[q] / r;
            j.pos[3 * i + q] = pos_scale * (2.0 * unif() - 1.0);
        }
        j.lmax[i] = lmax;
    }
    return j;
}

static void free_inj(inj_t* j)
{
    free(j->id);
    free(j->A);
    free(j->Z);
    free(j->E);
    free(j->pos);
    free(j->dir);
    free(j->lmax);
}

typedef struct {
    or_finished f;
    or_neutral u;
    or_traj t;
} outs_t;

static void alloc_outs(outs_t* o, int64_t fcap, int64_t ncap, int64_t tcap)
{
    int64_t fc = fcap > 0 ? fcap : 1, nc = ncap > 0 ? ncap : 1, tc = tcap > 0 ? tcap : 1;
    o->f.cap = fcap;
    o->f.id = calloc(fc, 4);
    o->f.lineage = calloc(fc, 4);
    o->f.m = calloc(fc, 4);
    o->f.nsteps = calloc(fc, 4);
    o->f.nrej = calloc(fc, 4);
    o->f.status = calloc(fc, 4);
    o->f.A = calloc(fc, 4);
    o->f.Z = calloc(fc, 4);
    o->f.E = calloc(fc, 8);
    o->f.x = calloc(3 * fc, 8);
    o->f.u = calloc(3 * fc, 8);
    o->f.L = calloc(fc, 8);
    o->f.u0 = calloc(3 * fc, 8);
    o->f.E0 = calloc(fc, 8);
    o->u.cap = ncap;
    o->u.id = calloc(nc, 4);
    o->u.lineage = calloc(nc, 4);
    o->u.m = calloc(nc, 4);
    o->u.chan = calloc(nc, 4);
    o->u.E = calloc(nc, 8);
    o->u.x = calloc(3 * nc, 8);
    o->u.u = calloc(3 * nc, 8);
    o->t.cap = tcap;
    o->t.id = calloc(tc, 4);
    o->t.lineage = calloc(tc, 4);
    o->t.n = calloc(tc, 4);
    o->t.A = calloc(tc, 4);
    o->t.L = calloc(tc, 8);
    o->t.E = calloc(tc, 8);
    o->t.x = calloc(3 * tc, 8);
}

static void free_outs(outs_t* o)
{
    void* p[] = {o->f.id, o->f.lineage, o->f.m, o->f.nsteps, o->f.nrej, o->f.status, o->f.A,
                 o->f.Z, o->f.E, o->f.x, o->f.u, o->f.L, o->f.u0, o->f.E0, o->u.id,
                 o->u.lineage, o->u.m, o->u.chan, o->u.E, o->u.x, o->u.u, o->t.id,
                 o->t.lineage, o->t.n, o->t.A, o->t.L, o->t.E, o->t.x};
    for (size_t i = 0; i < sizeof p / sizeof p[0]; ++i)
        free(p[i]);
}

static or_config base_config(void)
{
    or_config c;
    memset(&c, 0, sizeof c);
    c.precision = OR_FP64;
    c.renormalize = 1;
    c.tol = 1e-4;
    c.hmin = 10 * KPC;
    c.hmax = 1 * MPC;
    c.eps_loss = 0.1;
    c.kappa_pi = 0.2;
    c.e_floor = 1e16;
    c.seed = 7;
    c.charge_sign = 1;
    return c;
}

static void run(const char* name, const or_config* cfg, const or_grid* g, const or_tables* t,
                const inj_t* j, int64_t fcap, int64_t ncap, int64_t tcap)
{
    outs_t o;
    alloc_outs(&o, fcap, ncap, tcap);
    or_counts cnt;
    int64_t nf = 0, nn = 0, nt = 0;
    oracle_propagate_traj(cfg, g, t, j->n, j->id, j->A, j->Z, j->E, j->pos, j->dir, j->lmax, 2,
                          &o.f, &o.u, &cnt, &nf, &nn, tcap > 0 ? &o.t : NULL,
                          tcap > 0 ? &nt : NULL);
    /* which records a full buffer keeps depends on the thread order: such a
     * buffer enters the checksum only through its counters */
    int64_t kf = nf <= fcap ? nf : 0, kn = nn <= ncap ? nn : 0, kt = nt <= tcap ? nt : 0;
    uint64_t h = sum_bits(o.f.x, 3 * kf) + sum_bits(o.f.E, kf) + sum_bits(o.f.L, kf) +
                 sum_bits(o.u.x, 3 * kn) + sum_bits(o.u.E, kn) + sum_bits(o.t.x, 3 * kt);
    printf("%s: finished %lld observed %lld max_traj %lld floor %lld boundary %lld active %lld "
           "steps %lld attempts %lld rejects %lld forced %lld events %lld pi %lld n %lld "
           "charged %lld neutral %lld fin_dropped %lld neu_dropped %lld traj %lld "
           "traj_dropped %lld sum %016llx\n",
           name, (long long)cnt.finished, (long long)cnt.observed, (long long)cnt.max_traj,
           (long long)cnt.energy_floor, (long long)cnt.boundary, (long long)cnt.still_active,
           (long long)cnt.steps, (long long)cnt.attempts, (long long)cnt.rejects,
           (long long)cnt.forced, (long long)cnt.events, (long long)cnt.inter_pi,
           (long long)cnt.inter_n, (long long)cnt.charged_sec, (long long)cnt.neutral_sec,
           (long long)cnt.fin_dropped, (long long)cnt.neu_dropped, (long long)nt,
           (long long)cnt.traj_dropped, (unsigned long long)h);
    free_outs(&o);
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

int main(void)
{
    /* grid 16^3, 100 kpc cells, ~1 nG random vertices; FP64 and FP32 copies */
    const int64_t N = 16;
    const int64_t nv = N * N * N * 3;
    double* g64 = malloc(nv * sizeof *g64);
    float* g32 = malloc(nv * sizeof *g32);
    for (int64_t i = 0; i < nv; ++i) {
        g64[i] = 1e-13 * gauss();
        g32[i] = (float)g64[i];
    }
    or_grid G64 = {g64, OR_GRID_F64, 0, {N, N, N}, 100 * KPC, {0, 0, 0}, NULL, 0, 0, NULL};
    or_grid G32 = G64;
    G32.data = g32;
    G32.dtype = OR_GRID_F32;

    /* tables: 200 log nodes 1e16..1e23 eV, sigmoid rates (per metre) */
    enum { NT = 200 };
    double e[NT], tpi[NT], tn[NT], bp[NT];
    for (int i = 0; i < NT; ++i) {
        e[i] = pow(10.0, 16.0 + 7.0 * i / (NT - 1));
        double lg = log10(e[i]);
        bp[i] = (4e-3 * sigmoid((lg - 18.6) / 0.25) + 1e-5) / MPC;
        tpi[i] = 0.25 * sigmoid((lg - 19.7) / 0.15) / MPC;
        tn[i] = 0.5 * sigmoid((lg - 18.7) / 0.2) / MPC;
    }
    or_tables T = {NT, 0, e, tpi, tn, bp};

    /* A/B: both forms with interactions, an observer and a small neutral buffer */
    inj_t mixed = make_inj(256, 1e18, 1e21, 0.0, 20 * MPC);
    or_config c = base_config();
    c.obs[0] = 3 * MPC;
    c.obs_r = 1 * MPC;
    run("fp64_grid64", &c, &G64, &T, &mixed, 4096, 16, 0);
    c.precision = OR_MIX;
    run("mix_grid32", &c, &G32, &T, &mixed, 4096, 16, 0);
    c.precision = OR_FP64;
    run("fp64_grid32", &c, &G32, &T, &mixed, 4096, 4096, 0);
    /* a finished-record buffer too small, and a cycle cap */
    run("fin_overflow", &c, &G64, &T, &mixed, 32, 4096, 0);
    c.max_cycles = 10;
    run("cycle_cap", &c, &G64, &T, &mixed, 4096, 4096, 0);
    c.max_cycles = 0;

    /* C: a fixed step with forced accepts at low energy (large error
     * estimates), starting far beyond the box and with a far-reaching
     * trajectory limit */
    inj_t far = make_inj(64, 1e16, 1e17, 1e9 * MPC, 1e3 * MPC);
    for (int64_t i = 0; i < far.n; ++i)
        for (int q = 0; q < 3; ++q)
            far.pos[3 * i + q] *= (i % 3 == 0) ? 1e12 : 1.0;
    or_config cf = base_config();
    cf.hmin = cf.hmax = 100 * KPC;
    cf.e_floor = 0.0;
    run("fixed_step_far", &cf, &G64, &T, &far, 4096, 4096, 0);
    cf.precision = OR_MIX;
    run("fixed_step_far_mix", &cf, &G32, &T, &far, 4096, 4096, 0);

    /* D: two refinement patches (refine 2 and 4) on both grid types */
    int64_t pn = 9;
    int64_t pv = pn * pn * pn * 3;
    double* p64 = malloc(pv * sizeof *p64);
    float* p32 = malloc(pv * sizeof *p32);
    for (int64_t i = 0; i < pv; ++i) {
        p64[i] = 1e-13 * gauss();
        p32[i] = (float)p64[i];
    }
    or_patch P64[2] = {{p64, {pn, pn, pn}, {4, 4, 4}, 2, 0}, {p64, {pn, pn, pn}, {5, 5, 5}, 4, 0}};
    or_patch P32[2] = {{p32, {pn, pn, pn}, {4, 4, 4}, 2, 0}, {p32, {pn, pn, pn}, {5, 5, 5}, 4, 0}};
    or_grid N64 = G64, N32 = G32;
    N64.n_patches = N32.n_patches = 2;
    N64.patches = P64;
    N32.patches = P32;
    inj_t nest = make_inj(128, 1e18, 1e20, 0.0, 10 * MPC);
    for (int64_t i = 0; i < nest.n; ++i)
        for (int q = 0; q < 3; ++q)
            nest.pos[3 * i + q] = 5.5 * 100 * KPC + 50 * KPC * (2.0 * unif() - 1.0);
    or_config cn = base_config();
    run("nested_fp64", &cn, &N64, &T, &nest, 4096, 4096, 0);
    cn.precision = OR_MIX;
    run("nested_mix", &cn, &N32, &T, &nest, 4096, 4096, 0);

    /* E: analytic field, backtracking (charge -Z) inside a 20 kpc boundary */
    or_analytic an = {{0, 0, 0}, 6e-10, 5 * KPC, 0.4 * KPC, 4e-10, 6 * KPC, 2 * KPC, 1.5e-10,
                      4 * KPC, 3 * KPC};
    or_grid GA = G64;
    GA.analytic = &an;
    inj_t gal = make_inj(128, 1e18, 1e20, 8.5 * KPC, 100 * KPC);
    or_config cg = base_config();
    cg.hmin = 1 * PC;
    cg.hmax = 1 * KPC;
    cg.charge_sign = -1;
    cg.bnd_r = 20 * KPC;
    or_tables T0 = {NT, 0, e, tpi, tn, bp};
    double zero[NT] = {0};
    T0.tpi = zero;
    T0.tn = zero;
    T0.bp = zero;
    run("galactic_back", &cg, &GA, &T0, &gal, 4096, 16, 0);
    cg.precision = OR_MIX;
    run("galactic_back_mix", &cg, &GA, &T0, &gal, 4096, 16, 0);

    /* F: per-step output past its capacity */
    or_config ct = base_config();
    ct.traj_every = 2;
    ct.traj_ids = 50;
    run("traj_overflow", &ct, &G64, &T, &mixed, 4096, 4096, 100);
    run("traj_roomy", &ct, &G64, &T, &mixed, 4096, 4096, 1 << 20);

    /* G: single calls at special values */
    double pos[8][3] = {{NAN, 0, 0},           {INFINITY, 1, 2},      {0, -INFINITY, 0},
                        {0x1p70, -0x1p63, 0x1p31}, {-0x1p62, 0x1p62, 1e300}, {1e-300, -0.0, 0.0},
                        {-1e-30, -1e-30, -1e-30}, {12345.6, -7.5, 0.25}};
    double B[8][3];
    uint64_t hs = 0;
    for (int m = 0; m < 2; ++m) {
        oracle_eval_field(&G64, m, 8, &pos[0][0], &B[0][0]);
        hs += sum_bits(&B[3][0], 15);
        oracle_eval_field(&N32, m, 8, &pos[0][0], &B[0][0]);
        hs += sum_bits(&B[3][0], 15);
        oracle_eval_field(&GA, m, 8, &pos[0][0], &B[0][0]);
    }
    double x5[3], u5[3], err;
    double u0[3] = {0.6, 0.0, 0.8};
    oracle_ck_attempt(&G64, OR_FP64, pos[7], u0, 299792458.0 / 1e19, 0.3 * MPC, x5, u5, &err);
    hs += sum_bits(x5, 3) + sum_bits(u5, 3);
    oracle_ck_attempt(&G32, OR_MIX, pos[3], u0, 299792458.0 / 1e19, 0.3 * MPC, x5, u5, &err);
    hs += sum_bits(x5, 3) + sum_bits(u5, 3);
    int32_t ks = oracle_ctrl_k(NAN) + oracle_ctrl_k(INFINITY) + oracle_ctrl_k(0.0) +
                 oracle_ctrl_k(1e-300) + oracle_ctrl_k(1e300) + oracle_ctrl_k(1.0);
    double tx = oracle_texp(0) + oracle_texp(~0ull) + oracle_texp(1ull << 11);
    double tl = oracle_table_lookup(&T, 0, 0.0) + oracle_table_lookup(&T, 1, INFINITY) +
                oracle_table_lookup(&T, 2, 1e16) + oracle_table_lookup(&T, 2, 1e23) +
                oracle_table_lookup(&T, 0, 3.3e19);
    double rt[4];
    oracle_rates(&T, 255, 255, 1e21, rt);
    uint64_t ctr[4] = {~0ull, ~0ull, ~0ull, ~0ull}, key[2] = {~0ull, 0}, ph[4];
    oracle_philox4x64(ctr, key, ph);
    printf("single: fields %016llx ctrl %d texp %.17g tables %.17g rates %.17g philox %016llx\n",
           (unsigned long long)hs, ks, tx, tl, rt[0] + rt[1] + rt[2] + rt[3],
           (unsigned long long)(ph[0] ^ ph[3]));

    free_inj(&mixed);
    free_inj(&far);
    free_inj(&nest);
    free_inj(&gal);
    free(g64);
    free(g32);
    free(p64);
    free(p32);
    printf("DRIVER DONE\n");
    return 0;
}
