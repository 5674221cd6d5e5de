// Drives the host runtime of libcrp through its C-ABI on small synthetic
// problems, for a build whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer (device code is built as usual).  Every section
// checks its own results; the program prints one line per section and exits
// non-zero at the first failure.  Covered: context set-up and the error
// paths of the argument checks, grid and table upload, injection (including
// an all-or-nothing refusal), propagation with a cycle budget and with a
// neutral-record buffer too small for the run, partial reads, checkpoint and
// restore against an uninterrupted run, the trajectory output, the autotuner
// and its cache, field evaluation with and without per-call allocation,
// observables, refinement patches, the neural field (loss and gradient, Adam,
// training, evaluation, propagation) and backtracking with lenses.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "crp.h"

namespace {

const double KPC = 3.0856775814913673e19;
const double MPC = 1e3 * KPC;

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);             \
            std::fprintf(stderr, "\n");                    \
            std::exit(1);                                  \
        }                                                  \
    } while (0)

#define OK(call)                                                                  \
    do {                                                                          \
        const crp_status s_ = (call);                                             \
        CHECK(s_ == CRP_OK, "%s -> %d", #call, (int)s_);                          \
    } while (0)

// Small deterministic generator (xorshift64*), uniform in [0, 1).
struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 1) {}
    double u()
    {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        return (double)((s * 0x2545F4914F6CDD1Dull) >> 11) * 0x1p-53;
    }
};

crp_config base_config(int precision)
{
    crp_config c;
    std::memset(&c, 0, sizeof c);
    c.precision = precision;
    c.field_mode = CRP_FIELD_GRID;
    c.renormalize = 1;
    c.device = 0;
    c.tol = 1e-4;
    c.hmin = 10 * KPC;
    c.hmax = 1 * MPC;
    c.eps_loss = 0.1;
    c.kappa_pi = 0.2;
    c.e_floor = 1e16;
    c.seed = 7;
    c.queue_capacity = 4096;
    c.neutral_capacity = 1 << 14;
    c.charge_sign = 1;
    return c;
}

struct Grid {
    int n = 16;
    double spacing = 100 * KPC;
    std::vector<float> f;
    std::vector<double> d;
};

Grid make_grid(uint64_t seed)
{
    Grid g;
    Rng r(seed);
    const size_t m = (size_t)g.n * g.n * g.n * 3;
    g.f.resize(m);
    g.d.resize(m);
    for (size_t i = 0; i < m; ++i) {
        g.d[i] = (2.0 * r.u() - 1.0) * 1e-13;
        g.f[i] = (float)g.d[i];
    }
    return g;
}

struct Tables {
    std::vector<double> e, tpi, tn, beta;
};

Tables make_tables()
{
    Tables t;
    const int n = 64;
    for (int j = 0; j < n; ++j) {
        const double e = std::pow(10.0, 16.0 + 7.0 * j / (n - 1));
        const double x = std::log10(e);
        t.e.push_back(e);
        t.tpi.push_back(0.25 / MPC / (1.0 + std::exp(-(x - 19.7) / 0.15)));
        t.tn.push_back(0.05 / MPC / (1.0 + std::exp(-(x - 18.7) / 0.2)));
        t.beta.push_back(4e-3 / MPC / (1.0 + std::exp(-(x - 18.6) / 0.25)) + 1e-5 / MPC);
    }
    return t;
}

struct Inj {
    std::vector<uint32_t> id;
    std::vector<int32_t> A, Z;
    std::vector<double> E, pos, dir, lmax;
    int64_t n() const { return (int64_t)id.size(); }
};

Inj make_injection(int64_t n, uint64_t seed, double box, double lmax)
{
    static const int AA[4] = {1, 4, 14, 56}, ZZ[4] = {1, 2, 7, 26};
    Inj j;
    Rng r(seed);
    for (int64_t i = 0; i < n; ++i) {
        j.id.push_back((uint32_t)i);
        j.A.push_back(AA[i % 4]);
        j.Z.push_back(ZZ[i % 4]);
        j.E.push_back(1e18 * std::pow(1e3, r.u()));
        double v[3], nrm = 0.0;
        for (int a = 0; a < 3; ++a) {
            j.pos.push_back(box * r.u());
            v[a] = 2.0 * r.u() - 1.0;
            nrm += v[a] * v[a];
        }
        nrm = std::sqrt(nrm);
        for (int a = 0; a < 3; ++a)
            j.dir.push_back(v[a] / nrm);
        j.lmax.push_back(lmax);
    }
    return j;
}

crp_status inject(crp_ctx* ctx, const Inj& j)
{
    return crp_inject(ctx, j.n(), j.id.data(), j.A.data(), j.Z.data(), j.E.data(),
                      j.pos.data(), j.dir.data(), j.lmax.data(), 0);
}

crp_ctx* make_ctx(const crp_config& c, const Grid& g, const Tables& t, bool fp32)
{
    crp_ctx* ctx = nullptr;
    OK(crp_create(&c, nullptr, &ctx));
    const double org[3] = {0.0, 0.0, 0.0};
    OK(crp_set_field_grid(ctx, fp32 ? (const void*)g.f.data() : (const void*)g.d.data(),
                          fp32 ? CRP_F32 : CRP_F64, 0, g.n, g.n, g.n, g.spacing, org));
    OK(crp_set_tables(ctx, (int32_t)t.e.size(), t.e.data(), t.tpi.data(), t.tn.data(),
                      t.beta.data()));
    return ctx;
}

// Finished records, read in chunks of `chunk`.
struct Records {
    std::vector<uint32_t> id, lineage, m, nsteps, nrej;
    std::vector<int32_t> status, A, Z;
    std::vector<double> E, x, u, L, u0, E0;
    size_t size() const { return id.size(); }
};

int64_t read_all(crp_ctx* ctx, Records& R, int64_t chunk)
{
    int64_t total = 0;
    for (;;) {
        std::vector<uint32_t> id(chunk), lin(chunk), m(chunk), ns(chunk), nr(chunk);
        std::vector<int32_t> st(chunk), A(chunk), Z(chunk);
        std::vector<double> E(chunk), x(3 * chunk), u(3 * chunk), L(chunk), u0(3 * chunk),
            E0(chunk);
        crp_finished_soa o{id.data(), lin.data(), m.data(), ns.data(), nr.data(), st.data(),
                           A.data(), Z.data(), E.data(), x.data(), u.data(), L.data(),
                           u0.data(), E0.data()};
        int64_t got = 0;
        const crp_status s = crp_read_finished(ctx, chunk, &o, &got);
        CHECK(s == CRP_OK || s == CRP_EOVERFLOW, "read_finished -> %d", (int)s);
        CHECK(got >= 0 && got <= chunk, "read_finished count %lld", (long long)got);
        R.id.insert(R.id.end(), id.begin(), id.begin() + got);
        R.lineage.insert(R.lineage.end(), lin.begin(), lin.begin() + got);
        R.m.insert(R.m.end(), m.begin(), m.begin() + got);
        R.nsteps.insert(R.nsteps.end(), ns.begin(), ns.begin() + got);
        R.nrej.insert(R.nrej.end(), nr.begin(), nr.begin() + got);
        R.status.insert(R.status.end(), st.begin(), st.begin() + got);
        R.A.insert(R.A.end(), A.begin(), A.begin() + got);
        R.Z.insert(R.Z.end(), Z.begin(), Z.begin() + got);
        R.E.insert(R.E.end(), E.begin(), E.begin() + got);
        R.x.insert(R.x.end(), x.begin(), x.begin() + 3 * got);
        R.u.insert(R.u.end(), u.begin(), u.begin() + 3 * got);
        R.L.insert(R.L.end(), L.begin(), L.begin() + got);
        R.u0.insert(R.u0.end(), u0.begin(), u0.begin() + 3 * got);
        R.E0.insert(R.E0.end(), E0.begin(), E0.begin() + got);
        total += got;
        if (s == CRP_OK)
            return total;
    }
}

int64_t drain_neutral(crp_ctx* ctx, int64_t chunk, std::vector<uint64_t>* keys)
{
    int64_t total = 0;
    for (;;) {
        std::vector<uint32_t> id(chunk), lin(chunk), m(chunk);
        std::vector<int32_t> ch(chunk);
        std::vector<double> E(chunk), x(3 * chunk), u(3 * chunk);
        crp_neutral_soa o{id.data(), lin.data(), m.data(), ch.data(), E.data(), x.data(),
                          u.data()};
        int64_t got = 0;
        const crp_status s = crp_read_neutral(ctx, chunk, &o, &got);
        CHECK(s == CRP_OK || s == CRP_EOVERFLOW, "read_neutral -> %d", (int)s);
        for (int64_t i = 0; i < got; ++i) {
            CHECK(std::isfinite(E[i]) && E[i] > 0, "neutral energy");
            if (keys)
                keys->push_back(((uint64_t)id[i] << 32) ^ ((uint64_t)lin[i] << 12) ^ m[i]);
        }
        total += got;
        if (s == CRP_OK)
            return total;
    }
}

// Propagates to completion, reading neutral records whenever their buffer is full.
void run_to_end(crp_ctx* ctx, int64_t budget, std::vector<uint64_t>* nkeys)
{
    for (int it = 0; it < 100000; ++it) {
        const crp_status s = crp_propagate(ctx, budget);
        if (s == CRP_OK)
            return;
        CHECK(s == CRP_INCOMPLETE || s == CRP_EOVERFLOW, "propagate -> %d", (int)s);
        if (s == CRP_EOVERFLOW)
            drain_neutral(ctx, 37, nkeys);
    }
    CHECK(false, "propagation did not finish");
}

std::vector<size_t> order(const Records& R)
{
    std::vector<size_t> o(R.size());
    std::iota(o.begin(), o.end(), 0);
    std::sort(o.begin(), o.end(), [&](size_t a, size_t b) {
        return R.id[a] != R.id[b] ? R.id[a] < R.id[b] : R.lineage[a] < R.lineage[b];
    });
    return o;
}

void same_records(const Records& P, const Records& Q, const char* what)
{
    CHECK(P.size() == Q.size(), "%s: %zu vs %zu records", what, P.size(), Q.size());
    const std::vector<size_t> a = order(P), b = order(Q);
    for (size_t k = 0; k < a.size(); ++k) {
        const size_t i = a[k], j = b[k];
        CHECK(P.id[i] == Q.id[j] && P.lineage[i] == Q.lineage[j] && P.m[i] == Q.m[j] &&
                  P.nsteps[i] == Q.nsteps[j] && P.nrej[i] == Q.nrej[j] &&
                  P.status[i] == Q.status[j] && P.A[i] == Q.A[j] && P.Z[i] == Q.Z[j],
              "%s: integer fields of record %zu", what, k);
        CHECK(P.E[i] == Q.E[j] && P.L[i] == Q.L[j] && P.E0[i] == Q.E0[j], "%s: E/L/E0 %zu", what,
              k);
        for (int a3 = 0; a3 < 3; ++a3)
            CHECK(P.x[3 * i + a3] == Q.x[3 * j + a3] && P.u[3 * i + a3] == Q.u[3 * j + a3] &&
                      P.u0[3 * i + a3] == Q.u0[3 * j + a3],
                  "%s: vectors of record %zu", what, k);
    }
}

void section_errors(const Grid& g, const Tables& t)
{
    crp_config c = base_config(CRP_MIX);
    crp_ctx* ctx = nullptr;
    crp_config bad = c;
    bad.hmin = 2 * c.hmax;
    CHECK(crp_create(&bad, nullptr, &ctx) == CRP_EINVAL && ctx == nullptr, "bad config accepted");
    CHECK(crp_create(nullptr, nullptr, &ctx) == CRP_EINVAL, "null config accepted");
    OK(crp_create(&c, nullptr, &ctx));
    // no field or tables yet
    CHECK(crp_propagate(ctx, 0) == CRP_ESTATE, "propagate without field");
    const Inj j = make_injection(8, 1, g.n * g.spacing, 5 * MPC);
    CHECK(inject(ctx, j) == CRP_ESTATE, "inject without field");
    const double org[3] = {0, 0, 0};
    CHECK(crp_set_field_grid(ctx, g.f.data(), CRP_F32, 0, 1, g.n, g.n, g.spacing, org) ==
              CRP_EINVAL,
          "grid of one vertex accepted");
    CHECK(crp_set_field_grid(ctx, g.f.data(), 7, 0, g.n, g.n, g.n, g.spacing, org) == CRP_EINVAL,
          "bad dtype accepted");
    std::vector<double> e2 = t.e;
    std::swap(e2[3], e2[4]);
    CHECK(crp_set_tables(ctx, (int32_t)e2.size(), e2.data(), t.tpi.data(), t.tn.data(),
                         t.beta.data()) == CRP_EINVAL,
          "non-monotone table accepted");
    crp_launch l{100, 0, 4, CRP_LAYOUT_LINEAR};
    CHECK(crp_set_launch(ctx, &l) == CRP_EINVAL, "block 100 accepted");
    l = crp_launch{128, 0, 0, CRP_LAYOUT_LINEAR};
    CHECK(crp_set_launch(ctx, &l) == CRP_EINVAL, "refill 0 accepted");
    const char* msg = crp_last_error(ctx);
    CHECK(msg && std::strlen(msg) > 0, "no error message");
    // an injection with one bad candidate changes nothing
    OK(crp_set_field_grid(ctx, g.f.data(), CRP_F32, 0, g.n, g.n, g.n, g.spacing, org));
    OK(crp_set_tables(ctx, (int32_t)t.e.size(), t.e.data(), t.tpi.data(), t.tn.data(),
                      t.beta.data()));
    Inj b = j;
    b.Z[5] = b.A[5] + 1;
    CHECK(inject(ctx, b) == CRP_EINVAL, "Z > A accepted");
    b = j;
    b.dir[3 * 2] *= 1.01;
    CHECK(inject(ctx, b) == CRP_EINVAL, "non-unit direction accepted");
    crp_counters cnt;
    OK(crp_counts(ctx, &cnt));
    CHECK(cnt.pending == 0, "refused injection left %lld pending", (long long)cnt.pending);
    OK(inject(ctx, j));
    OK(crp_counts(ctx, &cnt));
    CHECK(cnt.pending == j.n(), "pending %lld", (long long)cnt.pending);
    crp_destroy(ctx);
    crp_destroy(nullptr);
    crp_free(nullptr);
    std::printf("errors ok\n");
}

void section_propagate_restore(const Grid& g, const Tables& t, int precision)
{
    crp_config c = base_config(precision);
    c.neutral_capacity = 16;                // the run overflows it many times
    c.traj_every = 1;
    c.traj_ids = 4;
    c.traj_capacity = 1 << 16;
    const Inj j = make_injection(400, 2 + precision, g.n * g.spacing, 20 * MPC);
    // uninterrupted run
    crp_ctx* a = make_ctx(c, g, t, precision == CRP_MIX);
    OK(inject(a, j));
    std::vector<uint64_t> na;
    run_to_end(a, 0, &na);
    drain_neutral(a, 37, &na);
    Records ra;
    read_all(a, ra, 97);
    crp_counters ca;
    OK(crp_counts(a, &ca));
    CHECK((int64_t)ra.size() == ca.finished && ca.finished == j.n() + ca.charged_sec,
          "finished %zu vs %lld", ra.size(), (long long)ca.finished);
    CHECK((int64_t)na.size() == ca.neutral_sec && ca.neutral_sec > 16,
          "neutral %zu vs %lld", na.size(), (long long)ca.neutral_sec);
    // trajectory points of ids < 4
    int64_t pts = 0;
    for (;;) {
        const int64_t cap = 500;
        std::vector<uint32_t> id(cap), lin(cap), n(cap);
        std::vector<int32_t> A(cap);
        std::vector<double> L(cap), E(cap), x(3 * cap);
        crp_traj_soa o{id.data(), lin.data(), n.data(), A.data(), L.data(), E.data(), x.data()};
        int64_t got = 0;
        const crp_status s = crp_read_trajectory(a, cap, &o, &got);
        CHECK(s == CRP_OK || s == CRP_EOVERFLOW, "read_trajectory -> %d", (int)s);
        for (int64_t i = 0; i < got; ++i)
            CHECK(id[i] < 4 && n[i] > 0, "trajectory point of id %u", id[i]);
        pts += got;
        if (s == CRP_OK)
            break;
    }
    CHECK(pts == ca.traj_points && pts > 0, "trajectory points %lld", (long long)pts);
    // interrupted by a cycle budget, checkpointed, restored into a new context
    crp_ctx* b = make_ctx(c, g, t, precision == CRP_MIX);
    OK(inject(b, j));
    std::vector<uint64_t> nb;
    crp_status s = crp_propagate(b, 5);
    CHECK(s == CRP_INCOMPLETE || s == CRP_EOVERFLOW, "budget run -> %d", (int)s);
    if (s == CRP_EOVERFLOW)
        drain_neutral(b, 37, &nb);
    void* blob = nullptr;
    size_t bytes = 0;
    OK(crp_snapshot(b, &blob, &bytes));
    CHECK(blob && bytes > 0, "empty snapshot");
    CHECK(crp_restore(b, blob, bytes / 2) == CRP_EINVAL, "truncated snapshot accepted");
    crp_destroy(b);
    crp_ctx* r = make_ctx(c, g, t, precision == CRP_MIX);
    OK(crp_restore(r, blob, bytes));
    crp_free(blob);
    run_to_end(r, 3, &nb);
    drain_neutral(r, 37, &nb);
    Records rr;
    read_all(r, rr, 53);
    same_records(ra, rr, "restored run");
    std::sort(na.begin(), na.end());
    std::sort(nb.begin(), nb.end());
    CHECK(na == nb, "neutral records of the restored run differ");
    crp_destroy(a);
    crp_destroy(r);
    std::printf("propagate/restore (precision %d) ok: %zu records, %zu neutral, %lld points\n",
                precision, ra.size(), na.size(), (long long)pts);
}

void section_tune_eval_observe(const Grid& g, const Tables& t)
{
    crp_config c = base_config(CRP_MIX);
    crp_ctx* ctx = make_ctx(c, g, t, true);
    const Inj j = make_injection(300, 5, g.n * g.spacing, 10 * MPC);
    OK(inject(ctx, j));
    const char* tmp = std::getenv("TMPDIR");
    const std::string path = std::string(tmp ? tmp : "/tmp") + "/crp_sanitize_tune_cache.txt";
    std::remove(path.c_str());
    crp_launch l1, l2;
    double r1 = 0, r2 = 0;
    OK(crp_tune(ctx, 0, path.c_str(), &l1, &r1));
    OK(crp_tune(ctx, 0, path.c_str(), &l2, &r2));   // from the cache, no trials
    // the cache keeps the rate to seven significant digits
    CHECK(std::memcmp(&l1, &l2, sizeof l1) == 0 && r1 > 0 && std::fabs(r2 / r1 - 1.0) < 1e-6,
          "cache read-back");
    std::remove(path.c_str());
    run_to_end(ctx, 0, nullptr);
    // field evaluation with and without a per-call allocation
    const int64_t n = 5000;
    Rng rng(9);
    std::vector<double> pos(3 * n), B1(3 * n), B2(3 * n);
    for (auto& p : pos)
        p = (rng.u() * 3.0 - 1.0) * g.n * g.spacing;
    for (int mode : {CRP_FP64, CRP_MIX}) {
        OK(crp_eval_field(ctx, n, pos.data(), B1.data(), mode, 0));
        OK(crp_eval_field_noalloc(ctx, n, pos.data(), B2.data(), mode));
        CHECK(std::memcmp(B1.data(), B2.data(), B1.size() * 8) == 0, "noalloc differs");
    }
    CHECK(crp_eval_field_noalloc(ctx, CRP_EVAL_NOALLOC_MAX + 1, pos.data(), B2.data(), CRP_MIX) ==
              CRP_EINVAL,
          "oversized noalloc accepted");
    // observables over the finished records
    std::vector<double> ee;
    for (int k = 0; k <= 8; ++k)
        ee.push_back(1e16 * std::pow(10.0, 6.0 * k / 8));
    const int32_t ae[5] = {1, 2, 7, 28, 57};
    crp_observables spec{8, 4, ee.data(), ae, 0x1f, 4, 1.0, 1e18, -1.5};
    OK(crp_set_observables(ctx, &spec));
    OK(crp_observe(ctx, nullptr));
    std::vector<uint64_t> counts(32), defl(32), sky(32 * 6 * 16);
    std::vector<double> wsum(32);
    uint64_t outside = 0;
    OK(crp_read_observables(ctx, counts.data(), wsum.data(), defl.data(), sky.data(), &outside));
    crp_counters cnt;
    OK(crp_counts(ctx, &cnt));
    const uint64_t in = std::accumulate(counts.begin(), counts.end(), 0ull);
    const uint64_t insky = std::accumulate(sky.begin(), sky.end(), 0ull);
    CHECK((int64_t)(in + outside) == cnt.finished_unread && insky == in,
          "observable counts %llu + %llu vs %lld", (unsigned long long)in,
          (unsigned long long)outside, (long long)cnt.finished_unread);
    Records rr;
    read_all(ctx, rr, 1000);
    crp_destroy(ctx);
    std::printf("tune/eval/observe ok: launch %d/%d/%d/%d\n", l1.block, l1.blocks_per_cu,
                l1.refill, l1.layout);
}

// FP64 grid: the corner-record layout (192-byte records, built on first use,
// freed and rebuilt when the grid is set again) gives the records of the
// linear layout; the tuner tries both layouts on it.  The reference run queues
// the batch in the caller's order, the others longest expected path first.
void section_fp64_corner(const Grid& g, const Tables& t)
{
    crp_config c = base_config(CRP_FP64);
    const Inj j = make_injection(300, 21, g.n * g.spacing, 10 * MPC);
    c.inject_order = CRP_ORDER_AS_GIVEN;
    crp_ctx* a = make_ctx(c, g, t, false);
    c.inject_order = CRP_ORDER_LONGEST_FIRST;
    OK(inject(a, j));
    run_to_end(a, 0, nullptr);
    Records ra;
    read_all(a, ra, 128);
    crp_destroy(a);
    crp_ctx* b = make_ctx(c, g, t, false);
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1)     // a new grid drops the records; the next run rebuilds them
            OK(crp_set_field_grid(b, g.d.data(), CRP_F64, 0, g.n, g.n, g.n, g.spacing, nullptr));
        crp_launch l{256, 0, 4, CRP_LAYOUT_CORNER};
        OK(crp_set_launch(b, &l));
        OK(inject(b, j));
        run_to_end(b, 0, nullptr);
        Records rb;
        read_all(b, rb, 128);
        same_records(ra, rb, "FP64 corner records");
    }
    OK(inject(b, j));
    crp_launch best;
    double rate = 0;
    OK(crp_tune(b, 16, nullptr, &best, &rate));
    CHECK(rate > 0, "tune on the FP64 grid");
    run_to_end(b, 0, nullptr);
    double rs = 0;
    CHECK(crp_gather_ceiling(b, 10, &rs) == CRP_EINVAL, "gather diagnostic on an FP64 grid");
    crp_destroy(b);
    std::printf("fp64 corner ok: %zu records, tuned %d/%d/%d/%d\n", ra.size(), best.block,
                best.blocks_per_cu, best.refill, best.layout);
}

void section_patches(const Grid& g, const Tables& t)
{
    crp_config c = base_config(CRP_MIX);
    crp_ctx* ctx = make_ctx(c, g, t, true);
    const int pn = 9;
    Rng r(11);
    std::vector<float> pd((size_t)pn * pn * pn * 3);
    for (auto& v : pd)
        v = (float)((2.0 * r.u() - 1.0) * 1e-13);
    crp_grid_patch p;
    std::memset(&p, 0, sizeof p);
    p.data = pd.data();
    for (int a = 0; a < 3; ++a) {
        p.n[a] = pn;
        p.offset[a] = 4;
    }
    p.refine = 2;
    p.on_device = 0;
    OK(crp_set_field_patches(ctx, 1, &p));
    crp_grid_patch q = p;
    q.offset[0] = g.n;        // sticks out of the base period
    CHECK(crp_set_field_patches(ctx, 1, &q) == CRP_EINVAL, "patch outside the period accepted");
    OK(crp_set_field_patches(ctx, 1, &p));
    const Inj j = make_injection(200, 13, g.n * g.spacing, 5 * MPC);
    OK(inject(ctx, j));
    for (int layout : {CRP_LAYOUT_LINEAR, CRP_LAYOUT_CORNER}) {
        crp_launch l{128, 0, 4, layout};
        OK(crp_set_launch(ctx, &l));
        if (layout == CRP_LAYOUT_CORNER)
            OK(inject(ctx, make_injection(200, 14, g.n * g.spacing, 5 * MPC)));
        run_to_end(ctx, 0, nullptr);
    }
    Records rr;
    read_all(ctx, rr, 64);
    crp_counters cnt;
    OK(crp_counts(ctx, &cnt));
    CHECK((int64_t)rr.size() == cnt.finished, "patch run records");
    crp_destroy(ctx);
    std::printf("patches ok: %zu records\n", rr.size());
}

void section_neural(const Grid& g, const Tables& t)
{
    crp_config c = base_config(CRP_MIX);
    c.field_mode = CRP_FIELD_NEURAL;
    crp_ctx* ctx = make_ctx(c, g, t, true);
    std::vector<int32_t> F(64 * 3);
    Rng r(17);
    for (auto& f : F)
        f = (int32_t)(r.u() * 9.0) - 4;
    std::vector<float> prm(CRP_NF_NPARAM);
    for (auto& p : prm)
        p = (float)((2.0 * r.u() - 1.0) * 0.08);
    OK(crp_nf_init(ctx, F.data(), prm.data(), 1e-13));
    std::vector<float> back(CRP_NF_NPARAM);
    OK(crp_nf_get_params(ctx, back.data()));
    CHECK(back == prm, "parameters read back differ");
    const int64_t n = 777;
    std::vector<double> pos(3 * n);
    for (auto& p : pos)
        p = r.u() * g.n * g.spacing;
    std::vector<float> tgt(3 * n), out(3 * n), grad(CRP_NF_NPARAM);
    for (auto& v : tgt)
        v = (float)(2.0 * r.u() - 1.0);
    double loss = 0;
    OK(crp_nf_loss_grad(ctx, n, pos.data(), tgt.data(), out.data(), grad.data(), &loss));
    CHECK(std::isfinite(loss) && loss > 0, "loss %g", loss);
    for (float v : grad)
        CHECK(std::isfinite(v), "non-finite gradient");
    OK(crp_nf_adam_step(ctx, grad.data(), 1e-3));
    grad[5] = NAN;
    CHECK(crp_nf_adam_step(ctx, grad.data(), 1e-3) == CRP_EINVAL, "NaN gradient accepted");
    std::vector<float> losses(20);
    OK(crp_nf_train(ctx, 20, 4096 + 37, 3e-3, 1e-5, 506, losses.data()));
    for (float v : losses)
        CHECK(std::isfinite(v), "training loss");
    std::vector<double> B(3 * n);
    OK(crp_eval_field(ctx, n, pos.data(), B.data(), CRP_FIELD_NEURAL + 16, 0));
    const Inj j = make_injection(130, 19, g.n * g.spacing, 2 * MPC);
    OK(inject(ctx, j));
    run_to_end(ctx, 0, nullptr);
    Records rr;
    read_all(ctx, rr, 1000);
    CHECK((int64_t)rr.size() >= j.n(), "neural run records");
    crp_destroy(ctx);
    std::printf("neural ok: loss %.4g -> %.4g\n", losses.front(), losses.back());
}

void section_galactic(const Tables& t)
{
    crp_config c = base_config(CRP_FP64);
    c.field_mode = CRP_FIELD_ANALYTIC;
    c.charge_sign = -1;
    c.boundary_radius = 20 * KPC;
    c.hmin = 1e-3 * KPC;
    c.hmax = 0.5 * KPC;
    c.e_floor = 0;
    crp_ctx* ctx = nullptr;
    OK(crp_create(&c, nullptr, &ctx));
    crp_analytic_field f{{-8.5 * KPC, 0, 0}, 2e-10, 5 * KPC, 1 * KPC, 1e-10, 10 * KPC, 2 * KPC,
                         5e-11, 3 * KPC, 1.5 * KPC};
    OK(crp_set_field_analytic(ctx, &f));
    std::vector<double> zero(t.e.size(), 0.0);
    OK(crp_set_tables(ctx, (int32_t)t.e.size(), t.e.data(), zero.data(), zero.data(),
                      zero.data()));
    Inj j = make_injection(600, 23, 0.0, 100 * KPC);
    for (auto& p : j.pos)
        p = 0.0;
    for (auto& e : j.E)
        e *= 10.0;
    OK(inject(ctx, j));
    run_to_end(ctx, 0, nullptr);
    const double re[4] = {1e17, 1e18, 1e19, 1e22};
    crp_lens_spec ls{3, 4, re, 1 << CRP_BOUNDARY, 0};
    int64_t nnz = 0;
    OK(crp_lens_build(ctx, &ls, &nnz, nullptr));
    const int64_t np = 6 * 16, rows = 3 * np;
    std::vector<int64_t> rowptr(rows + 1);
    std::vector<int32_t> col(nnz);
    std::vector<double> val(nnz);
    std::vector<uint64_t> cnt(nnz);
    OK(crp_lens_read(ctx, rowptr.data(), col.data(), val.data(), cnt.data()));
    CHECK(rowptr[0] == 0 && rowptr[rows] == nnz, "lens row pointers");
    for (int64_t i = 0; i < rows; ++i) {
        double s = 0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += val[k];
        CHECK(rowptr[i + 1] == rowptr[i] || std::fabs(s - 1.0) < 1e-12, "row %lld sums to %g",
              (long long)i, s);
    }
    std::vector<double> x(2 * rows, 1.0), y(2 * rows);
    OK(crp_lens_apply(ctx, 2, x.data(), y.data(), 0, nullptr));
    for (int64_t i = 0; i < rows; ++i)
        CHECK(y[i] == y[rows + i] && (rowptr[i + 1] == rowptr[i] ? y[i] == 0.0
                                                                   : std::fabs(y[i] - 1.0) < 1e-12),
              "lens applied to ones, row %lld: %g", (long long)i, y[i]);
    Records rr;
    read_all(ctx, rr, 250);
    crp_destroy(ctx);
    std::printf("galactic/lens ok: %zu records, %lld entries\n", rr.size(), (long long)nnz);
}

}  // namespace

int main()
{
    const Grid g = make_grid(3);
    const Tables t = make_tables();
    section_errors(g, t);
    section_propagate_restore(g, t, CRP_FP64);
    section_propagate_restore(g, t, CRP_MIX);
    section_tune_eval_observe(g, t);
    section_fp64_corner(g, t);
    section_patches(g, t);
    section_neural(g, t);
    section_galactic(t);
    std::printf("runtime driver ok\n");
    return 0;
}
