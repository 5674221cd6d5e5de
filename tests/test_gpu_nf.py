"""Neural field on the GPU (bf16 MFMA kernels through the C-ABI) against the
numpy oracle with the same bfloat16 rounding points, and training on the GPU.

Bars: the training forward and gradients within 1e-3 relative L2 per tensor
of the oracle's bf16-rounded FP64 evaluation (the GPU accumulates in FP32;
an activation whose FP32 and FP64 values straddle a bf16 rounding boundary
takes the neighbouring bf16 value); the Adam update within FP32 rounding of
the oracle's; the stepper through the network field against the oracle's
stepping through the oracle's network, within a bound derived from the
measured field difference of the two network evaluations."""
import sys

import numpy as np
import pytest

import crp_inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1307_2643_amd import crp
    crp.load()
    return crp


@pytest.fixture(scope="module")
def N():
    from oracle import nf_oracle
    return nf_oracle


def init_params(seed=509, scale=1.0):
    ws, bs = I.nf_init_weights(seed)
    rng = np.random.default_rng(seed + 1)
    bs = [rng.standard_normal(b.shape).astype(np.float32) * 0.05 for b in bs]
    ws = [w * scale for w in ws]
    from oracle import nf_oracle
    return nf_oracle.flatten(ws, bs).astype(np.float32)


def make_ctx(P, grid, spacing, **kw):
    prm = P.Params(precision=P.MIX, queue_capacity=1 << 14, neutral_capacity=1 << 14, **kw)
    ctx = P.Context(prm)
    ctx.set_field_grid(grid, spacing)
    ctx.set_tables(I.tables_loss_only())
    return ctx


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [3000, 37, 20011])
def test_nf_loss_and_gradients_match_oracle(P, N, n):
    """3000: several waves and a ragged tail; 37: one partial wave; 20011: 63
    chunks of the split weight-gradient sum, each over an odd and an even half."""
    w = I.W_SMALL
    grid = w.make_grid().astype(np.float32)
    ctx = make_ctx(P, grid, w.spacing_m)
    F = I.nf_frequencies()
    params = init_params()
    ctx.nf_init(F, params, I.NG_T)
    rng = np.random.default_rng(3)
    box = 32 * w.spacing_m
    pos = (rng.random((n, 3)) * 3 - 1) * box   # several periods, both signs
    target = rng.standard_normal((n, 3)).astype(np.float32)
    say(f"nf loss/grad, {n} points")
    out, grad, loss = ctx.nf_loss_grad(pos, target)
    xh = N.normalized_position(pos, (32, 32, 32), w.spacing_m).astype(np.float32)
    ws, bs = N.unflatten(params)
    ref_out, cache = N.forward(ws, bs, xh.astype(np.float64), F, bf16=True)
    ref_loss = N.mse_loss(ref_out, target)
    gW, gb = N.backward(ws, cache, N.mse_grad(ref_out, target))
    ref_grad = N.flatten(gW, gb)
    e_out = rel_l2(out, ref_out)
    say(f"out rel-L2 {e_out:.2e}, loss {loss:.6f} vs {ref_loss:.6f}")
    assert e_out < 1e-3
    assert abs(loss / ref_loss - 1) < 1e-3
    off = 0
    worst = 0.0
    for k, (W, b) in enumerate(zip(gW, gb)):
        eW = rel_l2(grad[off:off + W.size], W.ravel())
        off += W.size
        eb = rel_l2(grad[off:off + b.size], b)
        off += b.size
        say(f"layer {k + 1}: dW rel-L2 {eW:.2e}, db rel-L2 {eb:.2e}")
        worst = max(worst, eW, eb)
    assert worst < 1e-3, worst
    assert off == P.NF_NPARAM
    assert np.array_equal(ctx.nf_get_params(), params)
    ctx.close()


def test_nf_eval_field_matches_oracle(P, N):
    """The stepper's network evaluation (FP32 phases, hardware sin / cos of
    revolutions) against the oracle's: a feature moved by ~1e-5 takes the
    neighbouring bf16 value where it lies that close to a rounding boundary
    (about one feature in a hundred), each such change 2^-8 of that feature;
    relative L2 within 2e-3 (measured 7.7e-4)."""
    w = I.W_SMALL
    grid = w.make_grid().astype(np.float32)
    ctx = make_ctx(P, grid, w.spacing_m)
    F = I.nf_frequencies()
    params = init_params(seed=11)
    ctx.nf_init(F, params, I.NG_T)
    rng = np.random.default_rng(4)
    pos = rng.random((5000, 3)) * 32 * w.spacing_m
    say("nf eval")
    B = ctx.eval_field(pos, P.EVAL_NEURAL)
    xh = N.normalized_position(pos, (32, 32, 32), w.spacing_m).astype(np.float32)
    ws, bs = N.unflatten(params)
    ref, _ = N.forward(ws, bs, xh.astype(np.float64), F, bf16=True)
    e = rel_l2(B / I.NG_T, ref)
    say(f"eval rel-L2 {e:.2e}")
    assert e < 2e-3
    ctx.close()


def test_nf_training_reduces_field_error(P):
    """Training on the GPU (own forward/backward/Adam kernels) lowers the RMS
    error against the grid's trilinear field on held-out points."""
    w = I.W_SMALL
    grid = w.make_grid().astype(np.float32)
    ctx = make_ctx(P, grid, w.spacing_m)
    F = I.nf_frequencies(nmin=2, nmax=16)
    ctx.nf_init(F, init_params(), I.NG_T)
    rng = np.random.default_rng(5)
    pos = rng.random((20000, 3)) * 32 * w.spacing_m
    Bg = ctx.eval_field(pos, P.MIX)

    def rms():
        Bn = ctx.eval_field(pos, P.EVAL_NEURAL)
        return float(np.sqrt(((Bn - Bg) ** 2).sum(1).mean()) / I.NG_T)

    r0 = rms()
    say("nf training")
    losses = ctx.nf_train(300, 8192, 2e-3, 1e-4, 77)
    r1 = rms()
    say(f"RMS error {r0:.3f} -> {r1:.3f}; loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]
    assert r1 < 0.5 * r0
    ctx.close()


def test_nf_adam_matches_oracle(P, N):
    """Two Adam updates of the FP32 masters with given gradients (the library's
    Adam kernel, FP32 arithmetic) against the oracle's FP64 update of the same
    FP32 inputs: within FP32 rounding of the parameters plus 1e-5 of each
    update (m, v, their bias corrections, sqrt and quotient each rounded once
    in FP32, relative error a few 1e-7)."""
    w = I.W_SMALL
    grid = w.make_grid().astype(np.float32)
    ctx = make_ctx(P, grid, w.spacing_m)
    F = I.nf_frequencies()
    p0 = init_params()
    ctx.nf_init(F, p0, I.NG_T)
    rng = np.random.default_rng(8)
    lr = 1e-3
    grads = []
    for t in range(2):
        g = (rng.standard_normal(P.NF_NPARAM) * 10.0 ** rng.uniform(-9, -1, P.NF_NPARAM))
        g[:50] = 0.0                                   # zero gradients: m = v = 0
        grads.append(g.astype(np.float32))
        say(f"adam step {t + 1}")
        ctx.nf_adam_step(grads[-1], lr)
    got = ctx.nf_get_params().astype(np.float64)
    ps = [p0.astype(np.float64)]
    m = [np.zeros(P.NF_NPARAM)]
    v = [np.zeros(P.NF_NPARAM)]
    for t, g in enumerate(grads):
        N.adam_step(ps, [g.astype(np.float64)], m, v, t + 1, lr)
    ref = ps[0]
    tol = 2.0 ** -23 * np.abs(ref) + 2 * 1e-5 * lr
    err = np.abs(got - ref)
    say(f"adam: max |dp| / tol {np.max(err / tol):.3f}")
    assert np.all(err <= tol)
    assert np.array_equal(got[:50], p0[:50].astype(np.float64))
    # a non-finite gradient is refused and changes nothing
    bad = grads[0].copy()
    bad[7] = np.nan
    with pytest.raises(P.CrpError):
        ctx.nf_adam_step(bad, lr)
    assert np.array_equal(ctx.nf_get_params().astype(np.float64), got)
    ctx.close()


def test_nf_stepper_matches_oracle_stepping(P, N):
    """The surrogate stepper (network field per Cash-Karp stage, MFMA) against
    the oracle's precision-form stepping whose field is the oracle's network
    (bf16 rounding points as on the GPU, FP64 arithmetic), for 12 fixed steps
    (hmin = hmax: every attempt accepted, so no accept/reject decision can
    differ).  The two network evaluations differ by at most eps (measured on
    20000 points; the stepper's FP32 phases and hardware sin/cos move a few
    features to a neighbouring bf16 value); a step then changes the direction
    by at most h kappa eps more, so after K steps |du| <= K h kappa eps and
    |dx| <= K^2 h^2 kappa eps / 2, allowed 4x for the drift of the field
    along the slightly different paths, plus FP32 rounding of u."""
    from oracle import oracle as O
    w = I.W_SMALL
    grid = w.make_grid().astype(np.float32)
    h = 100 * I.KPC_M
    K = 12
    F = I.nf_frequencies()
    params = init_params(seed=21)
    prm = P.params_for(w, P.MIX, field_mode=P.FIELD_NEURAL, hmin=h, hmax=h,
                       queue_capacity=1 << 14, neutral_capacity=1 << 14)
    ctx = P.Context(prm)
    ctx.set_field_grid(grid, w.spacing_m)
    ctx.set_tables(w.make_tables())
    ctx.nf_init(F, params, I.NG_T)
    box = 32 * w.spacing_m
    ws, bs = N.unflatten(params)

    def xhat(p):
        f = (np.asarray(p, np.float64).reshape(-1, 3)) * (1.0 / box)
        return (f - np.floor(f)).astype(np.float32)

    def net_field(p):
        out, _ = N.forward(ws, bs, xhat(p).astype(np.float64), F, bf16=True)
        return float(np.float32(I.NG_T)) * out[0]

    # the two network evaluations on a sample of the box
    rng = np.random.default_rng(12)
    pts = rng.random((20000, 3)) * box
    Bg = ctx.eval_field(pts, P.EVAL_NEURAL)
    ref, _ = N.forward(ws, bs, xhat(pts).astype(np.float64), F, bf16=True)
    eps = float(np.max(np.linalg.norm(Bg - ref * float(np.float32(I.NG_T)), axis=1)))
    say(f"network field difference: max {eps / I.NG_T:.2e} B_rms")
    inj = w.make_injection(128)
    say("nf stepper, 12 fixed steps")
    ctx.inject(inj)
    assert not ctx.propagate(K)
    fg = ctx.read_finished()
    pend = ctx.peek_pending()
    ctx.close()
    fg = P.sort_finished({k: np.concatenate([fg[k], pend[k]]) for k in fg})
    cfg = O.config_for(w, precision=O.MIX, hmin=h, hmax=h, max_cycles=K)
    fo, _, co, _ = O.propagate(cfg, O.FieldRef(net_field), O.TablesRef(w.make_tables()), inj)
    fo = O.sort_finished(fo)
    for k in ("id", "lineage", "nsteps", "nrej", "status", "A", "Z", "m"):
        assert np.array_equal(fg[k], fo[k]), k
    assert np.all(fo["nsteps"] == K)
    kappa = 299792458.0 / inj.E[fo["id"]]
    du = np.linalg.norm(fg["u"] - fo["u"], axis=1)
    dx = np.linalg.norm(fg["x"] - fo["x"], axis=1)
    tol_u = 4 * K * h * kappa * eps + 1e-6
    tol_x = 4 * K * K * h * h * kappa * eps / 2 + K * h * 1e-6
    say(f"after {K} steps: max |du|/tol {np.max(du / tol_u):.3f}, max |dx|/tol "
        f"{np.max(dx / tol_x):.3f}, max |du| {du.max():.2e}")
    assert np.all(du <= tol_u) and np.all(dx <= tol_x)
    assert np.allclose(fg["E"], fo["E"], rtol=1e-6, atol=0)
    assert np.array_equal(fg["L"], fo["L"])
