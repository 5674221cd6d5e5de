"""Neural field on the GPU (bf16 MFMA kernels through the C-ABI) against the
numpy oracle with the same bfloat16 rounding points, and training on the GPU."""
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


def test_nf_loss_and_gradients_match_oracle(P, N):
    w = I.W_SMALL
    grid = w.make_grid().astype(np.float32)
    ctx = make_ctx(P, grid, w.spacing_m)
    F = I.nf_frequencies()
    params = init_params()
    ctx.nf_init(F, params, I.NG_T)
    n = 3000                                   # several waves and a ragged tail
    rng = np.random.default_rng(3)
    box = 32 * w.spacing_m
    pos = (rng.random((n, 3)) * 3 - 1) * box   # several periods, both signs
    target = rng.standard_normal((n, 3)).astype(np.float32)
    say("nf loss/grad")
    out, grad, loss = ctx.nf_loss_grad(pos, target)
    xh = N.normalized_position(pos, (32, 32, 32), w.spacing_m).astype(np.float32)
    ws, bs = N.unflatten(params)
    ref_out, cache = N.forward(ws, bs, xh.astype(np.float64), F, bf16=True)
    ref_loss = N.mse_loss(ref_out, target)
    gW, gb = N.backward(ws, cache, N.mse_grad(ref_out, target))
    ref_grad = N.flatten(gW, gb)
    e_out = rel_l2(out, ref_out)
    say(f"out rel-L2 {e_out:.2e}, loss {loss:.6f} vs {ref_loss:.6f}")
    assert e_out < 5e-3
    assert abs(loss / ref_loss - 1) < 5e-3
    off = 0
    for k, (W, b) in enumerate(zip(gW, gb)):
        eW = rel_l2(grad[off:off + W.size], W.ravel())
        off += W.size
        eb = rel_l2(grad[off:off + b.size], b)
        off += b.size
        say(f"layer {k + 1}: dW rel-L2 {eW:.2e}, db rel-L2 {eb:.2e}")
        assert eW < 2e-2 and eb < 2e-2
    assert off == P.NF_NPARAM
    assert np.array_equal(ctx.nf_get_params(), params)
    ctx.close()


def test_nf_eval_field_matches_oracle(P, N):
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
    assert e < 5e-3
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


def test_nf_propagation_runs_and_tracks_grid(P):
    """The surrogate stepper (MFMA field per Cash-Karp stage) propagates a batch;
    with an untrained network it still steps every candidate to its end."""
    w = I.W_SMALL
    grid = w.make_grid().astype(np.float32)
    ctx = make_ctx(P, grid, w.spacing_m, field_mode=P.FIELD_NEURAL)
    ctx.nf_init(I.nf_frequencies(), init_params(), I.NG_T)
    inj = w.make_injection(700)
    ctx.inject(inj)
    say("nf propagate")
    assert ctx.propagate()
    fin = ctx.read_finished()
    c = ctx.counts()
    say(f"nf propagation: {c['steps']} steps, {len(fin['id'])} finished")
    assert len(fin["id"]) == 700 and np.all(fin["status"] == P.MAX_TRAJ)
    assert np.all(np.isfinite(fin["x"])) and np.all(np.abs(np.linalg.norm(fin["u"], axis=1) - 1) < 1e-5)
    ctx.close()
