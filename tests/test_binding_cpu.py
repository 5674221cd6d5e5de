"""Host-side argument checks of the binding: the library reads exactly the sizes
it is given, so arrays whose shape, type or memory kind does not match are
rejected in Python before any pointer reaches it.  No GPU is needed: every case
here raises before the library is called."""
import numpy as np
import pytest
import torch

from paper_1307_2643_amd import crp


@pytest.fixture
def ctx():
    c = crp.Context.__new__(crp.Context)      # no library context: nothing may reach it
    c.params = crp.Params()
    c.L = None
    c.h = None
    return c


def _inj(n=5):
    return dict(id=np.arange(n, dtype=np.uint32), A=np.ones(n, np.int32), Z=np.ones(n, np.int32),
                E=np.full(n, 1e19), pos=np.zeros((n, 3)), dir=np.tile([1.0, 0, 0], (n, 1)),
                lmax=np.ones(n))


@pytest.mark.parametrize("field,bad", [("pos", np.zeros((4, 3))), ("dir", np.zeros((5, 2))),
                                       ("E", np.ones(6)), ("lmax", np.ones((5, 1))),
                                       ("A", np.ones(4, np.int32))])
def test_inject_rejects_mismatched_host_arrays(ctx, field, bad):
    a = _inj()
    a[field] = bad
    with pytest.raises(ValueError, match=field):
        ctx.inject(**a)


def test_inject_on_device_needs_gpu_tensors(ctx):
    with pytest.raises(ValueError, match="GPU"):
        ctx.inject(**_inj(), on_device=True)                  # host arrays
    t = {k: torch.as_tensor(v) for k, v in _inj().items()}
    t["id"] = t["id"].to(torch.int32)
    with pytest.raises(ValueError, match="GPU"):
        ctx.inject(**t, on_device=True)                       # CPU tensors
    with pytest.raises(ValueError, match="host"):
        ctx.inject(**t)                                       # tensors where host arrays go


def test_tables_grid_and_network_shapes(ctx):
    class T:
        e_nodes = np.geomspace(1e16, 1e23, 200)
        t_pi = np.zeros(200)
        t_n = np.zeros(199)
        beta_p = np.zeros(200)
    with pytest.raises(ValueError, match="tables"):
        ctx.set_tables(T)
    with pytest.raises(ValueError, match="grid"):
        ctx.set_field_grid(np.zeros((4, 4, 4, 2), np.float32), 1.0)
    with pytest.raises(ValueError, match="grid"):
        ctx.set_field_grid(np.zeros((4, 4, 4)), 1.0)
    with pytest.raises(ValueError, match="patch 0"):
        ctx.set_field_patches([dict(data=np.zeros((4, 4, 4)), offset=(0, 0, 0), refine=2)])
    with pytest.raises(ValueError, match="freq"):
        ctx.nf_init(np.zeros((63, 3)), np.zeros(crp.NF_NPARAM), 1.0)
    with pytest.raises(ValueError, match="params"):
        ctx.nf_init(np.zeros((64, 3)), np.zeros(crp.NF_NPARAM - 1), 1.0)
    with pytest.raises(ValueError, match="target"):
        ctx.nf_loss_grad(np.zeros((10, 3)), np.zeros((9, 3)))


def test_lens_maps_must_match_the_lens(ctx):
    ctx._lens_shape = (2, 24, 100)
    with pytest.raises(ValueError, match="x"):
        ctx.lens_apply(np.zeros((1, 3, 24)))
    with pytest.raises(ValueError, match="x"):
        ctx.lens_apply(np.zeros((2, 24)))
    with pytest.raises(ValueError, match="GPU"):
        crp._dev(np.zeros((1, 2, 24)), np.float64, (None, 2, 24), "x", 0)
    with pytest.raises(ValueError, match="GPU"):
        crp._dev(torch.zeros((1, 2, 24), dtype=torch.float64), np.float64, (None, 2, 24), "x", 0)
