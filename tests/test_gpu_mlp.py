"""GPU checks of the warm-start network's kernels (bfloat16 MFMA GEMMs, bias,
ReLU, MSE, Adam) against the FP64 reference in oracle/mlp_ref.py, which
rounds to bfloat16 at the same points.  Tolerances: a bfloat16 rounding
(relative 2^-9) can fall on the other side for an activation whose float32
and float64 values straddle a rounding boundary, which moves individual
outputs and gradients by up to ~2^-8 relative; compared relative to the
largest entry of each block, 2e-2 leaves headroom, and the cosine between the
full gradients must exceed 0.9999."""
import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu


def _net(dims, batch, seed):
    from paper_2110_11738_amd import drot
    return drot.MLP(*dims, max_batch=batch, seed=seed)


def _blocks(dims):
    i, h, o = dims
    sizes = [h * i, h, h * h, h, o * h, o]
    return np.cumsum([0] + sizes)


@pytest.mark.parametrize("dims,batch", [((64, 128, 64), 64), ((256, 64, 128), 128),
                                        ((2048, 512, 2048), 64)])
def test_forward_and_gradients_match_reference(dims, batch):
    import torch
    rng = np.random.default_rng([21, dims[0], batch])
    net = _net(dims, batch, seed=3)
    theta = net.get_weights().astype(np.float64)
    x = rng.standard_normal((batch, dims[0])).astype(np.float32)
    t = rng.standard_normal((batch, dims[2])).astype(np.float32)
    xd = torch.tensor(x, device="cuda")
    td = torch.tensor(t, device="cuda")
    y = net.forward(xd).cpu().numpy().astype(np.float64)
    y_ref = mlp_ref.forward(theta, x, dims)
    ey = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    loss, g = net.gradients(xd, td)
    loss_ref, g_ref = mlp_ref.loss_and_grad(theta, x, t, dims)
    g = g.cpu().numpy().astype(np.float64)
    cos = float(g @ g_ref / np.linalg.norm(g) / np.linalg.norm(g_ref))
    print(f"[mlp] {dims} batch {batch}: forward {ey:.2e} loss {loss:.6e} vs {loss_ref:.6e} "
          f"cos {cos:.8f}", flush=True)
    assert ey <= 2e-2
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    assert cos >= 0.9999
    b = _blocks(dims)
    for k in range(6):
        gk, rk = g[b[k]:b[k + 1]], g_ref[b[k]:b[k + 1]]
        assert np.abs(gk - rk).max() <= 2e-2 * np.abs(rk).max() + 1e-12, k
    net.close()


def test_adam_training_fits_a_teacher():
    """Fit the outputs of a fixed random teacher network: Adam on the GPU
    kernels drives the training loss down by more than an order of magnitude."""
    import torch
    dims = (128, 128, 64)
    rng = np.random.default_rng(22)
    teacher = _net(dims, 256, seed=11)
    x = torch.tensor(rng.standard_normal((256, 128)).astype(np.float32), device="cuda")
    t = teacher.forward(x)
    student = _net(dims, 256, seed=12)
    first = student.train_step(x, t, lr=3e-3)
    for _ in range(300):
        last = student.train_step(x, t, lr=3e-3)
    print(f"[mlp] teacher fit: loss {first:.4e} -> {last:.4e}", flush=True)
    assert last < 0.05 * first
    teacher.close()
    student.close()


def test_rejects_bad_shapes():
    import torch
    from paper_2110_11738_amd import drot
    with pytest.raises(drot.DrotError):
        drot.MLP(100, 64, 64, max_batch=64)
    net = _net((64, 64, 64), 64, seed=0)
    with pytest.raises(drot.DrotError):
        net.forward(torch.zeros((32, 64), device="cuda"))
    net.close()
