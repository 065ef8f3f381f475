"""GPU checks of the warm-start network's kernels (bfloat16 MFMA GEMMs, bias,
ReLU, MSE, Adam) against the FP64 reference in oracle/mlp_ref.py, which
rounds to bfloat16 at the same points.

Random data: a bfloat16 rounding (relative 2^-9) can fall on the other side
for an activation whose float32 and float64 values straddle a rounding
boundary, which moves individual outputs and gradients by up to ~2^-8
relative; compared relative to the largest entry of each block, 2e-2 leaves
headroom, and the cosine between the full gradients must exceed 0.9999.

Dyadic data (`_dyadic_case`): inputs, weights, biases and targets are small
multiples of powers of two, chosen so that every float32 sum the kernels
form is exact (at most 20 significant bits); the values entering each
bfloat16 rounding are then identical on both sides, and the forward pass,
the loss and the gradients must agree bit for bit.  Adam (Kingma and Ba,
Algorithm 1) is checked element by element: one train step on the dyadic
data, and ten steps on seeded gradients through drot_mlp_apply_gradients,
against oracle/mlp_ref.adam_step; the float32 update differs from the
float64 one by a few roundings of the update (relative ~1e-7) plus one
rounding of the stored weight per step."""
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


def _dyadic_case(seed=5, batch=64):
    """Dims (64, 64, 64): x in {0, 1} with four ones per row, W1 = +-1/2,
    b1 odd multiples of 1/4, W2 and W3 = +-1/8, b2 odd multiples of 2^-6,
    b3 odd multiples of 2^-10, targets t = y - s with s in {+-1/4, +-1/2,
    +-3/4} (y the reference output).  Products and sums then stay on a grid
    of 2^-22 with magnitudes below 2^20 of it, exact in float32."""
    dims = (64, 64, 64)
    rng = np.random.default_rng([23, seed])
    i, h, o = dims
    x = np.zeros((batch, i), dtype=np.float32)
    for r in range(batch):
        x[r, rng.choice(i, 4, replace=False)] = 1.0
    sign = lambda shape: rng.choice([-1.0, 1.0], size=shape)
    odd = lambda k, lim: rng.choice(np.arange(1, lim + 1, 2), size=k) * rng.choice([-1, 1], size=k)
    W1, b1 = 0.5 * sign((h, i)), odd(h, 3) / 4.0
    W2, b2 = 0.125 * sign((h, h)), odd(h, 7) / 64.0
    W3, b3 = 0.125 * sign((o, h)), odd(o, 7) / 1024.0
    theta = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    y = mlp_ref.forward(theta, x, dims)
    s = rng.choice([-0.75, -0.5, -0.25, 0.25, 0.5, 0.75], size=y.shape)
    t = y - s
    assert (t.astype(np.float32).astype(np.float64) == t).all()
    assert (theta.astype(np.float32).astype(np.float64) == theta).all()
    return dims, theta, x, t.astype(np.float32)


def test_dyadic_forward_gradients_bit_exact_and_one_adam_step():
    import torch
    dims, theta, x, t = _dyadic_case()
    net = _net(dims, 64, seed=0)
    net.set_weights(theta)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    y = net.forward(xd).cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(y, mlp_ref.forward(theta, x, dims))
    loss, g = net.gradients(xd, td)
    loss_ref, g_ref = mlp_ref.loss_and_grad(theta, x, t, dims)
    print(f"[mlp dyadic] loss {loss!r} vs {loss_ref!r}, nonzero grads {np.count_nonzero(g_ref)}",
          flush=True)
    assert loss == loss_ref
    np.testing.assert_array_equal(g.cpu().numpy().astype(np.float64), g_ref)
    lr = 1e-3
    net.train_step(xd, td, lr=lr)
    w1 = net.get_weights().astype(np.float64)
    w1_ref, _, _ = mlp_ref.adam_step(theta, g_ref, np.zeros_like(theta), np.zeros_like(theta), 1, lr)
    tol = np.spacing(np.abs(w1_ref).astype(np.float32)).astype(np.float64) + 1e-6 * lr
    err = np.abs(w1 - w1_ref)
    print(f"[mlp dyadic] one Adam step: max |w - w_ref| {err.max():.3e}", flush=True)
    assert (err <= tol).all()
    net.close()


def test_adam_ten_steps_on_given_gradients():
    """drot_mlp_apply_gradients against the float64 Adam on the same seeded
    gradient sequence (zeros, tiny and large entries included)."""
    import torch
    dims = (128, 64, 192)
    net = _net(dims, 64, seed=1)
    n = net.n_params
    rng = np.random.default_rng(24)
    w = (rng.standard_normal(n) * 0.3).astype(np.float32).astype(np.float64)
    net.set_weights(w)
    scale = 10.0 ** rng.uniform(-7, 1, size=n)
    grads = [(rng.standard_normal(n) * scale).astype(np.float32) for _ in range(10)]
    for g in grads:
        g[rng.choice(n, n // 50, replace=False)] = 0.0
    m1, m2 = np.zeros(n), np.zeros(n)
    lr = 1e-3
    for k, g in enumerate(grads, start=1):
        net.apply_gradients(torch.tensor(g, device="cuda"), lr)
        w, m1, m2 = mlp_ref.adam_step(w, g.astype(np.float64), m1, m2, k, lr)
        got = net.get_weights().astype(np.float64)
        tol = k * np.spacing(np.abs(w).astype(np.float32)).astype(np.float64) + 1e-6 * k * lr
        err = np.abs(got - w)
        if k in (1, 10):
            print(f"[adam] step {k}: max |w - w_ref| {err.max():.3e}, "
                  f"max err/tol {(err / tol).max():.3f}", flush=True)
        assert (err <= tol).all(), k
    with pytest.raises(Exception):
        net.apply_gradients(torch.zeros(n - 1, device="cuda"), lr)
    net.close()
