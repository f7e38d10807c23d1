"""GPU parity of the learned-guess network (BF16 matrix-core convolutions, FP32 head, FP32 master
weights, Adam) against the FP64 reference network.  BF16 operands carry 8 significant bits, so
outputs and gradients are compared by relative norm (<= 2e-2) and cosine (>= 0.999)."""
import numpy as np
import pytest

from oracle import cnn
from gpu_util import cpu, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def problem(k=40, B=6, seed=0):
    from synth.blobs import draw_seed, jitter_target, render, rng_for
    rng = np.random.default_rng(seed)
    theta = cnn.init_params(k, rng)
    # nonzero biases so that every bias path is exercised
    sizes = [int(np.prod(s)) for s in cnn.shapes(k)]
    offs = np.cumsum([0] + sizes)
    for t in (1, 3, 5, 7):
        theta[offs[t]:offs[t + 1]] = 0.1 * rng.standard_normal(sizes[t])
    r = rng_for(77, 64)
    sb = draw_seed(r, 64, 64, 8)
    imgs = np.stack([render(jitter_target(r, sb, 2.0, (0.9, 1.1)), 64, 64)[0].reshape(-1)
                     for _ in range(B)])
    steps = rng.integers(1, 101, B).astype(np.int32)
    target = rng.standard_normal((B, k))
    return k, theta, imgs, steps, target


def close(a, b):
    a, b = np.ravel(a), np.ravel(b)
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
    return rel, cos


def to_dev(X, imgs, steps):
    import torch
    return (torch.tensor(imgs, dtype=torch.float64, device=dev()),
            torch.tensor(steps, dtype=torch.int32, device=dev()))


def test_forward_matches_reference(X):
    import torch
    k, theta, imgs, steps, _ = problem()
    ctx = X.Context(4096, 40, 1)
    net = X.Net(ctx, k, len(imgs), theta)
    # images stored in reverse order, addressed through image_idx
    im, st = to_dev(X, imgs[::-1].copy(), steps)
    idx = torch.tensor(np.arange(len(imgs))[::-1].copy(), dtype=torch.int32, device=dev())
    alpha = torch.empty((len(imgs), k), dtype=torch.float32, device=dev())
    net.forward(im, st, alpha, image_idx=idx)
    torch.cuda.synchronize()
    ref = cnn.forward(theta, k, imgs, steps)
    rel, cos = close(cpu(alpha), ref)
    print(f"\nforward: rel {rel:.2e}, cos {cos:.6f}")
    assert rel <= 2e-2 and cos >= 0.999


def test_gradient_matches_reference(X):
    import torch
    k, theta, imgs, steps, target = problem(seed=1)
    ctx = X.Context(4096, 40, 1)
    net = X.Net(ctx, k, len(imgs), theta)
    im, st = to_dev(X, imgs, steps)
    # rows in shuffled order, scaled by 1/4: the kernel reads row perm[b] times 4
    perm = np.array([3, 0, 5, 1, 4, 2], dtype=np.int32)
    stored = np.empty_like(target)
    stored[perm] = target / 4.0
    tg = torch.tensor(stored, dtype=torch.float64, device=dev())
    ti = torch.tensor(perm, dtype=torch.int32, device=dev())
    alpha = torch.empty((len(imgs), k), dtype=torch.float32, device=dev())
    net.backward(im, st, tg, alpha, target_idx=ti, target_scale=4.0)
    torch.cuda.synchronize()
    L, g = cnn.loss_and_grad(theta, k, imgs, steps, target)
    gl = cpu(net.grad)
    assert abs(float(cpu(net.loss)[0]) - L) <= 2e-2 * L
    sizes = [int(np.prod(s)) for s in cnn.shapes(k)]
    offs = np.cumsum([0] + sizes)
    names = ["conv1.W", "conv1.b", "conv2.W", "conv2.b", "conv3.W", "conv3.b", "lin.W", "lin.b"]
    for t, name in enumerate(names):
        rel, cos = close(gl[offs[t]:offs[t + 1]], g[offs[t]:offs[t + 1]])
        print(f"\n{name}: rel {rel:.2e}, cos {cos:.6f}")
        assert rel <= 2e-2 and cos >= 0.999, name


def test_adam_step_matches_formula(X):
    import torch
    k = 8
    ctx = X.Context(1024, 8, 1)
    rng = np.random.default_rng(5)
    net = X.Net(ctx, k, 1, rng.standard_normal(X.load().xkp_cnn_param_count(k)))
    p0 = cpu(net.params).astype(np.float64)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    for t in range(1, 4):
        g = rng.standard_normal(p0.size).astype(np.float32)
        net.grad.copy_(torch.from_numpy(g))
        net.adam(1e-2)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g.astype(np.float64) ** 2
        p0 -= 1e-2 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    torch.cuda.synchronize()
    assert np.abs(cpu(net.params) - p0).max() <= 1e-5 * max(1.0, np.abs(p0).max())


def test_training_lowers_the_loss(X):
    """Fifty Adam steps on a fixed batch drive the regression loss well down."""
    import torch
    k, theta, imgs, steps, _ = problem(B=16, seed=2)
    target = 0.5 * np.tanh(cnn.forward(cnn.init_params(k, np.random.default_rng(9)), k, imgs, steps))
    ctx = X.Context(4096, 40, 1)
    net = X.Net(ctx, k, len(imgs), theta)
    im, st = to_dev(X, imgs, steps)
    tg = torch.tensor(target, dtype=torch.float64, device=dev())
    alpha = torch.empty((len(imgs), k), dtype=torch.float32, device=dev())
    losses = []
    for _ in range(50):
        net.backward(im, st, tg, alpha)
        net.adam(3e-3)
        losses.append(float(cpu(net.loss)[0]))
    print(f"\nloss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.2 * losses[0]
