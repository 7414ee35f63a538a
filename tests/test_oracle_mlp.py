"""Pins of the FP64 pruning-network reference: central finite differences,
and PyTorch's CPU autograd, BCE-with-logits and Adam as independent library
routines (all in float64 on the CPU)."""
import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")


def _data(seed=0, R=64):
    rng = np.random.default_rng(seed)
    theta = mlp.init_params(rng)
    theta[mlp.N_PARAMS - 1] = 0.3                       # non-zero output bias
    F = rng.standard_normal((R, 16))
    y = (rng.random(R) < 0.3).astype(np.float64)
    return theta, F, y


def test_param_count():
    assert mlp.N_PARAMS == 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1 == 5313


def test_gradient_central_differences():
    theta, F, y = _data()
    w = 3.7
    loss, g = mlp.loss_and_grad(theta, F, y, w)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [mlp.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.bce(mlp.forward(tp, F)[0], y, w) - mlp.bce(mlp.forward(tm, F)[0], y, w)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(g[i]), (i, fd, g[i])


def _torch_net(theta):
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in mlp.unpack(theta).items()}

    def fwd(F):
        h1 = torch.relu(F @ p["W1"].T + p["b1"])
        h2 = torch.relu(h1 @ p["W2"].T + p["b2"])
        return h2 @ p["w3"] + p["b3"][0]
    return p, fwd


def test_loss_and_gradient_match_autograd():
    theta, F, y = _data(seed=2, R=200)
    w = 5.0
    loss, g = mlp.loss_and_grad(theta, F, y, w)
    p, fwd = _torch_net(theta)
    z = fwd(torch.tensor(F))
    tl = torch.nn.functional.binary_cross_entropy_with_logits(
        z, torch.tensor(y), pos_weight=torch.tensor(w, dtype=torch.float64))
    tl.backward()
    assert abs(tl.item() - loss) < 1e-12 * max(1.0, abs(loss))
    tg = np.concatenate([p[name].grad.numpy().ravel() for name, _ in mlp.SHAPES])
    assert np.allclose(g, tg, rtol=1e-10, atol=1e-14)


def test_adam_matches_torch():
    theta, F, y = _data(seed=3)
    w = 2.0
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    p, fwd = _torch_net(theta)
    params = [p[name] for name, _ in mlp.SHAPES]
    opt = torch.optim.Adam(params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th = theta.copy()
    for t in range(1, 4):
        _, g = mlp.loss_and_grad(th, F, y, w)
        th, m, v = mlp.adam_step(th, m, v, g, t)
        opt.zero_grad()
        z = fwd(torch.tensor(F))
        torch.nn.functional.binary_cross_entropy_with_logits(
            z, torch.tensor(y), pos_weight=torch.tensor(w, dtype=torch.float64)).backward()
        opt.step()
    tt = np.concatenate([q.detach().numpy().ravel() for q in params])
    assert np.allclose(th, tt, rtol=1e-9, atol=1e-12)


def test_features_layout():
    traj = np.array([[[1.0, 1e-3], [2.0, 0.0], [3.0, 1.0], [4.0, 1e-20],
                      [5.0, 10.0], [6.0, 1e-6], [7.0, 0.5], [8.0, 1e-12]]])
    f = mlp.features(traj, np.zeros(16), np.ones(16))[0]
    assert list(f[0::2]) == [1, 2, 3, 4, 5, 6, 7, 8]
    assert np.allclose(f[1::2], [-3, -12, 0, -12, 1, -6, np.log10(0.5), -12])
    g = mlp.features(traj, np.full(16, 1.0), np.full(16, 2.0))[0]
    assert np.allclose(g, (f - 1.0) / 2.0)
