"""Learned pruner on the GPU, through the C ABI.

* Gradient, loss, prediction and one Adam step against the FP64 reference
  (oracle/mlp.py) on the same inputs.  The GPU forward pass uses the FP16 copy
  of the weights, so the reference runs on those FP16-rounded values (exact in
  FP64); the remaining difference is FP32 arithmetic:
  |g - g_ref| <= 1e-3 |g_ref| + 1e-4 max|g_ref|.
* Pruning inside the fixed point: threshold 0 prunes nothing (results equal
  the plain run bitwise); threshold 1 prunes every row still moving at pass 8,
  the guard then resumes them and the unique set equals the plain run's.
"""
import numpy as np
import pytest

from oracle import ica, mlp
from paper_2408_17118_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_17118_amd import oica
    c = oica.Context(0)
    yield c
    c.close()


def _traj(R, seed):
    rng = np.random.default_rng(seed)
    t = np.empty((R, 8, 2), np.float32)
    t[:, :, 0] = rng.normal(1.0, 2.0, (R, 8))
    t[:, :, 1] = 10.0 ** rng.uniform(-9, 0, (R, 8))
    y = (t[:, 7, 0] + rng.normal(0, 1, R) > 1.5).astype(np.uint8)
    return t, y


def _stats(t):
    f = np.empty((t.shape[0], 16))
    f[:, 0::2] = t[:, :, 0]
    f[:, 1::2] = np.log10(np.maximum(t[:, :, 1].astype(np.float64), 1e-12))
    return f.mean(axis=0), f.std(axis=0)


def _make(ctx, seed=0):
    from paper_2408_17118_amd import oica
    t, y = _traj(3000, seed)
    mean, std = _stats(t)
    w0 = mlp.init_params(np.random.default_rng(seed)).astype(np.float32)
    return oica.Pruner(ctx, w0, mean, std), t, y, w0, mean, std


def _ref_features(t, mean, std):
    # the GPU standardises with FP32 copies of the statistics
    return mlp.features(t.astype(np.float64), mean.astype(np.float32).astype(np.float64),
                        std.astype(np.float32).astype(np.float64))


def test_gradient_and_loss_match_reference(ctx):
    pr, t, y, w0, mean, std = _make(ctx)
    w16 = w0.astype(np.float16).astype(np.float64)
    w_pos = float((y == 0).sum() / max((y == 1).sum(), 1))
    g, loss = pr.grad(torch.from_numpy(t).cuda(), torch.from_numpy(y).cuda(), w_pos)
    lr, gr = mlp.loss_and_grad(w16, _ref_features(t, mean, std), y.astype(np.float64), w_pos)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss - lr) <= 1e-5 * abs(lr)
    assert np.all(np.abs(g - gr) <= 1e-3 * np.abs(gr) + 1e-4 * np.abs(gr).max()), \
        float(np.max(np.abs(g - gr)))


def test_predict_matches_reference(ctx):
    pr, t, y, w0, mean, std = _make(ctx, seed=1)
    p = pr.predict(torch.from_numpy(t).cuda()).cpu().numpy()
    z, _ = mlp.forward(w0.astype(np.float16).astype(np.float64), _ref_features(t, mean, std))
    assert np.allclose(p, mlp.sigmoid(z), atol=2e-5)


def test_adam_step_matches_reference(ctx):
    pr, t, y, w0, mean, std = _make(ctx, seed=2)
    w_pos = 2.0
    T, Y = torch.from_numpy(t).cuda(), torch.from_numpy(y).cuda()
    loss0 = pr.train_step(T, Y, w_pos, lr=1e-3)
    w1 = pr.weights().astype(np.float64)
    _, g = mlp.loss_and_grad(w0.astype(np.float16).astype(np.float64), _ref_features(t, mean, std),
                             y.astype(np.float64), w_pos)
    ref, _, _ = mlp.adam_step(w0.astype(np.float64), np.zeros_like(g), np.zeros_like(g), g, 1)
    # first Adam step moves every weight by ~lr sign(g); allow the FP32 gradient error
    assert np.all(np.abs(w1 - ref) <= 2e-5 + 1e-3 * np.abs(ref - w0))
    assert loss0 > 0


def test_training_reduces_loss(ctx):
    pr, t, y, w0, mean, std = _make(ctx, seed=3)
    T, Y = torch.from_numpy(t).cuda(), torch.from_numpy(y).cuda()
    w_pos = float((y == 0).sum() / max((y == 1).sum(), 1))
    first = pr.train_step(T, Y, w_pos, lr=3e-3)
    for _ in range(300):
        last = pr.train_step(T, Y, w_pos, lr=3e-3)
    assert last < 0.6 * first, (first, last)
    p = pr.predict(T).cpu().numpy()
    acc = ((p > 0.5) == (y == 1)).mean()
    assert acc > 0.85


def test_train_run_one_batch_equals_train_step(ctx):
    """A one-epoch run with one batch of all rows is one Adam step on the whole
    set, whatever the order: the loss (FP64 row sums) agrees to rounding, a
    dropped or repeated row would move it by about 1/R, and the weights agree
    except where a gradient component is at rounding level."""
    from paper_2408_17118_amd import oica
    pa, t, y, w0, mean, std = _make(ctx, seed=6)
    pb = oica.Pruner(ctx, w0, mean, std)
    T, Y = torch.from_numpy(t).cuda(), torch.from_numpy(y).cuda()
    R = t.shape[0]
    w_pos = float((y == 0).sum() / max((y == 1).sum(), 1))
    la = pa.train(T, Y, epochs=1, batch=R, lr=1e-3, seed=11, w_pos=w_pos)
    lb = pb.train_step(T, Y, w_pos, lr=1e-3)
    assert len(la) == 1 and abs(la[0] - lb) <= 1e-12 * abs(lb), (la, lb)
    d = np.abs(pa.weights().astype(np.float64) - pb.weights())
    assert np.mean(d <= 1e-6) >= 0.99 and d.max() <= 2.5e-3


def test_train_run_weights_and_order(ctx):
    """w_pos 0 is n_neg / n_pos of the labels; a seed fixes the weights; another
    seed (several steps per epoch) gives other weights; many epochs of small
    steps fit the training rows."""
    from paper_2408_17118_amd import oica
    _, t, y, w0, mean, std = _make(ctx, seed=7)
    T, Y = torch.from_numpy(t).cuda(), torch.from_numpy(y).cuda()
    w_pos = float(np.float32((y == 0).sum() / max((y == 1).sum(), 1)))

    def run(seed, wp, epochs=2):
        pr = oica.Pruner(ctx, w0, mean, std)
        return pr, pr.train(T, Y, epochs=epochs, batch=700, lr=3e-3, seed=seed, w_pos=wp)

    a, la = run(5, 0.0)
    b, lb = run(5, w_pos)
    c, _ = run(6, 0.0)
    assert np.array_equal(a.weights(), b.weights()) and la == lb
    assert not np.array_equal(a.weights(), c.weights())
    d, ld = run(5, 0.0, epochs=60)
    assert ld[:2] == la and ld[-1] < 0.6 * ld[0], ld
    acc = ((d.predict(T).cpu().numpy() > 0.5) == (y == 1)).mean()
    assert acc > 0.85
    with pytest.raises(oica.OicaError):
        d.train(T, Y, epochs=0)
    with pytest.raises(oica.OicaError):
        d.train(T, Y, batch=0)
    with pytest.raises(oica.OicaError):
        d.train(T, torch.ones_like(Y))          # every label positive and w_pos 0


def _same_unique_sets(ctx, a, b, T):
    """Full unique sets of two runs: the same counts, every cluster matched one
    to one at |cos| >= 1 - 1e-6, the same order up to near-equal criterion
    values."""
    ua = ctx.unique(a["W"], a["kurt"], a["status"], T)
    ub = ctx.unique(b["W"], b["kurt"], b["status"], T)
    assert ua["n_unique"] == ub["n_unique"] and ua["n_accepted"] == ub["n_accepted"]
    n = ua["n_unique"]
    cos = np.abs(ua["U"].cpu().numpy()[:n] @ ub["U"].cpu().numpy()[:n].T)
    assert np.all(cos.max(axis=1) >= 1 - 1e-6)
    j = cos.argmax(axis=1)
    assert len(set(j.tolist())) == n
    ups = ua["upsilon"].cpu().numpy()[:n]
    for k in range(n):
        if j[k] != k:
            assert abs(ups[j[k]] - ups[k]) <= 1e-5 * max(ups[k], 1e-3), (k, j[k])


def test_pruning_paths(ctx):
    from paper_2408_17118_amd import oica
    prob = synth.make_problem(synth.eeg_kinds(16), T=20_000, K=2048, seed=4)
    Xw, *_ = ica.whiten(prob.X)
    X = torch.from_numpy(Xw.astype(np.float32)).cuda()
    W0 = torch.from_numpy(prob.W0.astype(np.float32)).cuda()
    pr, *_ = _make(ctx, seed=5)
    plain = ctx.fixed_point(X, W0, tol=1e-6)
    pr.set_threshold(0.0)
    none = ctx.fixed_point(X, W0, tol=1e-6, pruner=pr)
    assert none["pruned"] == 0 and none["guard_tripped"] == 0
    for k in ("W", "kurt", "iters", "status"):
        assert torch.equal(plain[k], none[k]), k
    # both guard outcomes: every row active at pass 8 pruned (the guard, which
    # checks every accepted component and the cluster where the walk stops,
    # trips and the pruned rows finish), and a middle threshold
    # a middle threshold: the median prediction over the rows still active after pass 8
    rec = ctx.fixed_point(X, W0, tol=1e-6, traj_iters=8)
    late = rec["iters"].cpu().numpy() > 8
    prob8 = pr.predict(rec["traj"]).cpu().numpy()
    mid = float(np.median(prob8[late]))
    outcomes = set()
    for theta, gmin in ((1.0, 16), (mid, 1)):
        pr.set_threshold(theta)
        run = ctx.fixed_point(X, W0, tol=1e-6, pruner=pr, guard_min=gmin)
        assert run["pruned"] > 0
        outcomes.add(run["guard_tripped"])
        _same_unique_sets(ctx, plain, run, prob.T)
        st = run["status"].cpu().numpy()
        assert not np.any(st == ica.PRUNED) or not run["guard_tripped"]
    assert outcomes == {0, 1}
