"""GPU parity: every call goes through the C ABI (liboica.so) and is compared
with the FP64 oracle on the same seeded inputs.

Tolerances (FP32 path):
  * one update G and sum z^4/T: |gpu - oracle| <= 2e-5 + 1e-5 |oracle|
    (FP32 products and FP32 partial sums over <= ~3000 samples, FP64 across
    splits: relative error ~1e-6 of the summed magnitudes).
  * fixed points: |cos| >= 1 - 1e-6 against the oracle, kurtosis within
    1e-5 * max(|alpha|, 0.1).
"""
import ctypes as C
import math

import numpy as np
import pytest

from oracle import ica
from paper_2408_17118_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_17118_amd import oica
    c = oica.Context(0)
    yield c
    c.close()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def _mixture(N, T, K, seed):
    kinds = synth.eeg_kinds(N)
    return synth.make_problem(kinds, T=T, K=K, seed=seed)


# ---- one fused update ---------------------------------------------------------

@pytest.mark.parametrize("N,T,K", [(8, 10_000, 256), (33, 7_777, 300), (64, 20_031, 517),
                                   (100, 9_000, 129), (128, 12_345, 1), (1, 5_000, 3),
                                   (64, 100, 64)])
def test_update_matches_oracle(ctx, N, T, K):
    p = _mixture(N, T, K, seed=N + T)
    Xw, *_ = ica.whiten(p.X)
    X32 = Xw.astype(np.float32)
    B = ica.normalise_rows(p.W0).astype(np.float32)
    G, s4 = ctx.update(dev(X32), dev(B))
    Gr, s4r = ica.update(X32.astype(np.float64), B.astype(np.float64))
    G, s4 = host(G), host(s4)
    assert np.all(np.abs(G - Gr) <= 2e-5 + 1e-5 * np.abs(Gr)), np.max(np.abs(G - Gr))
    assert np.all(np.abs(s4 - s4r) <= 2e-5 + 1e-5 * np.abs(s4r))


def test_update_is_deterministic(ctx):
    p = _mixture(64, 30_000, 700, seed=3)
    Xw, *_ = ica.whiten(p.X)
    X = dev(Xw.astype(np.float32))
    B = dev(ica.normalise_rows(p.W0).astype(np.float32))
    G1, s1 = ctx.update(X, B)
    G2, s2 = ctx.update(X, B)
    assert torch.equal(G1, G2) and torch.equal(s1, s2)


# ---- kurtosis -------------------------------------------------------------------

@pytest.mark.parametrize("N,T,K", [(8, 10_000, 256), (64, 33_333, 1000), (128, 4_000, 70)])
def test_kurtosis_matches_oracle(ctx, N, T, K):
    p = _mixture(N, T, K, seed=7 * N)
    Xw, *_ = ica.whiten(p.X)
    X32 = Xw.astype(np.float32)
    B = ica.normalise_rows(p.W0).astype(np.float32)
    k = host(ctx.kurtosis(dev(X32), dev(B)))
    kr = ica.kurtosis(X32.astype(np.float64), B.astype(np.float64))
    assert np.all(np.abs(k - kr) <= 1e-5 * np.maximum(np.abs(kr), 0.1))


# ---- whitening ------------------------------------------------------------------

@pytest.mark.parametrize("N,T", [(8, 10_000), (64, 50_000), (128, 20_000), (1, 1000), (37, 999)])
def test_whiten_matches_oracle(ctx, N, T):
    p = _mixture(N, T, 1, seed=11 + N)
    X = p.X + 0.5  # non-zero means
    Xw, X32, V, mu, lam = ctx.whiten(dev(X))
    Xwr, Vr, mur, lamr = ica.whiten(X)
    assert np.allclose(host(mu), mur, rtol=1e-12, atol=1e-12)
    assert np.allclose(host(lam), lamr, rtol=1e-10)
    # V rows are eigen-directions; compare up to the canonical sign (equal by rule)
    assert np.allclose(host(V), Vr, rtol=1e-8, atol=1e-8 * np.abs(Vr).max())
    Xg = host(Xw).astype(np.float64)
    assert np.max(np.abs(Xg - Xwr)) <= 1e-6 * max(1.0, np.abs(Xwr).max())
    C = Xg @ Xg.T / T
    assert np.max(np.abs(C - np.eye(N))) < 1e-5


@pytest.mark.parametrize("N,T,f32", [(16, 2000, False), (17, 1023, True), (64, 257, False),
                                      (65, 1023, False), (80, 3001, True), (96, 1025, False),
                                      (113, 2500, False), (128, 3000, True)])
def test_whiten_kernel_class_edges(ctx, N, T, f32):
    """Row-block and kernel-class edges of the covariance and apply passes (one
    kernel for N <= 64, another above; 16-row blocks), short and ragged sample
    counts (one chunk, a partial last work item), raw FP32 and FP64 input,
    against the oracle."""
    X = _mixture(N, T, 1, seed=900 + N).X + 0.25
    Xd = dev(X.astype(np.float32)) if f32 else dev(X)
    Xw, X32, V, mu, lam = ctx.whiten(Xd)
    Xwr, Vr, mur, lamr = ica.whiten(host(Xd).astype(np.float64))
    assert np.allclose(host(mu), mur, rtol=1e-12, atol=1e-12)
    # the reference eigensolver fixes small eigenvalues to eps x the largest
    assert np.allclose(host(lam), lamr, rtol=1e-9, atol=1e-13 * lamr.max())
    assert np.allclose(host(V), Vr, rtol=1e-7, atol=1e-7 * np.abs(Vr).max())
    Xg = host(Xw).astype(np.float64)
    assert np.max(np.abs(Xg - Xwr)) <= 1e-5 * max(1.0, np.abs(Xwr).max())


def test_whiten_bf16_output(ctx):
    p = _mixture(16, 4096, 1, seed=5)
    Xw16, X32, V, mu, lam = ctx.whiten(dev(p.X), out_dtype=torch.bfloat16)
    Xwr, *_ = ica.whiten(p.X)
    assert X32 is not None and X32.dtype == torch.float32
    assert np.max(np.abs(host(X32).astype(np.float64) - Xwr)) < 1e-6 * np.abs(Xwr).max()
    # round to nearest even from the exact value: |error| <= half an ulp of bf16
    x16 = host(Xw16.float()).astype(np.float64)
    ulp = 2.0 ** (np.floor(np.log2(np.abs(Xwr))) - 7)
    assert np.all(np.abs(x16 - Xwr) <= 0.5 * ulp * (1 + 1e-9))


def test_whiten_errors(ctx):
    from paper_2408_17118_amd import oica
    rng = np.random.default_rng(0)
    S = rng.standard_normal((3, 500))
    with pytest.raises(oica.OicaError) as e:
        ctx.whiten(dev(np.vstack([S, S[:1]])))
    assert e.value.code == -3
    X = rng.standard_normal((4, 500))
    X[2, 77] = np.nan
    with pytest.raises(oica.OicaError) as e:
        ctx.whiten(dev(X))
    assert e.value.code == -4
    with pytest.raises(oica.OicaError) as e:
        ctx.whiten(dev(rng.standard_normal((4, 4))))
    assert e.value.code == -1
    with pytest.raises(oica.OicaError) as e:
        ctx.whiten(dev(rng.standard_normal((129, 500))))
    assert e.value.code == -7


def test_binding_rejects_wrong_dtypes_and_shapes(ctx):
    """The C ABI takes plain pointers, so the binding checks every tensor's dtype
    and shape before a call: a BF16 tensor where the FP32 copy belongs, or a row
    block of the wrong width, raise on the host and no kernel runs."""
    import torch
    N, T, K = 8, 1000, 16
    Xb = torch.zeros((N, T), dtype=torch.bfloat16, device="cuda")
    X32 = torch.zeros((N, T), dtype=torch.float32, device="cuda")
    W0 = torch.ones((K, N), dtype=torch.float32, device="cuda")
    with pytest.raises(TypeError):
        ctx.fixed_point(Xb, W0, precision="bf16")              # Xw_f32 defaults to Xw
    with pytest.raises(TypeError):
        ctx.fixed_point(Xb, W0, Xw_f32=Xb, precision="bf16")
    with pytest.raises(TypeError):
        ctx.fixed_point(X32, W0, precision="bf16")             # data type of the precision
    with pytest.raises(ValueError):
        ctx.fixed_point(X32, W0[:, :4].contiguous())
    with pytest.raises(ValueError):
        ctx.fixed_point(Xb, W0, Xw_f32=X32[:, :500].contiguous(), precision="bf16")
    with pytest.raises(TypeError):
        ctx.fixed_point_batched([{"Xw": Xb, "Xw_f32": Xb, "W0": W0}], precision="bf16")
    with pytest.raises(TypeError):
        ctx.kurtosis(Xb, W0)
    with pytest.raises(TypeError):
        ctx.unique(W0, torch.zeros(K, dtype=torch.float32, device="cuda"),
                   torch.zeros(K, dtype=torch.uint8, device="cuda"), T)
    with pytest.raises(TypeError):
        ctx.whiten(torch.zeros((N, T), dtype=torch.float16, device="cuda"))


def test_whiten_batched_equals_single(ctx):
    """One batched call gives every dataset exactly the single call's outputs
    (same kernels; the eigen-solve, canon and apply of the N <= 64 problems run
    on a second stream beside the others')."""
    shapes = [(1, 1000), (2, 3000), (7, 5001), (33, 4000), (64, 20_000), (100, 9000), (128, 12_000)]
    Xs = []
    for i, (N, T) in enumerate(shapes):
        X = _mixture(N, T, 1, seed=300 + i).X + 0.25
        Xs.append(dev(X) if i % 3 else dev(X.astype(np.float32)))
    for out_dtype in (torch.float32, torch.bfloat16):
        outs = ctx.whiten_batched(Xs, out_dtype=out_dtype)
        for X, o in zip(Xs, outs):
            ref = ctx.whiten(X, out_dtype=out_dtype)
            for a, b in zip(o, ref):
                assert torch.equal(a, b)
    # and against the oracle for the largest
    Vr = ica.whiten(host(Xs[-1]).astype(np.float64))[1]
    V = host(outs[-1][2])
    assert np.allclose(V, Vr, rtol=1e-8, atol=1e-8 * np.abs(Vr).max())


@pytest.mark.parametrize("shapes", [[(5, 3000), (48, 7001), (64, 9000)],
                                    [(65, 4001), (96, 6000), (128, 8000)]])
def test_whiten_batched_one_size_class(ctx, shapes):
    """A batch whose problems all fall in one size class (N <= 64, or N > 64)
    runs on the call's stream alone; every output still equals the single
    call's bit for bit, as with the mixed batch above (whose two classes finish
    on two streams)."""
    Xs = [dev(_mixture(N, T, 1, seed=700 + i).X) for i, (N, T) in enumerate(shapes)]
    for out_dtype in (torch.float32, torch.bfloat16):
        outs = ctx.whiten_batched(Xs, out_dtype=out_dtype)
        for X, o in zip(Xs, outs):
            for a, b in zip(o, ctx.whiten(X, out_dtype=out_dtype)):
                assert torch.equal(a, b)


def test_whiten_reads_a_window_in_place(ctx):
    """X_raw with a row stride ld_raw > T (a window of a longer recording): the
    outputs equal those of the contiguous copy bit for bit, single and batched,
    and samples outside the window (here NaN) are never read."""
    from paper_2408_17118_amd import oica
    L = 12_000
    # N > 64 takes the tiled covariance and apply, whose vector loads then start at
    # addresses aligned to 4 bytes only (FP32 window at offset 333)
    cases = [(9, 5000, 700, np.float64), (64, 7001, 1234, np.float32), (1, 999, 3, np.float64),
             (100, 5003, 333, np.float32), (128, 4001, 77, np.float64)]
    wins, refs = [], []
    for i, (N, T, a, dt) in enumerate(cases):
        rec = _mixture(N, L, 1, seed=700 + i).X.astype(dt) + 0.5
        rec[:, :a] = np.nan
        rec[:, a + T:] = np.nan
        R = dev(rec)
        W = R[:, a:a + T]
        assert W.stride(0) == L and (N == 1 or not W.is_contiguous())
        wins.append(W)
        refs.append(W.contiguous())
    for out_dtype in (torch.float32, torch.bfloat16):
        for W, Wc in zip(wins, refs):
            for x, y in zip(ctx.whiten(W, out_dtype=out_dtype), ctx.whiten(Wc, out_dtype=out_dtype)):
                assert torch.equal(x, y)
        for o, Wc in zip(ctx.whiten_batched(wins, out_dtype=out_dtype), refs):
            for x, y in zip(o, ctx.whiten(Wc, out_dtype=out_dtype)):
                assert torch.equal(x, y)
    Vr = ica.whiten(host(refs[0]))[1]
    assert np.allclose(host(ctx.whiten(wins[0])[2]), Vr, rtol=1e-8, atol=1e-8 * np.abs(Vr).max())
    # a stride shorter than a row is refused on the host; so is a column-strided view
    lib, N, T = ctx.lib, 9, 5000
    Xw = torch.empty((N, T), dtype=torch.float32, device="cuda")
    rc = lib.oica_whiten(ctx.h, N, T, C.c_void_p(refs[0].data_ptr()), oica.OICA_F64, T - 1,
                         C.c_void_p(Xw.data_ptr()), oica.OICA_F32, None, None, None, None)
    assert rc == -2
    with pytest.raises(ValueError):
        ctx.whiten(dev(np.ones((T, N))).t())


def test_whiten_batched_status(ctx):
    rng = np.random.default_rng(1)
    S = rng.standard_normal((3, 500))
    bad = rng.standard_normal((4, 500))
    bad[1, 10] = np.inf
    Xs = [dev(rng.standard_normal((5, 600))), dev(np.vstack([S, S[:1]])), dev(bad),
          dev(rng.standard_normal((6, 700)))]
    outs, st = ctx.whiten_batched(Xs, return_status=True)
    assert st == [0, -3, -4, 0]
    for i in (0, 3):
        ref = ctx.whiten(Xs[i])
        assert torch.equal(outs[i][0], ref[0])
    from paper_2408_17118_amd import oica
    with pytest.raises(oica.OicaError) as e:
        ctx.whiten_batched(Xs)
    assert e.value.code == -3


# ---- the fixed point --------------------------------------------------------------

def _rowwise_abs_cos(A, B):
    A = A / np.linalg.norm(A, axis=1, keepdims=True)
    B = B / np.linalg.norm(B, axis=1, keepdims=True)
    return np.abs(np.einsum("kn,kn->k", A, B))


@pytest.mark.parametrize("N,T,K,seed", [(8, 10_000, 256, 0), (24, 20_000, 700, 1),
                                        (64, 30_000, 1024, 2), (128, 30_011, 200, 3),
                                        (90, 15_000, 333, 4)])
def test_fixed_point_matches_oracle(ctx, N, T, K, seed):
    """Per-row agreement with the oracle from the same starts.  The cases cover
    every padded width (32 ... 128), ragged T, and runs that start on the thin
    items (K <= 256) or switch to them as rows converge."""
    if N == 8:
        p = synth.small_mixture()
    else:
        p = _mixture(N, T, K, seed)
    Xw, *_ = ica.whiten(p.X)
    X32 = Xw.astype(np.float32)
    res = ctx.fixed_point(dev(X32), dev(p.W0.astype(np.float32)), tol=1e-6, max_iter=1000)
    Br, itr, str_, _, tir = ica.fixed_point(X32.astype(np.float64), p.W0, tol=1e-6, max_iter=1000)
    W, st, it = host(res["W"]), host(res["status"]), host(res["iters"])
    assert np.allclose(np.linalg.norm(W, axis=1), 1.0, atol=1e-6)
    cos = _rowwise_abs_cos(W.astype(np.float64), Br)
    same = cos >= 1 - 1e-6
    # per-row basin agreement (FP32 vs FP64 trajectories from the same start)
    assert same.mean() >= 0.99, same.mean()
    agree_it = (it == itr)[same & (st == ica.CONV) & (str_ == ica.CONV)]
    assert agree_it.mean() >= 0.9
    assert (st == ica.CONV).mean() >= (str_ == ica.CONV).mean() - 0.01
    kr = ica.kurtosis(X32.astype(np.float64), W.astype(np.float64))
    k = host(res["kurt"])
    assert np.all(np.abs(k - kr) <= 1e-5 * np.maximum(np.abs(kr), 0.1))
    assert res["thread_iters"] == int(it.sum())


def test_fixed_point_edge_cases(ctx):
    p = synth.small_mixture()
    Xw, *_ = ica.whiten(p.X)
    X = dev(Xw.astype(np.float32))
    W0 = p.W0[:5].astype(np.float32).copy()
    W0[2] = 0.0                                     # zero start row -> DEGENERATE
    res = ctx.fixed_point(X, dev(W0), tol=1e-6, max_iter=1)
    st, it = host(res["status"]), host(res["iters"])
    assert st[2] == ica.DEGENERATE and it[2] == 0
    assert all(it[i] == 1 for i in (0, 1, 3, 4))    # do-while: exactly one pass
    assert all(st[i] == ica.NOTCONV for i in (0, 1, 3, 4))
    # single row, many passes
    res = ctx.fixed_point(X, dev(p.W0[:1].astype(np.float32)), tol=1e-6, max_iter=1000)
    assert host(res["status"])[0] == ica.CONV
    # one-dimensional data: every row converges after one update
    x = np.random.default_rng(1).laplace(size=(1, 3000))
    Xw1, *_ = ica.whiten(x)
    res = ctx.fixed_point(dev(Xw1.astype(np.float32)), dev(np.array([[0.5], [-3.0]], np.float32)),
                          tol=1e-6, max_iter=10)
    assert np.all(host(res["status"]) == ica.CONV) and np.all(host(res["iters"]) == 1)


def test_fixed_point_trajectory(ctx):
    """traj[l, t] = (kurtosis of the row before pass t+1, step of pass t+1).

    Checked two ways.  Step by step, on every row and every recorded pass: the
    GPU's iterates after t passes (runs capped at t passes) give the oracle's
    kurtosis of the row the pass started from and the step to the next iterate,
    and the next iterate is the oracle's normalised update of the previous one.
    Whole trajectories, on every row: the oracle's own run, within what the
    measured distance between the two sides' iterates allows (a wandering
    start amplifies FP32 and FP64 rounding from pass to pass).
    """
    p = synth.small_mixture()
    Xw, *_ = ica.whiten(p.X)
    X32 = Xw.astype(np.float32)
    X64 = X32.astype(np.float64)
    tol, R = 1e-6, 8
    W0d = dev(p.W0.astype(np.float32))
    res = ctx.fixed_point(dev(X32), W0d, tol=tol, max_iter=1000, traj_iters=R)
    tr = host(res["traj"]).astype(np.float64)
    it = host(res["iters"])
    _, itr, _, trr, _ = ica.fixed_point(X64, p.W0, tol=tol, max_iter=1000, traj_iters=R)
    B0 = ica.normalise_rows(p.W0.astype(np.float32).astype(np.float64))
    Wg = [B0] + [host(ctx.fixed_point(dev(X32), W0d, tol=tol, max_iter=t)["W"]).astype(np.float64)
                 for t in range(1, R + 1)]
    Wo = [B0] + [ica.fixed_point(X64, p.W0, tol=tol, max_iter=t)[0] for t in range(1, R + 1)]
    K = tr.shape[0]
    # Tolerances (reading of the recorded trajectory): the kurtosis entry is
    # sum z^4 / T - 3 with the fourth-power sum accumulated in FP32 per split,
    # so its error scales with alpha + 3 (the quantity summed); the step is
    # formed in FP64 from the FP32 row and the new row before it is rounded.
    for t in range(R):
        live = it > t                                   # rows updated in pass t+1
        assert np.array_equal(np.isfinite(tr[:, t, 0]), live), t
        a_ref = ica.kurtosis(X64, Wg[t][live])
        assert np.all(np.abs(tr[live, t, 0] - a_ref) <= 1e-5 * (np.abs(a_ref) + 3.0)), t
        d_ref = np.minimum(np.linalg.norm(Wg[t + 1][live] - Wg[t][live], axis=1),
                           np.linalg.norm(Wg[t + 1][live] + Wg[t][live], axis=1))
        assert np.all(np.abs(tr[live, t, 1] - d_ref) <= 1e-6), t
        G, _ = ica.update(X64, Wg[t][live])
        Bn = G / np.linalg.norm(G, axis=1, keepdims=True)
        assert np.all(_rowwise_abs_cos(Wg[t + 1][live], Bn) >= 1 - 1e-10), t
    # every row starts from the same vector: the first recorded kurtosis agrees
    assert np.all(np.abs(tr[:, 0, 0] - trr[:, 0, 0]) <= 1e-5 * (np.abs(trr[:, 0, 0]) + 3.0))
    # Whole trajectories against the oracle's own run, every row: the entries
    # may differ by what the measured distance e_t between the GPU's and the
    # oracle's iterates allows -- steps by e_t + e_{t+1} (triangle inequality),
    # kurtosis by 4 ||E[y^3 x]|| e_t (its gradient) -- plus the FP32 terms
    # above.  Rows whose iterates stay together are held to the FP32 terms;
    # a wandering start amplifies rounding from pass to pass and is held to
    # the distance its iterates actually drift apart by.
    e = [np.minimum(np.linalg.norm(Wg[t] - Wo[t], axis=1), np.linalg.norm(Wg[t] + Wo[t], axis=1))
         for t in range(R + 1)]
    close = 0
    for t in range(R):
        both = np.isfinite(tr[:, t, 0]) & np.isfinite(trr[:, t, 0])
        G, _ = ica.update(X64, Wo[t][both])
        lip = 4.0 * np.linalg.norm(G + 3.0 * Wo[t][both], axis=1)
        a, ar = tr[both, t, 0], trr[both, t, 0]
        assert np.all(np.abs(a - ar) <= 1.1 * lip * e[t][both] + 1e-5 * (np.abs(ar) + 3.0)), t
        d, dr = tr[both, t, 1], trr[both, t, 1]
        assert np.all(np.abs(d - dr) <= e[t][both] + e[t + 1][both] + 1e-6), t
        close += int(np.sum(e[t + 1][both] <= 1e-6))
    assert close >= 0.9 * int(np.sum(np.isfinite(trr[:, :, 0])))
    # where the two sides stop a pass apart, the oracle's step at the earlier
    # stop lies within the FP32 noise of the threshold
    for l in np.flatnonzero(it != itr):
        assert abs(int(it[l]) - int(itr[l])) == 1, l
        last = min(int(it[l]), int(itr[l])) - 1
        if last < R:
            assert abs(trr[l, last, 1] - tol) <= 2e-6 + e[last][l] + e[last + 1][l], l


def test_fixed_point_is_deterministic(ctx):
    p = _mixture(64, 20_000, 2048, seed=9)
    Xw, *_ = ica.whiten(p.X)
    X = dev(Xw.astype(np.float32))
    W0 = dev(p.W0.astype(np.float32))
    r1 = ctx.fixed_point(X, W0, tol=1e-6, max_iter=1000)
    r2 = ctx.fixed_point(X, W0, tol=1e-6, max_iter=1000)
    for k in ("W", "kurt", "iters", "status"):
        assert torch.equal(r1[k], r2[k]), k


# ---- unique ---------------------------------------------------------------------------

def _planted(seed=5, N=12, n_clusters=6, per=7, noise=1e-6):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    rows, labels = [], []
    for c in range(n_clusters):
        for _ in range(per):
            v = Q[c] + noise * rng.standard_normal(N)
            rows.append(v / np.linalg.norm(v) * rng.choice([-1.0, 1.0]))
            labels.append(c)
    perm = rng.permutation(len(rows))
    return np.array(rows)[perm], np.array(labels)[perm]


def test_unique_planted_matches_oracle(ctx):
    B, labels = _planted(N=12, n_clusters=9, per=40)
    K = len(labels)
    rng = np.random.default_rng(3)
    alpha = 5.0 - 0.5 * labels + 1e-6 * rng.standard_normal(K)
    status = np.full(K, ica.CONV, np.uint8)
    status[rng.choice(K, 20, replace=False)] = ica.NOTCONV
    B32 = B.astype(np.float32)
    for gtest, T in ((False, 1000), (True, 30)):
        ref = ica.unique(B32.astype(np.float64), alpha, status, T, tau=1e-3, gaussianity_test=gtest)
        res = ctx.unique(dev(B32), dev(alpha), dev(status), T, tau=1e-3, gaussianity_test=gtest)
        assert res["n_unique"] == len(ref["U"])
        assert res["n_accepted"] == ref["n_accepted"]
        assert np.array_equal(host(res["rep"]), ref["rep"])
        assert np.array_equal(host(res["size"]), ref["size"])
        assert np.array_equal(host(res["U"]), ref["U"])
        assert np.array_equal(host(res["upsilon"]), ref["upsilon"]) or \
            np.allclose(host(res["upsilon"]), ref["upsilon"], rtol=1e-15)


def test_unique_fallback_and_cap(ctx):
    from paper_2408_17118_amd import oica
    B, labels = _planted(seed=1, N=6, n_clusters=3, per=5)
    K = len(labels)
    status = np.full(K, ica.NOTCONV, np.uint8)    # nothing converged: all rows used
    status[0] = ica.DEGENERATE
    alpha = np.linspace(4, 1, K)
    ref = ica.unique(B, alpha, status, 500, gaussianity_test=False)
    res = ctx.unique(dev(B.astype(np.float32)), dev(alpha), dev(status), 500, gaussianity_test=False)
    assert res["n_unique"] == len(ref["U"]) and np.array_equal(host(res["rep"]), ref["rep"])
    with pytest.raises(oica.OicaError) as e:
        ctx.unique(dev(B.astype(np.float32)), dev(alpha), dev(status), 500, cap=1)
    assert e.value.code == -2
    res = ctx.unique(dev(B.astype(np.float32)), dev(alpha), dev(status), 500, n_top=1,
                     gaussianity_test=False)
    assert res["n_accepted"] == 1


@pytest.mark.parametrize("N,per", [(32, 1000), (24, 3300)])
def test_unique_large_problems(ctx, N, per):
    """K = 20000 (all rounds in one launch over many work-groups) and K = 66000
    (more work-groups than fit at once: round by round), against the oracle."""
    B, labels = _planted(seed=7, N=N, n_clusters=20, per=per)
    K = len(labels)
    rng = np.random.default_rng(4)
    alpha = 6.0 - 0.25 * labels + 1e-6 * rng.standard_normal(K)
    status = np.full(K, ica.CONV, np.uint8)
    B32 = B.astype(np.float32)
    ref = ica.unique(B32.astype(np.float64), alpha, status, 5000, tau=1e-3, gaussianity_test=True)
    res = ctx.unique(dev(B32), dev(alpha), dev(status), 5000, tau=1e-3)
    assert res["n_unique"] == len(ref["U"]) == 20
    assert res["n_accepted"] == ref["n_accepted"]
    assert np.array_equal(host(res["rep"]), ref["rep"])
    assert np.array_equal(host(res["size"]), ref["size"])
    assert np.array_equal(host(res["U"]), ref["U"])


def test_unique_batched_equals_single(ctx):
    """One batched call gives every problem exactly the single call's result
    (small problems in the one-work-group kernel, the large one round by round)."""
    items = []
    for i, (N, nc, per) in enumerate([(12, 9, 40), (6, 3, 5), (32, 20, 1000), (64, 30, 30),
                                      (128, 10, 100)]):
        B, labels = _planted(seed=20 + i, N=N, n_clusters=nc, per=per)
        K = len(labels)
        rng = np.random.default_rng(i)
        alpha = 5.0 - 0.1 * labels + 1e-6 * rng.standard_normal(K)
        status = np.full(K, ica.CONV, np.uint8)
        status[rng.choice(K, K // 10, replace=False)] = ica.NOTCONV
        if i == 1:
            status[:] = ica.NOTCONV   # nothing converged: every row is a candidate
        items.append((dev(B.astype(np.float32)), dev(alpha), dev(status), 40 * N))
    for gtest in (True, False):
        outs = ctx.unique_batched(items, gaussianity_test=gtest, row_cluster=True)
        for it, o in zip(items, outs):
            ref = ctx.unique(*it, gaussianity_test=gtest, row_cluster=True)
            assert o["n_unique"] == ref["n_unique"] and o["n_accepted"] == ref["n_accepted"]
            for k in ("U", "alpha", "upsilon", "rep", "size", "row_cluster"):
                assert torch.equal(o[k], ref[k]), k


# ---- end to end on raw data ------------------------------------------------------------

def _compare_unique(res, ref, V_gpu, tie_rel=1e-5):
    n = ref["n_accepted"]
    assert res["n_accepted"] == n, (res["n_accepted"], n)
    U = host(res["U"])[:n] @ V_gpu
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    Ur = ref["U_raw"][:n]
    a, ar = host(res["alpha"])[:n], ref["alpha"][:n]
    ups_r = ref["upsilon"][:n]
    # order: identical except inside groups of near-equal upsilon (compared as sets)
    cos = np.abs(U @ Ur.T)
    match = np.argmax(cos, axis=1)
    assert np.all(cos[np.arange(n), match] >= 1 - 1e-6), np.min(cos[np.arange(n), match])
    assert len(set(match)) == n
    for r in range(n):
        j = match[r]
        if j != r:
            assert abs(ups_r[j] - ups_r[r]) <= tie_rel * max(ups_r[r], 1e-3), (r, j)
        assert abs(a[r] - ar[j]) <= 1e-5 * max(abs(ar[j]), 0.1)


def test_end_to_end_small_mixture(ctx):
    from paper_2408_17118_amd import oica
    p = synth.small_mixture()
    res = oica.ordering_ica(ctx, dev(p.X), dev(p.W0.astype(np.float32)), tol=1e-6)
    ref = ica.ordering_ica(p.X, p.W0, tol=1e-10, max_iter=1000)
    assert res["n_unique"] == len(ref["U"])
    _compare_unique(res, ref, host(res["V"]))
    assert list(host(res["size"])) == list(ref["size"]) or \
        abs(int(host(res["size"]).sum()) - int(ref["size"].sum())) <= 2
